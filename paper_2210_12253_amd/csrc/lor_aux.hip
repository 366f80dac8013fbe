// Auxiliary LOR data for the auxiliary-space solvers (Section 3, Step S1.2,
// auxiliary computations): the discrete gradient and curl matrices, the interpolation of
// the high-order mesh nodes to the LOR (Gauss-Lobatto) lattice as an E-vector,
// and the E-vector to T-vector deduplication of those coordinates.
//
// Every per-dof kernel takes the dof's data from its first incidence (lowest
// element, then lowest local index), read from the sorted incidence lists of
// the lor_pattern schedule (for faces, which have no schedule, from an
// atomic-minimum pass over the face map): one thread per dof, as the paper
// threads them.
#include <algorithm>
#include <cmath>

#include "lor_common.hpp"

namespace lor {

int check_sched(const lor_sched* s, int space, int p, int64_t nel, int64_t nrows);

constexpr int kAuxThreads = 256;
constexpr int kMaxNodeOrder = 8;  // highest degree q of the high-order mesh nodes

// ------------------------------------------------------- discrete gradient

// Local endpoints (v0 -> v1, along the +axis) of local edge l of a degree-p
// macro element: x-edges i + p(j + (p+1)k), then y-edges, then z-edges.
__device__ __forceinline__ void local_edge_vertices(int p, int l, int& v0, int& v1) {
  const int q = p + 1;
  const int nx = p * q * q;
  if (l < nx) {
    const int i = l % p, j = (l / p) % q, k = l / (p * q);
    v0 = i + q * (j + q * k);
    v1 = v0 + 1;
  } else if (l < 2 * nx) {
    const int m = l - nx;
    const int i = m % q, j = (m / q) % p, k = m / (q * p);
    v0 = i + q * (j + q * k);
    v1 = v0 + q;
  } else {
    const int m = l - 2 * nx;
    const int i = m % q, j = (m / q) % q, k = m / (q * q);
    v0 = i + q * (j + q * k);
    v1 = v0 + q * q;
  }
}

// G maps vertex values (the H1 space) to edge values (the lowest-order
// Nedelec space) of the LOR mesh: the edge dof of edge e is the integral of
// grad u along e in the edge's global orientation.  For the piecewise
// trilinear u that integral is the difference of the vertex values at the
// edge's ends, so with lo -> hi the edge's direction in an element holding it
// (the local +axis) and sigma = +1 when the global orientation agrees with it,
// -1 when it is the reverse,
//   (G u)_e = sigma (u_hi - u_lo).
// Row e therefore holds two entries, -sigma in column lo and +sigma in column
// hi.  The element taken is the edge's first incidence, and the entries are
// kept in the element's (lo, hi) order, not sorted.
template <typename T>
__global__ __launch_bounds__(kAuxThreads) void k_discrete_gradient(
    int p, int64_t nedges, int64_t ndofs_h1, const int32_t* __restrict__ elem_dofs,
    const int32_t* __restrict__ elem_edges, const int32_t* __restrict__ inc_ptr, const int32_t* __restrict__ inc_list,
    int32_t* __restrict__ row_ptr, int32_t* __restrict__ col_idx, T* __restrict__ values, int32_t* __restrict__ diag) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= nedges) return;
  const int q = p + 1;
  const int nloce = 3 * p * q * q, nlocv = q * q * q;
  // every row has two entries
  row_ptr[e] = static_cast<int32_t>(2 * e);
  if (e == nedges - 1) row_ptr[nedges] = static_cast<int32_t>(2 * nedges);
  int32_t lo = 0, hi = 0;
  T sigma = T(0);  // an edge in no element keeps a zero row (counted in diag[0])
  if (inc_ptr[e] < inc_ptr[e + 1]) {
    const int32_t first = inc_list[inc_ptr[e]];  // element * nloce + local edge
    const int32_t el = first / nloce;
    int v_lo, v_hi;
    local_edge_vertices(p, first - el * nloce, v_lo, v_hi);
    const int32_t* ev = elem_dofs + static_cast<int64_t>(el) * nlocv;
    lo = ev[v_lo];
    hi = ev[v_hi];
    sigma = elem_edges[first] < 0 ? T(-1) : T(1);
    if ((lo < 0 || lo >= ndofs_h1 || hi < 0 || hi >= ndofs_h1) && diag) atomicAdd(&diag[1], 1);
  } else if (diag) {
    atomicAdd(&diag[0], 1);
  }
  col_idx[2 * e] = lo;
  values[2 * e] = -sigma;
  col_idx[2 * e + 1] = hi;
  values[2 * e + 1] = sigma;
}

// ------------------------------------------------------- discrete curl

__global__ __launch_bounds__(kAuxThreads) void k_fill_owner(int32_t* __restrict__ owner, int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) owner[i] = INT32_MAX;
}

// owner[f] = lowest flat index e * nlocf + lf of the faces map that names f
__global__ __launch_bounds__(kAuxThreads) void k_face_owner(const int32_t* __restrict__ elem_faces, int64_t total,
                                                            int64_t nfaces, int32_t* __restrict__ owner,
                                                            int32_t* __restrict__ diag) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int32_t raw = elem_faces[i];
  const int32_t f = raw < 0 ? -1 - raw : raw;
  if (f >= nfaces) {
    if (diag) atomicAdd(&diag[1], 1);
    return;
  }
  atomicMin(&owner[f], static_cast<int32_t>(i));
}

// The 4 boundary edges of local face lf of a degree-p macro element and their
// signs in the face's circulation (right-hand rule about the +axis normal):
// x-face boundary +y, +z, -y, -z; y-face +z, +x, -z, -x; z-face +x, +y, -x, -y.
__device__ __forceinline__ void local_face_edges(int p, int lf, int (&le)[4]) {
  const int q = p + 1;
  const int nfx = p * p * q, nex = p * q * q;
  auto xe = [&](int i, int j, int k) { return i + p * (j + q * k); };
  auto ye = [&](int i, int j, int k) { return nex + i + q * (j + p * k); };
  auto ze = [&](int i, int j, int k) { return 2 * nex + i + q * (j + q * k); };
  if (lf < nfx) {
    const int i = lf % q, j = (lf / q) % p, k = lf / (q * p);
    le[0] = ye(i, j, k);
    le[1] = ze(i, j + 1, k);
    le[2] = ye(i, j, k + 1);
    le[3] = ze(i, j, k);
  } else if (lf < 2 * nfx) {
    const int m = lf - nfx;
    const int i = m % p, j = (m / p) % q, k = m / (p * q);
    le[0] = ze(i, j, k);
    le[1] = xe(i, j, k + 1);
    le[2] = ze(i + 1, j, k);
    le[3] = xe(i, j, k);
  } else {
    const int m = lf - 2 * nfx;
    const int i = m % p, j = (m / p) % p, k = m / (p * p);
    le[0] = xe(i, j, k);
    le[1] = ye(i + 1, j, k);
    le[2] = xe(i, j + 1, k);
    le[3] = ye(i, j, k);
  }
}

template <typename T>
__global__ __launch_bounds__(kAuxThreads) void k_discrete_curl(
    int p, int64_t nfaces, int64_t nedges, const int32_t* __restrict__ elem_edges,
    const int32_t* __restrict__ elem_faces, const int32_t* __restrict__ owner, int32_t* __restrict__ row_ptr,
    int32_t* __restrict__ col_idx, T* __restrict__ values, int32_t* __restrict__ diag) {
  const int64_t f = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (f >= nfaces) return;
  const int q = p + 1;
  const int nlocf = 3 * p * p * q, nloce = 3 * p * q * q;
  row_ptr[f] = static_cast<int32_t>(4 * f);
  if (f == nfaces - 1) row_ptr[nfaces] = static_cast<int32_t>(4 * nfaces);
  const int32_t inc = owner[f];
  int32_t cols[4] = {0, 0, 0, 0};
  T vals[4] = {T(0), T(0), T(0), T(0)};
  if (inc != INT32_MAX) {
    const int32_t e = inc / nlocf;
    const int lf = inc - e * nlocf;
    const T sf = elem_faces[inc] < 0 ? T(-1) : T(1);
    int le[4];
    local_face_edges(p, lf, le);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int32_t raw = elem_edges[static_cast<int64_t>(e) * nloce + le[s]];
      const int32_t g = raw < 0 ? -1 - raw : raw;
      if (g >= nedges && diag) atomicAdd(&diag[1], 1);
      cols[s] = g;
      const T se = raw < 0 ? T(-1) : T(1);
      vals[s] = (s < 2 ? sf : -sf) * se;
    }
  } else if (diag) {
    atomicAdd(&diag[0], 1);  // face in no element: its row is left as four zeros at column 0
  }
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    col_idx[4 * f + s] = cols[s];
    values[4 * f + s] = vals[s];
  }
}

// ------------------------------------------- node interpolation (E-vector)

// 1D Lagrange basis of the degree-q Gauss-Lobatto nodes evaluated at the
// degree-p Gauss-Lobatto nodes, on [0, 1]: b[i * (q+1) + j] = l_j(x_i).
struct InterpBasis {
  double b[(LOR_MAX_P + 1) * (kMaxNodeOrder + 1)];
};

// Gauss-Lobatto nodes of degree n on [0, 1], ascending: the end points and
// the roots of P_n', found by Newton's method on P_n' from the
// Chebyshev-Gauss-Lobatto points (the Legendre recurrence gives P_n' and P_n'').
static void gll_nodes(int n, double* x) {
  x[0] = 0.0;
  x[n] = 1.0;
  for (int k = 1; k < n; ++k) {
    double t = -std::cos(3.14159265358979323846 * k / n);
    for (int it = 0; it < 100; ++it) {
      // P_0..P_n at t and the derivative of P_n
      double p0 = 1.0, p1 = t;
      for (int m = 2; m <= n; ++m) {
        const double p2 = ((2 * m - 1) * t * p1 - (m - 1) * p0) / m;
        p0 = p1;
        p1 = p2;
      }
      // P_n' = n (P_{n-1} - t P_n) / (1 - t^2);  (1 - t^2) P_n'' = 2 t P_n' - n (n+1) P_n
      const double dp = n * (p0 - t * p1) / (1.0 - t * t);
      const double d2p = (2.0 * t * dp - n * (n + 1.0) * p1) / (1.0 - t * t);
      const double dt = dp / d2p;
      t -= dt;
      if (std::fabs(dt) < 1e-16) break;
    }
    x[k] = 0.5 * (t + 1.0);
  }
}

static InterpBasis interp_basis(int p, int q) {
  InterpBasis B{};
  double xp[LOR_MAX_P + 1], xq[kMaxNodeOrder + 1];
  gll_nodes(p, xp);
  gll_nodes(q, xq);
  for (int i = 0; i <= p; ++i)
    for (int j = 0; j <= q; ++j) {
      double v = 1.0;
      for (int m = 0; m <= q; ++m)
        if (m != j) v *= (xp[i] - xq[m]) / (xq[j] - xq[m]);
      B.b[i * (q + 1) + j] = v;
    }
  return B;
}

// LDS doubles of k_interp_nodes: nodes, the two partial contractions, basis.
static int interp_lds_doubles(int p, int q, int ncomp) {
  const int P1 = p + 1, Q1 = q + 1;
  return (Q1 * Q1 * Q1 + P1 * Q1 * Q1 + P1 * P1 * Q1) * ncomp + P1 * Q1;
}

// One workgroup per element: nodes -> LDS, then the three 1D contractions
// (x, y, z) of the tensor-product basis, the last one written straight to the
// element's contiguous E-vector block.  LDS is sized for the actual (p, q),
// so small degrees keep many workgroups resident per CU.
// Templated on the lattice size P1 = p + 1 and the component count NC so
// that the index arithmetic divides by constants.
template <int P1, int NC>
__global__ __launch_bounds__(kAuxThreads) void k_interp_nodes(int q, const double* __restrict__ nodes,
                                                              double* __restrict__ out, InterpBasis B) {
  extern __shared__ double lds[];
  constexpr int ncomp = NC;
  const int Q1 = q + 1;
  double* s0 = lds;
  double* s1 = s0 + Q1 * Q1 * Q1 * ncomp;
  double* s2 = s1 + P1 * Q1 * Q1 * ncomp;
  double* sB = s2 + P1 * P1 * Q1 * ncomp;
  const int64_t e = blockIdx.x;
  const int tid = threadIdx.x;
  const int nin = Q1 * Q1 * Q1 * ncomp;
  const double* src = nodes + e * nin;
  for (int t = tid; t < nin; t += kAuxThreads) s0[t] = src[t];
  for (int t = tid; t < P1 * Q1; t += kAuxThreads) sB[t] = B.b[t];
  __syncthreads();
  // x: s1[k][j][i'][c] = sum_i B[i'][i] s0[k][j][i][c]
  for (int t = tid; t < P1 * Q1 * Q1 * ncomp; t += kAuxThreads) {
    const int c = t % ncomp, r = t / ncomp;
    const int ip = r % P1, j = (r / P1) % Q1, k = r / (P1 * Q1);
    double acc = 0.0;
    for (int i = 0; i < Q1; ++i) acc += sB[ip * Q1 + i] * s0[((k * Q1 + j) * Q1 + i) * ncomp + c];
    s1[t] = acc;
  }
  __syncthreads();
  // y: s2[k][j'][i'][c] = sum_j B[j'][j] s1[k][j][i'][c]
  for (int t = tid; t < P1 * P1 * Q1 * ncomp; t += kAuxThreads) {
    const int c = t % ncomp, r = t / ncomp;
    const int ip = r % P1, jp = (r / P1) % P1, k = r / (P1 * P1);
    double acc = 0.0;
    for (int j = 0; j < Q1; ++j) acc += sB[jp * Q1 + j] * s1[((k * Q1 + j) * P1 + ip) * ncomp + c];
    s2[t] = acc;
  }
  __syncthreads();
  // z: out[k'][j'][i'][c] = sum_k B[k'][k] s2[k][j'][i'][c]
  double* dst = out + e * (P1 * P1 * P1 * ncomp);
  for (int t = tid; t < P1 * P1 * P1 * ncomp; t += kAuxThreads) {
    const int c = t % ncomp, r = t / ncomp;
    const int ip = r % P1, jp = (r / P1) % P1, kp = r / (P1 * P1);
    double acc = 0.0;
    for (int k = 0; k < Q1; ++k) acc += sB[kp * Q1 + k] * s2[((k * P1 + jp) * P1 + ip) * ncomp + c];
    dst[t] = acc;
  }
}

// ------------------------------------------------ E-vector -> T-vector

__global__ __launch_bounds__(kAuxThreads) void k_evec_to_tvec(int64_t ndofs, int ncomp,
                                                              const int32_t* __restrict__ inc_ptr,
                                                              const int32_t* __restrict__ inc_list,
                                                              const double* __restrict__ evec,
                                                              double* __restrict__ tvec, int32_t* __restrict__ diag) {
  const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (g >= ndofs) return;
  const int32_t a = inc_ptr[g], b = inc_ptr[g + 1];
  if (a >= b) {
    if (diag) atomicAdd(&diag[0], 1);  // dof in no element: left as 0
    for (int c = 0; c < ncomp; ++c) tvec[g * ncomp + c] = 0.0;
    return;
  }
  const int64_t inc = inc_list[a];
  for (int c = 0; c < ncomp; ++c) tvec[g * ncomp + c] = evec[inc * ncomp + c];
}

}  // namespace lor

using namespace lor;

extern "C" int lor_discrete_gradient(int p, int64_t nel, int64_t ndofs_h1, int64_t nedges, const int32_t* elem_dofs,
                                     const int32_t* elem_edges, const lor_sched* sched, int32_t* row_ptr,
                                     int32_t* col_idx, void* values, int dtype, int32_t* diag, void* stream) {
  clear_error();
  if (p < 1 || p > LOR_MAX_P) LOR_FAIL(LOR_EINVAL, "p = %d outside [1, %d]", p, LOR_MAX_P);
  if (nel < 0 || ndofs_h1 < 1 || nedges < 1) LOR_FAIL(LOR_EINVAL, "nel < 0, ndofs_h1 < 1 or nedges < 1");
  if (2 * nedges >= (int64_t(1) << 31)) LOR_FAIL(LOR_EOVERFLOW, "2 * nedges >= 2^31");
  if (dtype != LOR_F64 && dtype != LOR_F32) LOR_FAIL(LOR_EINVAL, "dtype must be LOR_F64 or LOR_F32");
  if (!row_ptr || !col_idx || !values) LOR_FAIL(LOR_EINVAL, "an output pointer is NULL");
  if (nel > 0 && (!elem_dofs || !elem_edges)) LOR_FAIL(LOR_EINVAL, "elem_dofs or elem_edges is NULL");
  int rc = check_sched(sched, LOR_ND, p, nel, nedges);
  if (rc) return rc;
  const int32_t* inc_ptr = dev_at<int32_t>(sched, sched->off_inc_ptr);
  const int32_t* inc_list = dev_at<int32_t>(sched, sched->off_inc_list);
  hipStream_t st = as_stream(stream);
  const unsigned blocks = static_cast<unsigned>(ceil_div(nedges, kAuxThreads));
  if (dtype == LOR_F64)
    k_discrete_gradient<double><<<blocks, kAuxThreads, 0, st>>>(p, nedges, ndofs_h1, elem_dofs, elem_edges, inc_ptr,
                                                                inc_list, row_ptr, col_idx,
                                                                static_cast<double*>(values), diag);
  else
    k_discrete_gradient<float><<<blocks, kAuxThreads, 0, st>>>(p, nedges, ndofs_h1, elem_dofs, elem_edges, inc_ptr,
                                                               inc_list, row_ptr, col_idx, static_cast<float*>(values),
                                                               diag);
  LOR_LAUNCHED("k_discrete_gradient");
  return LOR_OK;
}

extern "C" int lor_discrete_curl(int p, int64_t nel, int64_t nedges, int64_t nfaces, const int32_t* elem_edges,
                                 const int32_t* elem_faces, int32_t* workspace, int32_t* row_ptr, int32_t* col_idx,
                                 void* values, int dtype, int32_t* diag, void* stream) {
  clear_error();
  if (p < 1 || p > LOR_MAX_P) LOR_FAIL(LOR_EINVAL, "p = %d outside [1, %d]", p, LOR_MAX_P);
  if (nel < 0 || nedges < 1 || nfaces < 1) LOR_FAIL(LOR_EINVAL, "nel < 0, nedges < 1 or nfaces < 1");
  if (4 * nfaces >= (int64_t(1) << 31)) LOR_FAIL(LOR_EOVERFLOW, "4 * nfaces >= 2^31");
  const int64_t nlocf = 3 * p * p * (p + 1);
  if (nel * nlocf >= (int64_t(1) << 31)) LOR_FAIL(LOR_EOVERFLOW, "nel * 3p^2(p+1) >= 2^31");
  if (nedges >= (int64_t(1) << 31)) LOR_FAIL(LOR_EOVERFLOW, "nedges >= 2^31");
  if (dtype != LOR_F64 && dtype != LOR_F32) LOR_FAIL(LOR_EINVAL, "dtype must be LOR_F64 or LOR_F32");
  if (!workspace || !row_ptr || !col_idx || !values) LOR_FAIL(LOR_EINVAL, "workspace or an output pointer is NULL");
  if (nel > 0 && (!elem_edges || !elem_faces)) LOR_FAIL(LOR_EINVAL, "elem_edges or elem_faces is NULL");
  hipStream_t st = as_stream(stream);
  k_fill_owner<<<static_cast<unsigned>(ceil_div(nfaces, kAuxThreads)), kAuxThreads, 0, st>>>(workspace, nfaces);
  LOR_LAUNCHED("k_fill_owner");
  if (nel > 0) {
    const int64_t total = nel * nlocf;
    k_face_owner<<<static_cast<unsigned>(ceil_div(total, kAuxThreads)), kAuxThreads, 0, st>>>(elem_faces, total,
                                                                                              nfaces, workspace, diag);
    LOR_LAUNCHED("k_face_owner");
  }
  const unsigned blocks = static_cast<unsigned>(ceil_div(nfaces, kAuxThreads));
  if (dtype == LOR_F64)
    k_discrete_curl<double><<<blocks, kAuxThreads, 0, st>>>(p, nfaces, nedges, elem_edges, elem_faces, workspace,
                                                            row_ptr, col_idx, static_cast<double*>(values), diag);
  else
    k_discrete_curl<float><<<blocks, kAuxThreads, 0, st>>>(p, nfaces, nedges, elem_edges, elem_faces, workspace,
                                                           row_ptr, col_idx, static_cast<float*>(values), diag);
  LOR_LAUNCHED("k_discrete_curl");
  return LOR_OK;
}

extern "C" int lor_interp_nodes(int p, int q, int64_t nel, int ncomp, const double* nodes, double* out,
                                void* stream) {
  clear_error();
  if (p < 1 || p > LOR_MAX_P) LOR_FAIL(LOR_EINVAL, "p = %d outside [1, %d]", p, LOR_MAX_P);
  if (q < 1 || q > kMaxNodeOrder) LOR_FAIL(LOR_EINVAL, "q = %d outside [1, %d]", q, kMaxNodeOrder);
  if (ncomp < 1 || ncomp > 3) LOR_FAIL(LOR_EINVAL, "ncomp = %d outside [1, 3]", ncomp);
  if (nel < 0) LOR_FAIL(LOR_EINVAL, "nel < 0");
  if (nel >= (int64_t(1) << 31)) LOR_FAIL(LOR_EOVERFLOW, "nel >= 2^31");
  if (nel == 0) return LOR_OK;
  if (!nodes || !out) LOR_FAIL(LOR_EINVAL, "nodes or out is NULL");
  const InterpBasis B = interp_basis(p, q);
  const size_t lds = sizeof(double) * interp_lds_doubles(p, q, ncomp);
  const dim3 grid(static_cast<unsigned>(nel));
  hipStream_t st = as_stream(stream);
#define LOR_INTERP_CASE(PP)                                                                        \
  case PP:                                                                                         \
    if (ncomp == 1)                                                                                \
      k_interp_nodes<PP + 1, 1><<<grid, kAuxThreads, lds, st>>>(q, nodes, out, B);                  \
    else if (ncomp == 2)                                                                           \
      k_interp_nodes<PP + 1, 2><<<grid, kAuxThreads, lds, st>>>(q, nodes, out, B);                  \
    else                                                                                           \
      k_interp_nodes<PP + 1, 3><<<grid, kAuxThreads, lds, st>>>(q, nodes, out, B);                  \
    break;
  switch (p) {
    LOR_INTERP_CASE(1)
    LOR_INTERP_CASE(2)
    LOR_INTERP_CASE(3)
    LOR_INTERP_CASE(4)
    LOR_INTERP_CASE(5)
    LOR_INTERP_CASE(6)
  }
#undef LOR_INTERP_CASE
  LOR_LAUNCHED("k_interp_nodes");
  return LOR_OK;
}

extern "C" int lor_evec_to_tvec(int p, int64_t nel, int64_t ndofs, const lor_sched* sched, int ncomp,
                                const double* evec, double* tvec, int32_t* diag, void* stream) {
  clear_error();
  if (p < 1 || p > LOR_MAX_P) LOR_FAIL(LOR_EINVAL, "p = %d outside [1, %d]", p, LOR_MAX_P);
  if (ncomp < 1 || ncomp > 3) LOR_FAIL(LOR_EINVAL, "ncomp = %d outside [1, 3]", ncomp);
  if (nel < 0 || ndofs < 1) LOR_FAIL(LOR_EINVAL, "nel < 0 or ndofs < 1");
  if (!tvec || (nel > 0 && !evec)) LOR_FAIL(LOR_EINVAL, "evec or tvec is NULL");
  int rc = check_sched(sched, LOR_H1, p, nel, ndofs);
  if (rc) return rc;
  const int32_t* inc_ptr = dev_at<int32_t>(sched, sched->off_inc_ptr);
  const int32_t* inc_list = dev_at<int32_t>(sched, sched->off_inc_list);
  k_evec_to_tvec<<<static_cast<unsigned>(ceil_div(ndofs, kAuxThreads)), kAuxThreads, 0, as_stream(stream)>>>(
      ndofs, ncomp, inc_ptr, inc_list, evec, tvec, diag);
  LOR_LAUNCHED("k_evec_to_tvec");
  return LOR_OK;
}
