// Adjoint of the LOR H1 assembly with respect to kappa and the coordinates.
//
// L = sum_b <Gbar_b, A_b>,  A_b = sum_s kappa_{b,s} K^s + beta M^s  (K^s at kappa = 1).
//   dL/dkappa_{b,s} = sum_{u,v} Gbar_b[pos(s,u,v)] K^s_uv,
//   dL/dX = sum_s <sum_b kappa_{b,s} Gbar_b|s, dK^s/dX> + <sum_b Gbar_b|s, dM^s/dX>.
// One lane per subelement recomputes the geometry and K^s (nothing is stored
// by the forward pass), gathers the cotangent at the 64 CSR positions of its
// 8x8 block for every batch entry, writes dL/dkappa, and runs the reverse of
// the sum-factorised integration to get the adjoint of its 8 corner
// coordinates.  The corners are summed per element vertex in LDS in a fixed
// order (element E-vector), then per global vertex over its sorted
// incidences (deterministic; coordinates are shared by the batch, so their
// gradient is the sum over the batch).
#include <mutex>

#include "lor_common.hpp"
#include "lor_h1_adjoint.hpp"

namespace lor {

// Workspace of the allocation-free entry point: a file-scope device array, one
// copy per GPU, alive until the process ends.  Host code never uses its name
// as an address (on the host it is only a stand-in for the symbol): the
// device address comes from hipGetSymbolAddress, taken once per device with
// that device current, and is what the kernels receive.
constexpr size_t kBwScratchBytes = size_t(32) << 20;
__device__ __align__(256) unsigned char scratch[kBwScratchBytes];

static int bw_scratch_address(void** out) {
  static std::mutex mu;
  static void* addr[64] = {};
  int dev = -1;
  LOR_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) LOR_FAIL(LOR_EDEVICE, "device index %d outside [0, 64)", dev);
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* ptr = nullptr;
    LOR_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) LOR_FAIL(LOR_EDEVICE, "hipGetSymbolAddress returned NULL for the workspace array");
    addr[dev] = ptr;
  }
  *out = addr[dev];
  return LOR_OK;
}

__global__ void k_bw_zero_f64(double* __restrict__ x, int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) x[i] = 0.0;
}

int check_sched(const lor_sched* s, int space, int p, int64_t nel, int64_t nrows);

// One small workgroup per group of E elements (one wave where the
// subelements allow: E p^3 <= 64 lanes), one workgroup per group, so that
// several independent workgroups share a CU and hide each other's latency
// (gathers of coordinates and cotangents, LDS round trips).
template <int P>
struct BwCfg {
  static constexpr int Q = P + 1;
  static constexpr int NSUB = P * P * P;
  static constexpr int NLOC = Q * Q * Q;
  static constexpr int T1 = 3 * P + 1;
  static constexpr int NENT = T1 * T1 * T1;
  static constexpr int NENTP = (NENT + 15) / 16 * 16;
  static constexpr int E = NSUB >= 64 ? 1 : 64 / NSUB;
  static constexpr int THREADS = (E * NSUB + 63) / 64 * 64;
  static constexpr int TWE = NENTP / 4;
};

// Waves per SIMD to reserve registers for: one.  A lane keeps 108
// accumulators, the next batch entry's gathered cotangents and its 64 packed
// pair indices in registers; at two waves per SIMD the FP32 form spills
// (measured at p = 4, 16^3, batch 8: 0.192 ms at two waves with 57 spilled
// registers, 0.143 ms at one).
template <typename R>
struct BwOcc {
  static constexpr int WPE = 1;
};

// Compact index of stencil entry (vertex (x,y,z), offset (dx,dy,dz)) inside
// the element table: rows in lexicographic order, each row's valid offsets in
// (dz, dy, dx) lexicographic order.
template <int P>
__device__ __forceinline__ int compact_index(int x, int y, int z, int dx, int dy, int dz) {
  constexpr int T1 = 3 * P + 1;
  auto cnt = [](int t) { return (t == 0 || t == P) ? 2 : 3; };
  auto pre = [](int t) { return t == 0 ? 0 : 3 * t - 1; };
  const int nx = cnt(x), ny = cnt(y);
  const int rbase = pre(z) * T1 * T1 + cnt(z) * pre(y) * T1 + cnt(z) * ny * pre(x);
  return rbase + ((dz + (z > 0 ? 1 : 0)) * ny + (dy + (y > 0 ? 1 : 0))) * nx + (dx + (x > 0 ? 1 : 0));
}

template <int P, typename T, typename R>
__global__ __launch_bounds__(BwCfg<P>::THREADS, (BwOcc<R>::WPE)) void k_h1_backward(
    int64_t nel, int32_t chunk, const int32_t* __restrict__ elem_dofs, const double* __restrict__ coords,
    const T* __restrict__ kappa, T beta, const int32_t* __restrict__ row_ptr, const uint8_t* __restrict__ tables,
    const int32_t* __restrict__ elem_class, int64_t tab_stride, const uint16_t* __restrict__ ent_row, int batch,
    int64_t nnz, const T* __restrict__ gvals, T* __restrict__ gkappa, double* __restrict__ ework) {
  using C = BwCfg<P>;
  constexpr int Q = C::Q, NSUB = C::NSUB, NLOC = C::NLOC, NENT = C::NENT, NENTP = C::NENTP, E = C::E;
  constexpr int TH = C::THREADS, TWE = C::TWE;
  constexpr int NJ = (E * NENT + TH - 1) / TH;            // gathered entries per lane
  constexpr int GW = E * NENT > 3 * E * 8 * NSUB ? E * NENT : 3 * E * 8 * NSUB;
  // coordinates by component ([d][element vertex]): lanes reading the same
  // corner of neighbouring subelements then hit consecutive words
  __shared__ double sX[3 * E * NLOC];
  __shared__ int32_t sRp[E * NLOC];
  __shared__ uint32_t sTabW[E * TWE];
  // cotangent entries in compact order, later the corner adjoints; in the
  // arithmetic's precision (both are R values), which halves this buffer in
  // the FP32 form
  __shared__ R sGX[GW];
  const uint8_t* sTab = reinterpret_cast<const uint8_t*>(sTabW);
  R* sG = sGX;
  R* sXb = sGX;

  const int64_t cbeg = static_cast<int64_t>(blockIdx.x) * chunk;
  const int nce = static_cast<int>(nel - cbeg < chunk ? nel - cbeg : chunk);
  const int ngr = (nce + E - 1) / E;
  for (int g = 0; g < ngr; ++g) {
    int tid = threadIdx.x;
    __asm__ volatile("" : "+v"(tid));
    __builtin_assume(tid >= 0 && tid < TH);
    const int ne = nce - g * E < E ? nce - g * E : E;
    const int64_t e0 = cbeg + static_cast<int64_t>(g) * E;  // elements e0 .. e0+ne-1
    __syncthreads();
    // staging: every load of a phase is issued before the first is used (a
    // loop that loads, waits and writes LDS per trip would pay one memory
    // round trip per trip); indices past the group are clamped, their values
    // not written
    {
      constexpr int NV = (E * NLOC + TH - 1) / TH, NW = (E * TWE + TH - 1) / TH;
      int32_t vid[NV], cls[NW];
#pragma unroll
      for (int k = 0; k < NV; ++k) {
        const int i = tid + k * TH;
        const int i2 = i < ne * NLOC ? i : 0;
        vid[k] = elem_dofs[e0 * NLOC + i2];
      }
#pragma unroll
      for (int k = 0; k < NW; ++k) {
        const int i = tid + k * TH;
        cls[k] = elem_class[e0 + (i < ne * TWE ? i : 0) / TWE];
      }
      double xv[NV][3];
      int32_t rpv[NV];
      uint32_t tw[NW];
#pragma unroll
      for (int k = 0; k < NV; ++k) {
        const int64_t v = vid[k];
        xv[k][0] = coords[3 * v + 0];
        xv[k][1] = coords[3 * v + 1];
        xv[k][2] = coords[3 * v + 2];
        rpv[k] = row_ptr[v];
      }
#pragma unroll
      for (int k = 0; k < NW; ++k) {
        const int i = tid + k * TH;
        const int i2 = i < ne * TWE ? i : 0;
        tw[k] = reinterpret_cast<const uint32_t*>(tables + cls[k] * tab_stride)[i2 % TWE];
      }
#pragma unroll
      for (int k = 0; k < NV; ++k) {
        const int i = tid + k * TH;
        if (i < ne * NLOC) {
          sX[i] = xv[k][0];
          sX[E * NLOC + i] = xv[k][1];
          sX[2 * E * NLOC + i] = xv[k][2];
          sRp[i] = rpv[k];
        }
      }
#pragma unroll
      for (int k = 0; k < NW; ++k) {
        const int i = tid + k * TH;
        if (i < ne * TWE) sTabW[i] = tw[k];
      }
    }
    // CSR position of every compact entry of the group (row pointer + rank)
    int32_t gpos[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int i = tid + j * TH;
      const int i2 = i < ne * NENT ? i : 0;
      const int el = i2 / NENT;
      gpos[j] = static_cast<int32_t>(ent_row[i2 - el * NENT]);  // local row, completed below
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int i = tid + j * TH;
      const int i2 = i < ne * NENT ? i : 0;
      const int el = i2 / NENT;
      gpos[j] = sRp[el * NLOC + gpos[j]] + (sTab[el * NENTP + (i2 - el * NENT)] & kRankMask);
    }

    const bool act = tid < ne * NSUB;
    const int el = act ? tid / NSUB : 0;
    const int s = act ? tid - el * NSUB : 0;
    const int64_t e = e0 + el;
    const int si = s % P, sj = (s / P) % P, sk = s / (P * P);
    auto edges = [&](R (&ex)[2][2][3], R (&ey)[2][2][3], R (&ez)[2][2][3]) {
      double X[8][3];
#pragma unroll
      for (int v = 0; v < 8; ++v) {
        const int lv = (si + (v & 1)) + Q * ((sj + ((v >> 1) & 1)) + Q * (sk + (v >> 2)));
#pragma unroll
        for (int d = 0; d < 3; ++d) X[v][d] = sX[d * E * NLOC + el * NLOC + lv];
      }
      h1_edges<R>(X, ex, ey, ez);
    };
    R Kt[36], Wk[36], Wm[36];
#pragma unroll
    for (int i = 0; i < 36; ++i) Kt[i] = Wk[i] = Wm[i] = R(0);
    if (act) {
      R ex[2][2][3], ey[2][2][3], ez[2][2][3];
      edges(ex, ey, ez);
      H1Factors<R> F;
      (void)h1_factors<R>(ex, ey, ez, R(1), R(0), F);
#pragma unroll
      for (int u = 0; u < 8; ++u)
#pragma unroll
        for (int v = u; v < 8; ++v) Kt[pair_index(u, v)] = h1_entry<R>(F, u, v);
    }
    // compact index of the 64 ordered corner pairs inside the element's table,
    // two 16-bit indices per register, the same for every batch entry
    uint32_t kpair[32];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int x = si + (u & 1), y = sj + ((u >> 1) & 1), z = sk + (u >> 2);
#pragma unroll
      for (int v = 0; v < 8; v += 2) {
        const uint32_t i0 = static_cast<uint32_t>(
            compact_index<P>(x, y, z, (v & 1) - (u & 1), ((v >> 1) & 1) - ((u >> 1) & 1), (v >> 2) - (u >> 2)));
        const uint32_t i1 = static_cast<uint32_t>(compact_index<P>(
            x, y, z, ((v + 1) & 1) - (u & 1), (((v + 1) >> 1) & 1) - ((u >> 1) & 1), ((v + 1) >> 2) - (u >> 2)));
        kpair[(u * 8 + v) / 2] = i0 | (i1 << 16);
      }
    }
    // the group's cotangent entries in compact (row-contiguous) order and the
    // lane's coefficient: those of the next batch entry are loaded before this
    // entry's compute (unconditionally: the last entry reloads itself), so
    // that their latency is hidden behind it
    const int64_t kofs = e * NSUB + s;
    T gv[NJ];
    T kn;
#pragma unroll
    for (int j = 0; j < NJ; ++j) gv[j] = gvals[gpos[j]];
    kn = kappa[kofs];
    for (int b = 0; b < batch; ++b) {
      lds_barrier();  // the previous entry of the batch has been consumed
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        const int i = tid + j * TH;
        if (i < ne * NENT) sG[i] = static_cast<R>(gv[j]);
      }
      const R kb = static_cast<R>(kn);
      {
        const int bn = b + 1 < batch ? b + 1 : b;
        const T* gn = gvals + static_cast<int64_t>(bn) * nnz;
#pragma unroll
        for (int j = 0; j < NJ; ++j) gv[j] = gn[gpos[j]];
        kn = kappa[static_cast<int64_t>(bn) * nel * NSUB + kofs];
      }
      lds_barrier();
      if (act) {
        const R* ge = sG + el * NENT;
        R gk = R(0);
        // ordered pairs (u, v) and (v, u) both feed the unique entry {u, v};
        // the 8 entries of a corner row are read first, so that the LDS reads
        // overlap instead of each waiting for the previous one
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          R w[8];
#pragma unroll
          for (int v = 0; v < 8; ++v) {
            const uint32_t kp = kpair[(u * 8 + v) / 2];
            w[v] = ge[(v & 1) ? (kp >> 16) : (kp & 0xFFFFu)];
          }
          __builtin_amdgcn_sched_barrier(0);  // keep the 8 reads ahead of their uses
#pragma unroll
          for (int v = 0; v < 8; ++v) {
            gk += Kt[pair_index(u, v)] * w[v];
            Wk[pair_index(u, v)] += kb * w[v];
            Wm[pair_index(u, v)] += w[v];
          }
        }
        gkappa[static_cast<int64_t>(b) * nel * NSUB + kofs] = static_cast<T>(gk);
      }
    }
    __syncthreads();  // sG is reused for the corner adjoints
    if (act) {
      R ex[2][2][3], ey[2][2][3], ez[2][2][3];
      edges(ex, ey, ez);
      R gx[2][2][3], gy[2][2][3], gz[2][2][3];
      h1_adjoint<R>(ex, ey, ez, Wk, Wm, static_cast<R>(beta), gx, gy, gz);
      // corner adjoints from the edge adjoints: e = X(hi) - X(lo)
      R* xb = sXb + el * 24 * NSUB + s;
#pragma unroll
      for (int v = 0; v < 8; ++v) {
        const int a = v & 1, b2 = (v >> 1) & 1, c = v >> 2;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const R val = (a ? gx[b2][c][d] : -gx[b2][c][d]) + (b2 ? gy[a][c][d] : -gy[a][c][d]) +
                        (c ? gz[a][b2][d] : -gz[a][b2][d]);
          xb[(v * 3 + d) * NSUB] = val;
        }
      }
    }
    __syncthreads();
    // per element vertex: sum its <= 8 subelement corners in a fixed order
    for (int i = tid; i < ne * NLOC; i += TH) {
      const int el2 = i / NLOC;
      const int l = i - el2 * NLOC;
      const int x = l % Q, y = (l / Q) % Q, z = l / (Q * Q);
      double acc[3] = {0.0, 0.0, 0.0};
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int sx = x - (u & 1), sy = y - ((u >> 1) & 1), sz = z - (u >> 2);
        if (sx >= 0 && sx < P && sy >= 0 && sy < P && sz >= 0 && sz < P) {
          const int s2 = sx + P * (sy + P * sz);
#pragma unroll
          for (int d = 0; d < 3; ++d) acc[d] += static_cast<double>(sXb[el2 * 24 * NSUB + (u * 3 + d) * NSUB + s2]);
        }
      }
      double* w = ework + ((e0 + el2) * NLOC + l) * 3;
      w[0] = acc[0];
      w[1] = acc[1];
      w[2] = acc[2];
    }
  }
}

// grad_coords[g] = sum over the sorted incidences (e, l) of g of the element
// E-vector adjoint.
__global__ void k_gather_vertices(const int32_t* __restrict__ inc_ptr, const int32_t* __restrict__ inc_list,
                                  int64_t nrows, const double* __restrict__ ework, double* __restrict__ gcoords) {
  const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (g >= nrows) return;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  for (int32_t i = inc_ptr[g]; i < inc_ptr[g + 1]; ++i) {
    const double* w = ework + 3 * static_cast<int64_t>(inc_list[i]);
    a0 += w[0];
    a1 += w[1];
    a2 += w[2];
  }
  gcoords[3 * g + 0] = a0;
  gcoords[3 * g + 1] = a1;
  gcoords[3 * g + 2] = a2;
}

template <int P, typename T, typename R>
static int launch_bw(const lor_sched* sched, int batch, const int32_t* elem_dofs, const double* coords,
                     const void* kappa, double beta, const int32_t* row_ptr, const void* gvals, void* gkappa,
                     double* gcoords, void* workspace, hipStream_t st) {
  using C = BwCfg<P>;
  if (sched->tab_stride != C::NENTP || sched->nent != C::NENT)
    LOR_FAIL(LOR_EINVAL, "schedule tables do not match p = %d", P);
  const uint8_t* tab = dev_at<uint8_t>(sched, sched->off_tables);
  const int64_t nel = sched->nel;
  const int32_t chunk = C::E;  // one group of E elements per workgroup
  double* ework = static_cast<double*>(workspace);
  k_h1_backward<P, T, R><<<static_cast<unsigned>(ceil_div(nel, chunk)), C::THREADS, 0, st>>>(
      nel, chunk, elem_dofs, coords, static_cast<const T*>(kappa), static_cast<T>(beta), row_ptr, tab,
      dev_at<int32_t>(sched, sched->off_class), sched->tab_stride, dev_at<uint16_t>(sched, sched->off_ent_row),
      batch, sched->nnz, static_cast<const T*>(gvals), static_cast<T*>(gkappa), ework);
  LOR_LAUNCHED("k_h1_backward");
  k_gather_vertices<<<static_cast<unsigned>(ceil_div(sched->nrows, 256)), 256, 0, st>>>(
      dev_at<int32_t>(sched, sched->off_inc_ptr), dev_at<int32_t>(sched, sched->off_inc_list), sched->nrows, ework,
      gcoords);
  LOR_LAUNCHED("k_gather_vertices");
  return LOR_OK;
}

template <typename T, typename R>
static int dispatch_bw(int p, const lor_sched* s, int batch, const int32_t* ed, const double* x, const void* k,
                       double beta, const int32_t* rp, const void* gv, void* gk, double* gx, void* ws,
                       hipStream_t st) {
  switch (p) {
    case 1: return launch_bw<1, T, R>(s, batch, ed, x, k, beta, rp, gv, gk, gx, ws, st);
    case 2: return launch_bw<2, T, R>(s, batch, ed, x, k, beta, rp, gv, gk, gx, ws, st);
    case 3: return launch_bw<3, T, R>(s, batch, ed, x, k, beta, rp, gv, gk, gx, ws, st);
    case 4: return launch_bw<4, T, R>(s, batch, ed, x, k, beta, rp, gv, gk, gx, ws, st);
    case 5: return launch_bw<5, T, R>(s, batch, ed, x, k, beta, rp, gv, gk, gx, ws, st);
    case 6: return launch_bw<6, T, R>(s, batch, ed, x, k, beta, rp, gv, gk, gx, ws, st);
    default: LOR_FAIL(LOR_EUNSUPPORTED, "p = %d not compiled", p);
  }
}

}  // namespace lor

using namespace lor;

extern "C" size_t lor_backward_workspace(int p, int64_t nel, int batch, int dtype) {
  if (p < 1 || p > LOR_MAX_P || nel < 0 || batch < 1 || (dtype != LOR_F64 && dtype != LOR_F32)) return 0;
  return sizeof(double) * 3 * static_cast<size_t>(nel) * nloc_h1(p);
}

namespace lor {

// Host-side checks shared by both backward entry points (workspace excluded).
static int check_bw_args(int p, int64_t nel, int64_t ndofs, int batch, const int32_t* elem_dofs,
                         const double* coords, const void* kappa, const int32_t* row_ptr, const void* grad_values,
                         void* grad_kappa, double* grad_coords, int dtype) {
  if (p < 1 || p > LOR_MAX_P) LOR_FAIL(LOR_EINVAL, "p = %d outside [1, %d]", p, LOR_MAX_P);
  if (nel < 0 || ndofs < 1) LOR_FAIL(LOR_EINVAL, "nel < 0 or ndofs < 1");
  if (batch < 1) LOR_FAIL(LOR_EINVAL, "batch < 1");
  if (dtype != LOR_F64 && dtype != LOR_F32) LOR_FAIL(LOR_EINVAL, "dtype must be LOR_F64 or LOR_F32");
  if (!grad_coords) LOR_FAIL(LOR_EINVAL, "grad_coords is NULL");
  if (nel > 0 && (!elem_dofs || !coords || !kappa || !row_ptr || !grad_values || !grad_kappa))
    LOR_FAIL(LOR_EINVAL, "a required pointer is NULL");
  return LOR_OK;
}

static int run_bw(int p, int64_t nel, int64_t ndofs, int batch, const int32_t* elem_dofs, const double* coords,
                  const void* kappa, double beta, const int32_t* row_ptr, const lor_sched* sched,
                  const void* grad_values, void* grad_kappa, double* grad_coords, void* workspace, int dtype,
                  hipStream_t st) {
  if (nel == 0) {
    // a fill kernel rather than a memset node, so that the call can be captured
    k_bw_zero_f64<<<static_cast<unsigned>(ceil_div(3 * ndofs, 256)), 256, 0, st>>>(grad_coords, 3 * ndofs);
    LOR_LAUNCHED("k_bw_zero_f64");
    return LOR_OK;
  }
  if (dtype == LOR_F64)
    return dispatch_bw<double, double>(p, sched, batch, elem_dofs, coords, kappa, beta, row_ptr, grad_values,
                                       grad_kappa, grad_coords, workspace, st);
  return dispatch_bw<float, float>(p, sched, batch, elem_dofs, coords, kappa, beta, row_ptr, grad_values,
                                   grad_kappa, grad_coords, workspace, st);
}

}  // namespace lor

extern "C" int lor_assemble_backward(int p, int64_t nel, int64_t ndofs, int batch, const int32_t* elem_dofs,
                                     const double* coords, const void* kappa, double beta, const int32_t* row_ptr,
                                     const lor_sched* sched, const void* grad_values, void* grad_kappa,
                                     double* grad_coords, void* workspace, int dtype, void* stream) {
  clear_error();
  int rc = check_bw_args(p, nel, ndofs, batch, elem_dofs, coords, kappa, row_ptr, grad_values, grad_kappa,
                         grad_coords, dtype);
  if (rc) return rc;
  if (nel > 0 && !workspace) LOR_FAIL(LOR_EINVAL, "workspace is NULL");
  rc = check_sched(sched, LOR_H1, p, nel, ndofs);
  if (rc) return rc;
  return run_bw(p, nel, ndofs, batch, elem_dofs, coords, kappa, beta, row_ptr, sched, grad_values, grad_kappa,
                grad_coords, workspace, dtype, as_stream(stream));
}

extern "C" size_t lor_backward_noalloc_max_workspace(void) { return kBwScratchBytes; }

extern "C" int lor_assemble_backward_noalloc(int p, int64_t nel, int64_t ndofs, int batch,
                                             const int32_t* elem_dofs, const double* coords, const void* kappa,
                                             double beta, const int32_t* row_ptr, const lor_sched* sched,
                                             const void* grad_values, void* grad_kappa, double* grad_coords,
                                             int dtype, void* stream) {
  clear_error();
  int rc = check_bw_args(p, nel, ndofs, batch, elem_dofs, coords, kappa, row_ptr, grad_values, grad_kappa,
                         grad_coords, dtype);
  if (rc) return rc;
  const size_t need = lor_backward_workspace(p, nel, batch, dtype);
  if (need > kBwScratchBytes)
    LOR_FAIL(LOR_EUNSUPPORTED,
             "the backward needs %zu workspace bytes, above the %zu bytes of the built-in workspace "
             "(nel * (p+1)^3 must be at most %zu); use lor_assemble_backward with a caller workspace",
             need, kBwScratchBytes, kBwScratchBytes / (3 * sizeof(double)));
  rc = check_sched(sched, LOR_H1, p, nel, ndofs);
  if (rc) return rc;
  void* ws = nullptr;
  rc = bw_scratch_address(&ws);
  if (rc) return rc;
  return run_bw(p, nel, ndofs, batch, elem_dofs, coords, kappa, beta, row_ptr, sched, grad_values, grad_kappa,
                grad_coords, ws, dtype, as_stream(stream));
}
