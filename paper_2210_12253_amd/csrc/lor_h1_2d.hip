// Values of the 2D LOR H1 matrix (the 2D variant of Step S1.2): each
// degree-p quadrilateral macro element is split at its Gauss-Lobatto lattice
// into p^2 bilinear subelements; the matrix is the Q1 diffusion + mass matrix
// of that mesh, 9 nonzeros per interior row (Section 3 and Section 4.1).
//
// A workgroup walks a chunk of same-colour macro elements, E at a time:
//   phase 0  gather vertex coordinates, row pointers and the rank table;
//   phase 1  one lane per subelement: the 4x4 matrix (10 unique entries) at
//            the 2x2 Gauss points, into LDS;
//   phase 2  one lane per local stencil entry (vertex l, vertex l'): the sum
//            over the <= 4 subelements holding both, in increasing subelement
//            order (FP64), stored at row_ptr[row] + position-in-row (first
//            contributor: store; later colours: add to the stored value).
#include "lor_common.hpp"
#include "lor_h1_2d_math.hpp"

namespace lor {

int check_sched(const lor_sched* s, int space, int p, int64_t nel, int64_t nrows);
template <typename T, typename R>
int dispatch_2d_owner(int p, const lor_sched* s, int batch, const double* x, const void* k, double beta, void* v,
                      unsigned f, double thr, int32_t* diag, hipStream_t st);

template <int P, typename R>
struct H12Cfg {
  static constexpr int Q = P + 1;
  static constexpr int NSUB = P * P;
  static constexpr int NLOC = Q * Q;
  static constexpr int NENT = (3 * P + 1) * (3 * P + 1);
  static constexpr int NENTP = (NENT + 15) / 16 * 16;
  static constexpr int THREADS = 256;
  static constexpr int PER_EL = NSUB * 10 * static_cast<int>(sizeof(R)) + NENTP + NLOC * 20;
  static constexpr int E0 = THREADS / NSUB < 64 ? THREADS / NSUB : 64;
  // small groups (5 elements at p = 6 in both precisions) and up to 6
  // resident workgroups per CU: the kernel is latency bound
  static constexpr int E1 = (sizeof(R) == 8 ? 24 * 1024 : 16 * 1024) / PER_EL;
  static constexpr int E = (E0 < E1 ? E0 : E1) > 0 ? (E0 < E1 ? E0 : E1) : 1;
  static constexpr int TWE = NENTP / 4;
  static constexpr int CH = 8;
  static constexpr int MAXCHUNK = 256;
  static constexpr int LDS = E * PER_EL + 2 * MAXCHUNK * 4 + 256;
  static constexpr int WPC1 = 160 * 1024 / LDS;
  static constexpr int WPC = WPC1 < 6 ? (WPC1 > 0 ? WPC1 : 1) : 6;  // resident workgroups per CU
  static_assert(E * NSUB <= THREADS, "one subelement per lane");
};

template <int P, typename T, typename R>
__global__ __launch_bounds__(256, (H12Cfg<P, R>::WPC)) void k_h1_2d_assemble(
    const int32_t* __restrict__ order, const int32_t* __restrict__ order_class, int32_t ncol, int32_t chunk,
    const int32_t* __restrict__ elem_dofs, const double* __restrict__ coords, const T* __restrict__ kappa, T beta,
    const int32_t* __restrict__ row_ptr, const uint8_t* __restrict__ tables, int64_t tab_stride,
    const uint16_t* __restrict__ ent_row, const uint64_t* __restrict__ recipe, int64_t nel, int64_t nnz,
    T* __restrict__ values, const T* __restrict__ zero, unsigned flags, R det_thresh, int32_t* __restrict__ diag) {
  using C = H12Cfg<P, R>;
  constexpr int Q = C::Q, NSUB = C::NSUB, NLOC = C::NLOC, NENT = C::NENT, NENTP = C::NENTP, E = C::E;
  constexpr int TH = C::THREADS, TWE = C::TWE, CH = C::CH;
  __shared__ double sX[E * NLOC * 2];
  __shared__ int32_t sRp[E * NLOC];
  __shared__ uint32_t sTabW[E * TWE];
  __shared__ R sSub[E * 10 * NSUB];
  __shared__ int32_t sOrd[C::MAXCHUNK];
  __shared__ int32_t sCls[C::MAXCHUNK];
  const uint8_t* sTab = reinterpret_cast<const uint8_t*>(sTabW);

  kappa += static_cast<int64_t>(blockIdx.y) * nel * NSUB;
  values += static_cast<int64_t>(blockIdx.y) * nnz;
  const int64_t cbeg = static_cast<int64_t>(blockIdx.x) * chunk;
  const int nce = static_cast<int>(ncol - cbeg < chunk ? ncol - cbeg : chunk);
  const int ngr = (nce + E - 1) / E;
  if (static_cast<int>(threadIdx.x) < nce) {
    sOrd[threadIdx.x] = order[cbeg + threadIdx.x];
    sCls[threadIdx.x] = order_class[cbeg + threadIdx.x];
  }
  __syncthreads();

  for (int g = 0; g < ngr; ++g) {
    int tid = threadIdx.x;
    __asm__ volatile("" : "+v"(tid));
    __builtin_assume(tid >= 0 && tid < TH);
    const int ne = nce - g * E < E ? nce - g * E : E;
    lds_barrier();  // the previous group is done with every LDS buffer
    // phase 0
    for (int i = tid; i < ne * NLOC; i += TH) {
      const int el = i / NLOC;
      const int32_t v = elem_dofs[static_cast<int64_t>(sOrd[g * E + el]) * NLOC + (i - el * NLOC)];
      sX[2 * i + 0] = coords[2 * static_cast<int64_t>(v) + 0];
      sX[2 * i + 1] = coords[2 * static_cast<int64_t>(v) + 1];
      sRp[i] = row_ptr[v];
    }
    for (int i = tid; i < ne * TWE; i += TH) {
      const int el = i / TWE;
      const uint32_t* row = reinterpret_cast<const uint32_t*>(tables + sCls[g * E + el] * tab_stride);
      sTabW[i] = row[i - el * TWE];
    }
    lds_barrier();

    // phase 1: subelement matrices
    if (tid < ne * NSUB) {
      const int el = tid / NSUB;
      const int s = tid - el * NSUB;
      const int si = s % P, sj = s / P;
      const R kap = static_cast<R>(kappa[static_cast<int64_t>(sOrd[g * E + el]) * NSUB + s]);
      double X[4][2];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int lv = (si + (v & 1)) + Q * (sj + (v >> 1));
        X[v][0] = sX[2 * (el * NLOC + lv) + 0];
        X[v][1] = sX[2 * (el * NLOC + lv) + 1];
      }
      double e64[2][2], f64[2][2];
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int d = 0; d < 2; ++d) {
          e64[t][d] = X[1 + 2 * t][d] - X[2 * t][d];  // along xi at eta = t
          f64[t][d] = X[t + 2][d] - X[t][d];          // along eta at xi = t
        }
      bool fallback = false;
      R ent[10];
      if constexpr (!std::is_same<R, double>::value) {
        if (flags & LOR_FP64_FALLBACK) {
          R dmin = R(3.0e38), dmax = R(-3.0e38);
#pragma unroll
          for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int a = 0; a < 2; ++a) {
              const R d = R(e64[b][0]) * R(f64[a][1]) - R(e64[b][1]) * R(f64[a][0]);
              dmin = d < dmin ? d : dmin;
              dmax = d > dmax ? d : dmax;
            }
          fallback = !(dmin > R(0)) || dmax > det_thresh * dmin;
        }
      }
      if (!fallback) {
        R e[2][2], f[2][2];
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
          for (int d = 0; d < 2; ++d) {
            e[t][d] = static_cast<R>(e64[t][d]);
            f[t][d] = static_cast<R>(f64[t][d]);
          }
        const bool ok = q1_2d_entries<R>(e, f, kap, static_cast<R>(beta), ent);
        if (!ok && diag) atomicAdd(&diag[1], 1);
      } else {
        double d10[10];
        const bool ok = q1_2d_entries<double>(e64, f64, static_cast<double>(kap), static_cast<double>(beta), d10);
#pragma unroll
        for (int k = 0; k < 10; ++k) ent[k] = static_cast<R>(d10[k]);
        if (diag) {
          atomicAdd(&diag[0], 1);
          if (!ok) atomicAdd(&diag[1], 1);
        }
      }
      R* out = sSub + el * 10 * NSUB + s;
#pragma unroll
      for (int k = 0; k < 10; ++k) out[k * NSUB] = ent[k];
    }
    lds_barrier();

    // phase 2: entry sums and CSR stores (loads before stores, no branch
    // around a memory instruction; a first contributor reads the zero slot)
    for (int base = 0; base < ne * NENT; base += CH * TH) {
      if (base + tid >= ne * NENT) break;
      uint32_t pos[CH];
      T val[CH];
      T old[CH];
      uint64_t recs[CH];
      int32_t ls[CH];
#pragma unroll
      for (int j = 0; j < CH; ++j) {
        const int i0 = base + tid + j * TH;
        const int i = i0 < ne * NENT ? i0 : base + tid;
        const int k = i - (i / NENT) * NENT;
        recs[j] = recipe[k];
        ls[j] = ent_row[k];
      }
#pragma unroll
      for (int j = 0; j < CH; ++j) {
        const int i0 = base + tid + j * TH;
        const int i = i0 < ne * NENT ? i0 : base + tid;
        const int el = i / NENT;
        const int k = i - el * NENT;
        double acc = 0.0;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          const uint32_t code = static_cast<uint32_t>((recs[j] >> (16 * m)) & 0xffffu);
          if (code != 0xffffu)
            acc += static_cast<double>(sSub[(el * 10 + static_cast<int>(code & 127u)) * NSUB + (code >> 7)]);
        }
        const uint32_t t = sTab[el * NENTP + k];
        pos[j] = static_cast<uint32_t>(sRp[el * NLOC + ls[j]]) + (t & kRankMask);
        val[j] = static_cast<T>(acc);
        old[j] = *((t & kFirstBit) ? zero : values + pos[j]);
      }
#pragma unroll
      for (int j = 0; j < CH; ++j) values[pos[j]] = val[j] + old[j];
    }
  }
}

static int num_cus_2d() {
  static int cached[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (cached[dev] == 0) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
    cached[dev] = n;
  }
  return cached[dev];
}

template <int P, typename T, typename R>
static int launch_2d(const lor_sched* sched, int batch, const int32_t* elem_dofs, const double* coords,
                     const void* kappa, double beta, const int32_t* row_ptr, void* values, unsigned flags, double thr,
                     int32_t* diag, hipStream_t st) {
  using C = H12Cfg<P, R>;
  if (sched->tab_stride != C::NENTP || sched->nent != C::NENT)
    LOR_FAIL(LOR_EINVAL, "schedule tables do not match p = %d", P);
  const int32_t* order = dev_at<int32_t>(sched, sched->off_order);
  const int32_t* ocls = dev_at<int32_t>(sched, sched->off_order_class);
  const uint8_t* tab = dev_at<uint8_t>(sched, sched->off_tables);
  const uint16_t* ent_row = dev_at<uint16_t>(sched, sched->off_ent_row);
  const uint64_t* recipe = dev_at<uint64_t>(sched, sched->off_recipe);
  const int wgs = C::WPC * num_cus_2d();
  for (int c = 0; c < sched->ncolors; ++c) {
    const int32_t n = sched->color_ptr[c + 1] - sched->color_ptr[c];
    if (n <= 0) continue;
    const int64_t groups = ceil_div(n, C::E);
    int64_t gpw = ceil_div(groups, wgs);
    if (gpw * C::E > C::MAXCHUNK) gpw = C::MAXCHUNK / C::E;
    const int32_t chunk = static_cast<int32_t>(gpw * C::E);
    dim3 grid(static_cast<unsigned>(ceil_div(n, chunk)), static_cast<unsigned>(batch));
    k_h1_2d_assemble<P, T, R><<<grid, C::THREADS, 0, st>>>(
        order + sched->color_ptr[c], ocls + sched->color_ptr[c], n, chunk, elem_dofs, coords,
        static_cast<const T*>(kappa), static_cast<T>(beta), row_ptr, tab, sched->tab_stride, ent_row, recipe,
        sched->nel, sched->nnz, static_cast<T*>(values), dev_at<T>(sched, sched->off_zero), flags,
        static_cast<R>(thr), diag);
    LOR_LAUNCHED("k_h1_2d_assemble");
  }
  return LOR_OK;
}

template <typename T, typename R>
static int dispatch_2d(int p, const lor_sched* s, int batch, const int32_t* ed, const double* x, const void* k,
                       double beta, const int32_t* rp, void* v, unsigned f, double thr, int32_t* diag,
                       hipStream_t st) {
  switch (p) {
    case 1: return launch_2d<1, T, R>(s, batch, ed, x, k, beta, rp, v, f, thr, diag, st);
    case 2: return launch_2d<2, T, R>(s, batch, ed, x, k, beta, rp, v, f, thr, diag, st);
    case 3: return launch_2d<3, T, R>(s, batch, ed, x, k, beta, rp, v, f, thr, diag, st);
    case 4: return launch_2d<4, T, R>(s, batch, ed, x, k, beta, rp, v, f, thr, diag, st);
    case 5: return launch_2d<5, T, R>(s, batch, ed, x, k, beta, rp, v, f, thr, diag, st);
    case 6: return launch_2d<6, T, R>(s, batch, ed, x, k, beta, rp, v, f, thr, diag, st);
    default: LOR_FAIL(LOR_EUNSUPPORTED, "lor_assemble_h1_2d: p = %d not supported", p);
  }
}

}  // namespace lor

using namespace lor;

extern "C" int lor_assemble_h1_2d(int p, int64_t nel, int64_t ndofs, int batch, const int32_t* elem_dofs,
                                  const double* coords, const void* kappa, double beta, const int32_t* row_ptr,
                                  const lor_sched* sched, void* values, int dtype, unsigned flags,
                                  double det_ratio_thresh, int32_t* diag, void* stream) {
  clear_error();
  if (p < 1 || p > LOR_MAX_P) LOR_FAIL(LOR_EINVAL, "p = %d outside [1, %d]", p, LOR_MAX_P);
  if (nel < 0 || ndofs < 1) LOR_FAIL(LOR_EINVAL, "nel < 0 or ndofs < 1");
  if (batch < 1 || batch > 65535) LOR_FAIL(LOR_EINVAL, "batch outside [1, 65535]");
  if (dtype != LOR_F64 && dtype != LOR_F32) LOR_FAIL(LOR_EINVAL, "dtype must be LOR_F64 or LOR_F32");
  if (flags & ~(LOR_FP64_FALLBACK | LOR_COLORED | LOR_OWNER)) LOR_FAIL(LOR_EINVAL, "unknown flag bits 0x%x", flags);
  if ((flags & LOR_COLORED) && (flags & LOR_OWNER)) LOR_FAIL(LOR_EINVAL, "LOR_COLORED and LOR_OWNER both set");
  if ((flags & LOR_FP64_FALLBACK) && !(det_ratio_thresh >= 1.0))
    LOR_FAIL(LOR_EINVAL, "det_ratio_thresh must be >= 1");
  if (nel > 0 && (!elem_dofs || !coords || !kappa || !row_ptr || !values))
    LOR_FAIL(LOR_EINVAL, "a required pointer is NULL");
  int rc = check_sched(sched, LOR_H1_2D, p, nel, ndofs);
  if (rc) return rc;
  if (static_cast<int64_t>(batch) * sched->nnz >= (int64_t(1) << 40)) LOR_FAIL(LOR_EOVERFLOW, "batch * nnz too large");
  if (nel == 0) return LOR_OK;
  if ((flags & LOR_OWNER) && !sched->owner)
    LOR_FAIL(LOR_EUNSUPPORTED, "LOR_OWNER: the mesh is no 2D box lattice (no owner-computes schedule)");
  hipStream_t st = as_stream(stream);
  // default: owner-computes wherever the schedule has it
  const bool owner = sched->owner && !(flags & LOR_COLORED);
  const unsigned fb = flags & LOR_FP64_FALLBACK;
  if (dtype == LOR_F64)
    return owner ? dispatch_2d_owner<double, double>(p, sched, batch, coords, kappa, beta, values, 0u,
                                                     det_ratio_thresh, diag, st)
                 : dispatch_2d<double, double>(p, sched, batch, elem_dofs, coords, kappa, beta, row_ptr, values, 0u,
                                               det_ratio_thresh, diag, st);
  return owner ? dispatch_2d_owner<float, float>(p, sched, batch, coords, kappa, beta, values, fb, det_ratio_thresh,
                                                 diag, st)
               : dispatch_2d<float, float>(p, sched, batch, elem_dofs, coords, kappa, beta, row_ptr, values, fb,
                                           det_ratio_thresh, diag, st);
}
