// Values of the LOR H(div) matrix: lowest-order Raviart-Thomas div-div + mass
// on the refined mesh, with the orientation of every face carried by the sign
// of its entry in the signed face map (processor-local assembly step A2).
//
// Same structure as the H(curl) kernel:
//   phase 0  gather vertex coordinates, the row pointers and orientation
//            signs of the element faces and the element rank table into LDS;
//   phase 1  one lane per subelement integrates its 6x6 matrix (21 unique
//            entries) into LDS;
//   phase 2  one lane per local stencil entry (face l, face l') sums the
//            entries of the <= 2 subelements holding both faces, in
//            increasing subelement order, applies sigma_l sigma_l' and stores
//            the sum at row_ptr[row] + position-in-row (first contributor:
//            store, the others: add to the stored value).  A face is shared
//            by at most two subelements (and two macro elements), so the
//            matrix is sparser than the vertex and edge ones.
#include "lor_common.hpp"
#include "lor_rt_math.hpp"

namespace lor {

int check_sched(const lor_sched* s, int space, int p, int64_t nel, int64_t nrows);
template <typename T, typename R>
int dispatch_rt_owner(int p, const lor_sched* s, int batch, const int32_t* ed, const int32_t* fm, const double* x,
                      const void* k, double beta, void* v, unsigned f, double thr, int32_t* diag, hipStream_t st);

template <int P, typename R>
struct RTCfg {
  static constexpr int Q = P + 1;
  static constexpr int NSUB = P * P * P;
  static constexpr int NLOCV = Q * Q * Q;      // vertices per element
  static constexpr int NLOCF = 3 * P * P * Q;  // faces per element
  // local stencil entries: 11 for each of the 3P^2(P-1) faces inside the
  // element, 6 for each of its 6P^2 boundary faces
  static constexpr int NENT = 33 * P * P * P + 3 * P * P;
  static constexpr int NENTP = (NENT + 15) / 16 * 16;
  static constexpr int THREADS = 256;
  static constexpr int PER_EL = NSUB * 21 * static_cast<int>(sizeof(R)) + NENTP + NLOCV * 24 + NLOCF * 5;
  // latency bound like the H(curl) kernel: small groups (2 elements at
  // p = 3) and up to 4 resident workgroups per CU, as LDS allows; the RT
  // integration needs ~128 VGPRs, so FP64 does not spill at 4 either
  static constexpr bool F64 = sizeof(R) == 8;
  static constexpr int BUDGET = F64 ? 16 * 1024 : 12 * 1024;
  static constexpr int E0 = THREADS / NSUB < 64 ? THREADS / NSUB : 64;
  static constexpr int E1 = BUDGET / PER_EL;
  static constexpr int E = (E0 < E1 ? E0 : E1) > 0 ? (E0 < E1 ? E0 : E1) : 1;
  static constexpr int TWE = NENTP / 4;
  static constexpr int CH = 8;  // phase-2 entries per lane handled together
  static constexpr int MAXCHUNK = 256;
  static constexpr int LDS = E * PER_EL + 2 * MAXCHUNK * 4 + 256;
  static constexpr int WPC0 = 4;
  static constexpr int WPC1 = 160 * 1024 / LDS;
  static constexpr int WPC = (WPC0 < WPC1 ? WPC0 : WPC1) > 0 ? (WPC0 < WPC1 ? WPC0 : WPC1) : 1;
  static_assert(E * NSUB <= THREADS, "one subelement per lane");
};

template <int P, typename T, typename R>
__global__ __launch_bounds__(256, (RTCfg<P, R>::WPC)) void k_rt_assemble(
    const int32_t* __restrict__ order, const int32_t* __restrict__ order_class, int32_t ncol, int32_t chunk,
    const int32_t* __restrict__ elem_dofs, const int32_t* __restrict__ elem_faces, const double* __restrict__ coords,
    const T* __restrict__ kappa, T beta, const int32_t* __restrict__ row_ptr, const uint8_t* __restrict__ tables,
    int64_t tab_stride, const uint16_t* __restrict__ ent_row, const int32_t* __restrict__ ent_col,
    const uint64_t* __restrict__ recipe, int64_t nel, int64_t nnz, T* __restrict__ values,
    const T* __restrict__ zero, unsigned flags, R det_thresh, int32_t* __restrict__ diag) {
  using C = RTCfg<P, R>;
  constexpr int Q = C::Q, NSUB = C::NSUB, NLOCV = C::NLOCV, NLOCF = C::NLOCF, NENT = C::NENT;
  constexpr int NENTP = C::NENTP, E = C::E, TH = C::THREADS, TWE = C::TWE, CH = C::CH;
  __shared__ double sX[E * NLOCV * 3];
  __shared__ int32_t sRp[E * NLOCF];
  __shared__ uint8_t sSg[E * NLOCF];
  __shared__ uint32_t sTabW[E * TWE];
  __shared__ R sSub[E * 21 * NSUB];
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
    for (int i = tid; i < ne * NLOCV; i += TH) {
      const int el = i / NLOCV;
      const int32_t v = elem_dofs[static_cast<int64_t>(sOrd[g * E + el]) * NLOCV + (i - el * NLOCV)];
      sX[3 * i + 0] = coords[3 * static_cast<int64_t>(v) + 0];
      sX[3 * i + 1] = coords[3 * static_cast<int64_t>(v) + 1];
      sX[3 * i + 2] = coords[3 * static_cast<int64_t>(v) + 2];
    }
    for (int i = tid; i < ne * NLOCF; i += TH) {
      const int el = i / NLOCF;
      const int32_t raw = elem_faces[static_cast<int64_t>(sOrd[g * E + el]) * NLOCF + (i - el * NLOCF)];
      const int32_t gid = raw < 0 ? -1 - raw : raw;
      sRp[i] = row_ptr[gid];
      sSg[i] = raw < 0 ? 1 : 0;
    }
    for (int i = tid; i < ne * TWE; i += TH) {
      const int el = i / TWE;
      const uint32_t* row = reinterpret_cast<const uint32_t*>(tables + sCls[g * E + el] * tab_stride);
      sTabW[i] = row[i - el * TWE];
    }
    lds_barrier();

    // phase 1: subelement matrices (local +axis orientation)
    if (tid < ne * NSUB) {
      const int el = tid / NSUB;
      const int s = tid - el * NSUB;
      const int si = s % P, sj = (s / P) % P, sk = s / (P * P);
      const R kap = static_cast<R>(kappa[static_cast<int64_t>(sOrd[g * E + el]) * NSUB + s]);
      R* out = sSub + el * 21 * NSUB + s;
      auto load_X = [&](double (&X)[8][3]) {
#pragma unroll
        for (int v = 0; v < 8; ++v) {
          const int lv = (si + (v & 1)) + Q * ((sj + ((v >> 1) & 1)) + Q * (sk + (v >> 2)));
#pragma unroll
          for (int d = 0; d < 3; ++d) X[v][d] = sX[3 * (el * NLOCV + lv) + d];
        }
      };
      bool fallback = false;
      if constexpr (!std::is_same<R, double>::value) {
        if (flags & LOR_FP64_FALLBACK) {
          R ex[2][2][3], ey[2][2][3], ez[2][2][3];
          double X[8][3];
          load_X(X);
          h1_edges<R>(X, ex, ey, ez);
          R dmin, dmax;
          h1_corner_det_range<R>(ex, ey, ez, dmin, dmax);
          fallback = !(dmin > R(0)) || dmax > det_thresh * dmin;
        }
      }
      if (!fallback) {
        R ex[2][2][3], ey[2][2][3], ez[2][2][3];
        {
          double X[8][3];
          load_X(X);
          h1_edges<R>(X, ex, ey, ez);
        }
        RTFactors<R> F;
        const bool ok = rt_factors<R>(ex, ey, ez, kap, static_cast<R>(beta), F);
#pragma unroll
        for (int u = 0; u < 6; ++u)
#pragma unroll
          for (int v = u; v < 6; ++v) out[pair_index6(u, v) * NSUB] = rt_entry<R>(F, u, v);
        if (!ok && diag) atomicAdd(&diag[1], 1);
      }
      if (fallback) {
        double ex[2][2][3], ey[2][2][3], ez[2][2][3];
        {
          double X[8][3];
          load_X(X);
          h1_edges<double>(X, ex, ey, ez);
        }
        RTFactors<double> F;
        const bool ok = rt_factors<double>(ex, ey, ez, static_cast<double>(kap), static_cast<double>(beta), F);
#pragma unroll
        for (int u = 0; u < 6; ++u)
#pragma unroll
          for (int v = u; v < 6; ++v) out[pair_index6(u, v) * NSUB] = static_cast<R>(rt_entry<double>(F, u, v));
        if (diag) {
          atomicAdd(&diag[0], 1);
          if (!ok) atomicAdd(&diag[1], 1);
        }
      }
    }
    lds_barrier();

    // phase 2: entry sums and CSR stores, CH entries per lane at a time with
    // every load issued before the stores and no branch around a memory
    // instruction (a first contributor reads its old value from the zero
    // slot; a lane past the end repeats its first store of the chunk)
    for (int base = 0; base < ne * NENT; base += CH * TH) {
      if (base + tid >= ne * NENT) break;
      uint32_t pos[CH];
      T val[CH];
      T old[CH];
      uint64_t recs[CH];
      int32_t ls[CH], cs[CH];
#pragma unroll
      for (int j = 0; j < CH; ++j) {  // reference-element tables (cache resident), all in flight
        const int i0 = base + tid + j * TH;
        const int i = i0 < ne * NENT ? i0 : base + tid;
        const int k = i - (i / NENT) * NENT;
        recs[j] = recipe[k];
        ls[j] = ent_row[k];
        cs[j] = ent_col[k];
      }
#pragma unroll
      for (int j = 0; j < CH; ++j) {
        const int i0 = base + tid + j * TH;
        const int i = i0 < ne * NENT ? i0 : base + tid;
        const int el = i / NENT;
        const int k = i - el * NENT;
        const int l = ls[j];
        const int c = cs[j];
        const uint64_t rec = recs[j];
        double acc = 0.0;
#pragma unroll
        for (int m = 0; m < 2; ++m) {  // a face lies in at most two subelements
          const uint32_t code = static_cast<uint32_t>((rec >> (16 * m)) & 0xffffu);
          if (code != 0xffffu)
            acc += static_cast<double>(sSub[(el * 21 + static_cast<int>(code & 127u)) * NSUB + (code >> 7)]);
        }
        if (sSg[el * NLOCF + l] ^ sSg[el * NLOCF + c]) acc = -acc;
        const uint32_t t = sTab[el * NENTP + k];
        pos[j] = static_cast<uint32_t>(sRp[el * NLOCF + l]) + (t & kRankMask);
        val[j] = static_cast<T>(acc);
        old[j] = *((t & kFirstBit) ? zero : values + pos[j]);
      }
#pragma unroll
      for (int j = 0; j < CH; ++j) values[pos[j]] = val[j] + old[j];
    }
  }
}

static int num_cus_rt() {
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
static int launch_rt(const lor_sched* sched, int batch, const int32_t* elem_dofs, const int32_t* elem_faces,
                     const double* coords, const void* kappa, double beta, const int32_t* row_ptr, void* values,
                     unsigned flags, double thr, int32_t* diag, hipStream_t st) {
  using C = RTCfg<P, R>;
  if (sched->tab_stride != C::NENTP || sched->nent != C::NENT)
    LOR_FAIL(LOR_EINVAL, "schedule tables do not match p = %d", P);
  const int32_t* order = dev_at<int32_t>(sched, sched->off_order);
  const int32_t* ocls = dev_at<int32_t>(sched, sched->off_order_class);
  const uint8_t* tab = dev_at<uint8_t>(sched, sched->off_tables);
  const uint16_t* ent_row = dev_at<uint16_t>(sched, sched->off_ent_row);
  const int32_t* ent_col = dev_at<int32_t>(sched, sched->off_st_col);
  const uint64_t* recipe = dev_at<uint64_t>(sched, sched->off_recipe);
  const int wgs = C::WPC * num_cus_rt();
  for (int c = 0; c < sched->ncolors; ++c) {
    const int32_t n = sched->color_ptr[c + 1] - sched->color_ptr[c];
    if (n <= 0) continue;
    const int64_t groups = ceil_div(n, C::E);
    int64_t gpw = ceil_div(groups, wgs);
    if (gpw * C::E > C::MAXCHUNK) gpw = C::MAXCHUNK / C::E;
    const int32_t chunk = static_cast<int32_t>(gpw * C::E);
    dim3 grid(static_cast<unsigned>(ceil_div(n, chunk)), static_cast<unsigned>(batch));
    k_rt_assemble<P, T, R><<<grid, C::THREADS, 0, st>>>(
        order + sched->color_ptr[c], ocls + sched->color_ptr[c], n, chunk, elem_dofs, elem_faces, coords,
        static_cast<const T*>(kappa), static_cast<T>(beta), row_ptr, tab, sched->tab_stride, ent_row, ent_col, recipe,
        sched->nel, sched->nnz, static_cast<T*>(values), dev_at<T>(sched, sched->off_zero), flags,
        static_cast<R>(thr), diag);
    LOR_LAUNCHED("k_rt_assemble");
  }
  return LOR_OK;
}

template <typename T, typename R>
static int dispatch_rt(int p, const lor_sched* s, int batch, const int32_t* ed, const int32_t* fm, const double* x,
                       const void* k, double beta, const int32_t* rp, void* v, unsigned f, double thr, int32_t* diag,
                       hipStream_t st) {
  switch (p) {
    case 1: return launch_rt<1, T, R>(s, batch, ed, fm, x, k, beta, rp, v, f, thr, diag, st);
    case 2: return launch_rt<2, T, R>(s, batch, ed, fm, x, k, beta, rp, v, f, thr, diag, st);
    case 3: return launch_rt<3, T, R>(s, batch, ed, fm, x, k, beta, rp, v, f, thr, diag, st);
    case 4: return launch_rt<4, T, R>(s, batch, ed, fm, x, k, beta, rp, v, f, thr, diag, st);
    case 5: return launch_rt<5, T, R>(s, batch, ed, fm, x, k, beta, rp, v, f, thr, diag, st);
    case 6: return launch_rt<6, T, R>(s, batch, ed, fm, x, k, beta, rp, v, f, thr, diag, st);
    default: LOR_FAIL(LOR_EUNSUPPORTED, "lor_assemble_rt: p = %d not supported", p);
  }
}

}  // namespace lor

using namespace lor;

extern "C" int lor_assemble_rt(int p, int64_t nel, int64_t ndofs_h1, int64_t nfaces, int batch,
                               const int32_t* elem_dofs, const int32_t* elem_faces, const double* coords,
                               const void* kappa, double beta, const int32_t* row_ptr, const lor_sched* sched,
                               void* values, int dtype, unsigned flags, double det_ratio_thresh, int32_t* diag,
                               void* stream) {
  clear_error();
  if (p < 1 || p > LOR_MAX_P) LOR_FAIL(LOR_EINVAL, "p = %d outside [1, %d]", p, LOR_MAX_P);
  if (nel < 0 || ndofs_h1 < 1 || nfaces < 1) LOR_FAIL(LOR_EINVAL, "nel < 0, ndofs_h1 < 1 or nfaces < 1");
  if (batch < 1 || batch > 65535) LOR_FAIL(LOR_EINVAL, "batch outside [1, 65535]");
  if (dtype != LOR_F64 && dtype != LOR_F32) LOR_FAIL(LOR_EINVAL, "dtype must be LOR_F64 or LOR_F32");
  if (flags & ~(LOR_FP64_FALLBACK | LOR_COLORED | LOR_OWNER)) LOR_FAIL(LOR_EINVAL, "unknown flag bits 0x%x", flags);
  if ((flags & LOR_COLORED) && (flags & LOR_OWNER)) LOR_FAIL(LOR_EINVAL, "LOR_COLORED and LOR_OWNER both set");
  if ((flags & LOR_FP64_FALLBACK) && !(det_ratio_thresh >= 1.0))
    LOR_FAIL(LOR_EINVAL, "det_ratio_thresh must be >= 1");
  if (nel > 0 && (!elem_dofs || !elem_faces || !coords || !kappa || !row_ptr || !values))
    LOR_FAIL(LOR_EINVAL, "a required pointer is NULL");
  int rc = check_sched(sched, LOR_RT, p, nel, nfaces);
  if (rc) return rc;
  if (static_cast<int64_t>(batch) * sched->nnz >= (int64_t(1) << 40)) LOR_FAIL(LOR_EOVERFLOW, "batch * nnz too large");
  if (nel == 0) return LOR_OK;
  if ((flags & LOR_OWNER) && !sched->owner)
    LOR_FAIL(LOR_EUNSUPPORTED, "LOR_OWNER: the face map is no face lattice (no owner-computes schedule)");
  hipStream_t st = as_stream(stream);
  // default: owner-computes wherever the schedule has it
  const bool owner = sched->owner && !(flags & LOR_COLORED);
  const unsigned fb = flags & LOR_FP64_FALLBACK;
  if (dtype == LOR_F64)
    return owner ? dispatch_rt_owner<double, double>(p, sched, batch, elem_dofs, elem_faces, coords, kappa, beta,
                                                     values, 0u, det_ratio_thresh, diag, st)
                 : dispatch_rt<double, double>(p, sched, batch, elem_dofs, elem_faces, coords, kappa, beta, row_ptr,
                                               values, 0u, det_ratio_thresh, diag, st);
  return owner ? dispatch_rt_owner<float, float>(p, sched, batch, elem_dofs, elem_faces, coords, kappa, beta, values,
                                                 fb, det_ratio_thresh, diag, st)
               : dispatch_rt<float, float>(p, sched, batch, elem_dofs, elem_faces, coords, kappa, beta, row_ptr,
                                           values, fb, det_ratio_thresh, diag, st);
}
