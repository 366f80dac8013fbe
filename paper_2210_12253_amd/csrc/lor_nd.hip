// Values of the LOR H(curl) matrix: lowest-order Nedelec curl-curl + mass on
// the refined mesh, with the orientation of every edge carried by the sign of
// its entry in the signed edge map (processor-local assembly step A2).
//
// A workgroup walks a chunk of macro elements of one colour, E at a time:
//   phase 0  gather vertex coordinates, the row pointers and orientation
//            signs of the element edges and the element rank table into LDS
//            (in FP64 from registers filled while the previous group was
//            computed);
//   phase 1  one lane per subelement integrates its 12x12 matrix (78 unique
//            entries) into LDS;
//   phase 2  one lane per local stencil entry (edge l, edge l') sums the
//            entries of the <= 4 subelements holding both edges, in
//            increasing subelement order (atomic-free, FP64, bitwise
//            symmetric), applies sigma_l sigma_l' and stores the sum at
//            row_ptr[row] + position-in-row (first contributor: store, the
//            others: add to the stored value).  The reference-element recipe
//            of every entry is computed once on the host (the shared column
//            pattern of step A1).
#include "lor_common.hpp"
#include "lor_nd_math.hpp"

namespace lor {

int check_sched(const lor_sched* s, int space, int p, int64_t nel, int64_t nrows);
template <typename T, typename R>
int dispatch_nd_owner(int p, const lor_sched* s, int batch, const int32_t* ed, const int32_t* em, const double* x,
                      const void* k, double beta, const int32_t* rp, void* v, unsigned f, double thr, int32_t* diag,
                      hipStream_t st);

template <int P, typename R>
struct NDCfg {
  static constexpr int Q = P + 1;
  static constexpr int NSUB = P * P * P;
  static constexpr int NLOCV = Q * Q * Q;       // vertices per element
  static constexpr int NLOCE = 3 * P * Q * Q;   // edges per element
  static constexpr int NENT = 99 * P * P * P + 42 * P * P + 3 * P;  // local stencil entries
  static constexpr int NENTP = (NENT + 15) / 16 * 16;
  static constexpr int THREADS = 256;
  static constexpr int PER_EL = NSUB * 78 * static_cast<int>(sizeof(R)) + NENTP + NLOCV * 24 + NLOCE * 5;
  // The kernel is latency bound (few elements per colour, short phases
  // between barriers), so small groups and several resident workgroups per
  // CU beat one large group per CU.  FP64 keeps 256 VGPRs per lane (two
  // workgroups per CU) because the subelement integration spills below
  // that; FP32 runs four workgroups per CU.
  static constexpr bool F64 = sizeof(R) == 8;
  static constexpr int BUDGET = F64 ? 50 * 1024 : 30 * 1024;  // LDS for the per-element buffers
  static constexpr int E0 = THREADS / NSUB < 64 ? THREADS / NSUB : 64;
  static constexpr int E1 = BUDGET / PER_EL;
  static constexpr int E = (E0 < E1 ? E0 : E1) > 0 ? (E0 < E1 ? E0 : E1) : 1;
  static constexpr int TWE = NENTP / 4;
  static constexpr int CH = 8;  // phase-2 entries per lane handled together
  static constexpr int NVS = (E * NLOCV + THREADS - 1) / THREADS;  // staged vertices per lane
  static constexpr int NES = (E * NLOCE + THREADS - 1) / THREADS;  // staged edges per lane
  static constexpr int NTS = (E * TWE + THREADS - 1) / THREADS;    // staged table words per lane
  static constexpr int MAXCHUNK = 256;
  static constexpr int LDS = E * PER_EL + 2 * MAXCHUNK * 4 + 256;
  static constexpr int WPC0 = F64 ? 2 : 4;
  static constexpr int WPC1 = 160 * 1024 / LDS;
  static constexpr int WPC = (WPC0 < WPC1 ? WPC0 : WPC1) > 0 ? (WPC0 < WPC1 ? WPC0 : WPC1) : 1;  // workgroups per CU
  static_assert(E * NSUB <= THREADS, "one subelement per lane");
};

template <int P, typename T, typename R>
__global__ __launch_bounds__(256, (NDCfg<P, R>::WPC)) void k_nd_assemble(
    const int32_t* __restrict__ order, const int32_t* __restrict__ order_class, int32_t ncol, int32_t chunk,
    const int32_t* __restrict__ elem_dofs,
    const int32_t* __restrict__ elem_edges, const double* __restrict__ coords, const T* __restrict__ kappa, T beta,
    const int32_t* __restrict__ row_ptr, const uint8_t* __restrict__ tables, int64_t tab_stride,
    const uint16_t* __restrict__ ent_row, const int32_t* __restrict__ ent_col, const uint64_t* __restrict__ recipe,
    int64_t nel, int64_t nnz, T* __restrict__ values, const T* __restrict__ zero, unsigned flags, R det_thresh,
    int32_t* __restrict__ diag) {
  using C = NDCfg<P, R>;
  constexpr int Q = C::Q, NSUB = C::NSUB, NLOCV = C::NLOCV, NLOCE = C::NLOCE, NENT = C::NENT;
  constexpr int NENTP = C::NENTP, E = C::E, TH = C::THREADS, TWE = C::TWE, CH = C::CH;
  __shared__ double sX[E * NLOCV * 3];
  __shared__ int32_t sRp[E * NLOCE];
  __shared__ uint8_t sSg[E * NLOCE];
  __shared__ uint32_t sTabW[E * TWE];
  __shared__ R sSub[E * 78 * NSUB];
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

  // FP64 staging is software-pipelined: the element-map words of group g + 2
  // and the coordinates, row pointers, table words and coefficients of group
  // g + 1 are loaded into registers while group g is computed.  FP32 runs four
  // workgroups per CU at 128 VGPRs, where those registers spill; it gathers
  // each group straight into LDS instead (measured: pipelining takes the
  // p = 3 FP64 launch from 0.346 to 0.329 ms and the FP32 one from 0.202 to
  // 0.221 ms).
  constexpr int NVS = C::NVS, NES = C::NES, NTS = C::NTS;
  constexpr bool PIPE = C::F64;
  auto gsize = [&](int g) { return nce - g * E < E ? nce - g * E : E; };
  auto load_ids = [&](int g, int32_t (&vid)[NVS], int32_t (&eid)[NES]) {
    const int t = threadIdx.x;
#pragma unroll
    for (int j = 0; j < NVS; ++j) {
      const int i = t + j * TH;
      vid[j] = 0;
      if (g < ngr && i < gsize(g) * NLOCV) {
        const int el = i / NLOCV;
        vid[j] = elem_dofs[static_cast<int64_t>(sOrd[g * E + el]) * NLOCV + (i - el * NLOCV)];
      }
    }
#pragma unroll
    for (int j = 0; j < NES; ++j) {
      const int i = t + j * TH;
      eid[j] = 0;
      if (g < ngr && i < gsize(g) * NLOCE) {
        const int el = i / NLOCE;
        eid[j] = elem_edges[static_cast<int64_t>(sOrd[g * E + el]) * NLOCE + (i - el * NLOCE)];
      }
    }
  };
  auto load_data = [&](int g, const int32_t (&vid)[NVS], const int32_t (&eid)[NES], double (&xq)[NVS][3],
                       int32_t (&rq)[NES], uint32_t (&tq)[NTS], T& kq) {
    const int t = threadIdx.x;
    if (g >= ngr) return;
    const int n = gsize(g);
#pragma unroll
    for (int j = 0; j < NVS; ++j) {
      if (t + j * TH < n * NLOCV) {
        const int64_t v3 = 3 * static_cast<int64_t>(vid[j]);
        xq[j][0] = coords[v3 + 0];
        xq[j][1] = coords[v3 + 1];
        xq[j][2] = coords[v3 + 2];
      }
    }
#pragma unroll
    for (int j = 0; j < NES; ++j) {
      if (t + j * TH < n * NLOCE) rq[j] = row_ptr[eid[j] < 0 ? -1 - eid[j] : eid[j]];
    }
#pragma unroll
    for (int j = 0; j < NTS; ++j) {
      const int i = t + j * TH;
      if (i < n * TWE) {
        const int el = i / TWE;
        tq[j] = reinterpret_cast<const uint32_t*>(tables + sCls[g * E + el] * tab_stride)[i - el * TWE];
      }
    }
    if (t < n * NSUB) {
      const int el = t / NSUB;
      kq = kappa[static_cast<int64_t>(sOrd[g * E + el]) * NSUB + (t - el * NSUB)];
    }
  };
  int32_t vid_n[NVS], eid_n[NES], eq[NES];
  double xq[NVS][3] = {};
  int32_t rq[NES] = {};
  uint32_t tq[NTS] = {};
  T kq = T(0);
  if constexpr (PIPE) {
    int32_t v0[NVS], e0[NES];
    load_ids(0, v0, e0);
    load_data(0, v0, e0, xq, rq, tq, kq);
#pragma unroll
    for (int j = 0; j < NES; ++j) eq[j] = e0[j];
    load_ids(1, vid_n, eid_n);
  }

  for (int g = 0; g < ngr; ++g) {
    int tid = threadIdx.x;
    __asm__ volatile("" : "+v"(tid));
    __builtin_assume(tid >= 0 && tid < TH);
    const int ne = gsize(g);
    lds_barrier();  // the previous group is done with every LDS buffer
    // phase 0: stage the group in LDS
    T kcur = T(0);
    if constexpr (PIPE) {
#pragma unroll
      for (int j = 0; j < NVS; ++j) {
        const int i = tid + j * TH;
        if (i < ne * NLOCV) {
          sX[3 * i + 0] = xq[j][0];
          sX[3 * i + 1] = xq[j][1];
          sX[3 * i + 2] = xq[j][2];
        }
      }
#pragma unroll
      for (int j = 0; j < NES; ++j) {
        const int i = tid + j * TH;
        if (i < ne * NLOCE) {
          sRp[i] = rq[j];
          sSg[i] = eq[j] < 0 ? 1 : 0;
        }
      }
#pragma unroll
      for (int j = 0; j < NTS; ++j) {
        const int i = tid + j * TH;
        if (i < ne * TWE) sTabW[i] = tq[j];
      }
      kcur = kq;
      load_data(g + 1, vid_n, eid_n, xq, rq, tq, kq);
#pragma unroll
      for (int j = 0; j < NES; ++j) eq[j] = eid_n[j];
      load_ids(g + 2, vid_n, eid_n);
    } else {
      // every load of a phase before the first use: the map words, then the
      // coordinates, row pointers, table words and the lane's coefficient
      // (indices past the group clamped, their values not written)
      int32_t vid[NVS], eid[NES];
#pragma unroll
      for (int j = 0; j < NVS; ++j) {
        const int i = tid + j * TH;
        const int i2 = i < ne * NLOCV ? i : 0;
        const int el = i2 / NLOCV;
        vid[j] = elem_dofs[static_cast<int64_t>(sOrd[g * E + el]) * NLOCV + (i2 - el * NLOCV)];
      }
#pragma unroll
      for (int j = 0; j < NES; ++j) {
        const int i = tid + j * TH;
        const int i2 = i < ne * NLOCE ? i : 0;
        const int el = i2 / NLOCE;
        eid[j] = elem_edges[static_cast<int64_t>(sOrd[g * E + el]) * NLOCE + (i2 - el * NLOCE)];
      }
      uint32_t tw[NTS];
#pragma unroll
      for (int j = 0; j < NTS; ++j) {
        const int i = tid + j * TH;
        const int i2 = i < ne * TWE ? i : 0;
        const int el = i2 / TWE;
        tw[j] = reinterpret_cast<const uint32_t*>(tables + sCls[g * E + el] * tab_stride)[i2 - el * TWE];
      }
      {
        const int t2 = tid < ne * NSUB ? tid : 0;
        const int el = t2 / NSUB;
        kcur = kappa[static_cast<int64_t>(sOrd[g * E + el]) * NSUB + (t2 - el * NSUB)];
      }
      double xv[NVS][3];
      int32_t rv[NES];
#pragma unroll
      for (int j = 0; j < NVS; ++j) {
        const int64_t v3 = 3 * static_cast<int64_t>(vid[j]);
        xv[j][0] = coords[v3 + 0];
        xv[j][1] = coords[v3 + 1];
        xv[j][2] = coords[v3 + 2];
      }
#pragma unroll
      for (int j = 0; j < NES; ++j) rv[j] = row_ptr[eid[j] < 0 ? -1 - eid[j] : eid[j]];
#pragma unroll
      for (int j = 0; j < NVS; ++j) {
        const int i = tid + j * TH;
        if (i < ne * NLOCV) {
          sX[3 * i + 0] = xv[j][0];
          sX[3 * i + 1] = xv[j][1];
          sX[3 * i + 2] = xv[j][2];
        }
      }
#pragma unroll
      for (int j = 0; j < NES; ++j) {
        const int i = tid + j * TH;
        if (i < ne * NLOCE) {
          sRp[i] = rv[j];
          sSg[i] = eid[j] < 0 ? 1 : 0;
        }
      }
#pragma unroll
      for (int j = 0; j < NTS; ++j) {
        const int i = tid + j * TH;
        if (i < ne * TWE) sTabW[i] = tw[j];
      }
    }
    lds_barrier();

    // phase 1: subelement matrices (local +axis orientation)
    if (tid < ne * NSUB) {
      const int el = tid / NSUB;
      const int s = tid - el * NSUB;
      const int si = s % P, sj = (s / P) % P, sk = s / (P * P);
      const R kap = static_cast<R>(kcur);
      R* out = sSub + el * 78 * NSUB + s;
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
        H1Factors<R> F;
        NDCurl<R> W;
        const bool ok = nd_factors<R>(ex, ey, ez, kap, static_cast<R>(beta), F, W);
#pragma unroll
        for (int u = 0; u < 12; ++u)
#pragma unroll
          for (int v = u; v < 12; ++v) out[pair_index12(u, v) * NSUB] = nd_entry<R>(F, W, u, v);
        if (!ok && diag) atomicAdd(&diag[1], 1);
      }
      if (fallback) {
        double ex[2][2][3], ey[2][2][3], ez[2][2][3];
        {
          double X[8][3];
          load_X(X);
          h1_edges<double>(X, ex, ey, ez);
        }
        H1Factors<double> F;
        NDCurl<double> W;
        const bool ok = nd_factors<double>(ex, ey, ez, static_cast<double>(kap), static_cast<double>(beta), F, W);
#pragma unroll
        for (int u = 0; u < 12; ++u)
#pragma unroll
          for (int v = u; v < 12; ++v) out[pair_index12(u, v) * NSUB] = static_cast<R>(nd_entry<double>(F, W, u, v));
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
        for (int m = 0; m < 4; ++m) {
          const uint32_t code = static_cast<uint32_t>((rec >> (16 * m)) & 0xffffu);
          if (code != 0xffffu)
            acc += static_cast<double>(sSub[(el * 78 + static_cast<int>(code & 127u)) * NSUB + (code >> 7)]);
        }
        if (sSg[el * NLOCE + l] ^ sSg[el * NLOCE + c]) acc = -acc;
        const uint32_t t = sTab[el * NENTP + k];
        pos[j] = static_cast<uint32_t>(sRp[el * NLOCE + l]) + (t & kRankMask);
        val[j] = static_cast<T>(acc);
        old[j] = *((t & kFirstBit) ? zero : values + pos[j]);
      }
#pragma unroll
      for (int j = 0; j < CH; ++j) values[pos[j]] = val[j] + old[j];
    }
  }
}

static int num_cus_nd() {
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
static int launch_nd(const lor_sched* sched, int batch, const int32_t* elem_dofs, const int32_t* elem_edges,
                     const double* coords, const void* kappa, double beta, const int32_t* row_ptr, void* values,
                     unsigned flags, double thr, int32_t* diag, hipStream_t st) {
  using C = NDCfg<P, R>;
  if (sched->tab_stride != C::NENTP || sched->nent != C::NENT)
    LOR_FAIL(LOR_EINVAL, "schedule tables do not match p = %d", P);
  const int32_t* order = dev_at<int32_t>(sched, sched->off_order);
  const int32_t* ocls = dev_at<int32_t>(sched, sched->off_order_class);
  const uint8_t* tab = dev_at<uint8_t>(sched, sched->off_tables);
  const uint16_t* ent_row = dev_at<uint16_t>(sched, sched->off_ent_row);
  const int32_t* ent_col = dev_at<int32_t>(sched, sched->off_st_col);
  const uint64_t* recipe = dev_at<uint64_t>(sched, sched->off_recipe);
  const int wgs = C::WPC * num_cus_nd();
  for (int c = 0; c < sched->ncolors; ++c) {
    const int32_t n = sched->color_ptr[c + 1] - sched->color_ptr[c];
    if (n <= 0) continue;
    const int64_t groups = ceil_div(n, C::E);
    int64_t gpw = ceil_div(groups, wgs);
    if (gpw * C::E > C::MAXCHUNK) gpw = C::MAXCHUNK / C::E;
    const int32_t chunk = static_cast<int32_t>(gpw * C::E);
    dim3 grid(static_cast<unsigned>(ceil_div(n, chunk)), static_cast<unsigned>(batch));
    k_nd_assemble<P, T, R><<<grid, C::THREADS, 0, st>>>(
        order + sched->color_ptr[c], ocls + sched->color_ptr[c], n, chunk, elem_dofs, elem_edges, coords, static_cast<const T*>(kappa),
        static_cast<T>(beta), row_ptr, tab, sched->tab_stride, ent_row, ent_col, recipe, sched->nel, sched->nnz,
        static_cast<T*>(values), dev_at<T>(sched, sched->off_zero), flags, static_cast<R>(thr), diag);
    LOR_LAUNCHED("k_nd_assemble");
  }
  return LOR_OK;
}

template <typename T, typename R>
static int dispatch_nd(int p, const lor_sched* s, int batch, const int32_t* ed, const int32_t* ee, const double* x,
                       const void* k, double beta, const int32_t* rp, void* v, unsigned f, double thr, int32_t* diag,
                       hipStream_t st) {
  switch (p) {
    case 1: return launch_nd<1, T, R>(s, batch, ed, ee, x, k, beta, rp, v, f, thr, diag, st);
    case 2: return launch_nd<2, T, R>(s, batch, ed, ee, x, k, beta, rp, v, f, thr, diag, st);
    case 3: return launch_nd<3, T, R>(s, batch, ed, ee, x, k, beta, rp, v, f, thr, diag, st);
    case 4: return launch_nd<4, T, R>(s, batch, ed, ee, x, k, beta, rp, v, f, thr, diag, st);
    case 5: return launch_nd<5, T, R>(s, batch, ed, ee, x, k, beta, rp, v, f, thr, diag, st);
    default: LOR_FAIL(LOR_EUNSUPPORTED, "lor_assemble_nd: p = %d not supported (the 12x12 subelement "
                                        "matrices of a macro element must fit in LDS; p <= 5)", p);
  }
}

}  // namespace lor

using namespace lor;

extern "C" int lor_assemble_nd(int p, int64_t nel, int64_t ndofs_h1, int64_t nedges, int batch,
                               const int32_t* elem_dofs, const int32_t* elem_edges, const double* coords,
                               const void* kappa, double beta, const int32_t* row_ptr, const lor_sched* sched,
                               void* values, int dtype, unsigned flags, double det_ratio_thresh, int32_t* diag,
                               void* stream) {
  clear_error();
  if (p < 1 || p > LOR_MAX_P) LOR_FAIL(LOR_EINVAL, "p = %d outside [1, %d]", p, LOR_MAX_P);
  if (nel < 0 || ndofs_h1 < 1 || nedges < 1) LOR_FAIL(LOR_EINVAL, "nel < 0, ndofs_h1 < 1 or nedges < 1");
  if (batch < 1 || batch > 65535) LOR_FAIL(LOR_EINVAL, "batch outside [1, 65535]");
  if (dtype != LOR_F64 && dtype != LOR_F32) LOR_FAIL(LOR_EINVAL, "dtype must be LOR_F64 or LOR_F32");
  if (flags & ~(LOR_FP64_FALLBACK | LOR_COLORED | LOR_OWNER)) LOR_FAIL(LOR_EINVAL, "unknown flag bits 0x%x", flags);
  if ((flags & LOR_COLORED) && (flags & LOR_OWNER)) LOR_FAIL(LOR_EINVAL, "LOR_COLORED and LOR_OWNER both set");
  if ((flags & LOR_FP64_FALLBACK) && !(det_ratio_thresh >= 1.0))
    LOR_FAIL(LOR_EINVAL, "det_ratio_thresh must be >= 1");
  if (nel > 0 && (!elem_dofs || !elem_edges || !coords || !kappa || !row_ptr || !values))
    LOR_FAIL(LOR_EINVAL, "a required pointer is NULL");
  int rc = check_sched(sched, LOR_ND, p, nel, nedges);
  if (rc) return rc;
  if (static_cast<int64_t>(batch) * sched->nnz >= (int64_t(1) << 40)) LOR_FAIL(LOR_EOVERFLOW, "batch * nnz too large");
  if (nel == 0) return LOR_OK;
  if ((flags & LOR_OWNER) && !sched->owner)
    LOR_FAIL(LOR_EUNSUPPORTED, "LOR_OWNER: the edge map is no edge lattice (no owner-computes schedule)");
  hipStream_t st = as_stream(stream);
  // default: owner-computes wherever the schedule has it (also at p = 6,
  // which the coloured kernel does not take)
  const bool owner = sched->owner && !(flags & LOR_COLORED);
  const unsigned fb = flags & LOR_FP64_FALLBACK;
  if (dtype == LOR_F64)
    return owner ? dispatch_nd_owner<double, double>(p, sched, batch, elem_dofs, elem_edges, coords, kappa, beta,
                                                     row_ptr, values, 0u, det_ratio_thresh, diag, st)
                 : dispatch_nd<double, double>(p, sched, batch, elem_dofs, elem_edges, coords, kappa, beta, row_ptr,
                                               values, 0u, det_ratio_thresh, diag, st);
  return owner ? dispatch_nd_owner<float, float>(p, sched, batch, elem_dofs, elem_edges, coords, kappa, beta, row_ptr,
                                                 values, fb, det_ratio_thresh, diag, st)
               : dispatch_nd<float, float>(p, sched, batch, elem_dofs, elem_edges, coords, kappa, beta, row_ptr,
                                           values, fb, det_ratio_thresh, diag, st);
}
