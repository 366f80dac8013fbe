// Values of the LOR H1 matrix (Step S1.2, A1 + A2 fused).
//
// The paper assembles each macro element's sparse block in global memory with
// one thread per subelement and atomic additions, then scatters the blocks
// into CSR.  Here the block never leaves the chip.  A workgroup walks a chunk
// of macro elements of one colour (E elements at a time, "group"), and for
// every group:
//
//   stage    the vertex coordinates, row pointers and rank table of the group,
//            prefetched into registers while the previous group was computed,
//            are written to LDS; the loads for the next group are issued
//            (software pipelining: the gather latency hides behind the
//            arithmetic);
//   phase 1  one lane per subelement integrates its 8x8 matrix (36 unique
//            entries, sum-factorised 2x2x2 Gauss) into LDS;
//   phase 2  one lane per local vertex (row) sums the rows of the <= 8
//            subelements around it in a fixed order (atomic-free, FP64 sums,
//            bitwise symmetric) and writes the finished row into LDS in the
//            compact local-stencil order;
//   phase 3  lanes walk the compact entries and store them at
//            row_ptr[row] + position-in-row: a plain store for the entry's
//            first contributor, an add to the stored value for the others.
//            All loads of the phase are issued before any store.
// Colours run as separate launches in increasing order, so every entry's
// contributions are summed in the same order (deterministic).
#include "lor_common.hpp"
#include "lor_h1_math.hpp"

namespace lor {

template <int P>
struct H1Cfg {
  static constexpr int Q = P + 1;
  static constexpr int NSUB = P * P * P;
  static constexpr int NLOC = Q * Q * Q;
  static constexpr int T1 = 3 * P + 1;             // stencil entries per axis
  static constexpr int NENT = T1 * T1 * T1;        // local stencil entries per element
  static constexpr int NENTP = (NENT + 15) / 16 * 16;  // table stride in bytes
  // elements per group: 256 lanes cover the subelements and every lane owns
  // at most two local rows
  static constexpr int E = P == 1 ? 64 : P == 2 ? 16 : P == 3 ? 8 : P == 4 ? 4 : P == 5 ? 2 : 1;
  static constexpr int THREADS = 256;
  static constexpr int RV = (E * NLOC + THREADS - 1) / THREADS;         // vertex slots per lane
  static constexpr int TW = E * NENTP / 4;                             // table words per group
  static constexpr int RW = (TW + THREADS - 1) / THREADS;              // table words per lane
  static constexpr int NJ = (E * NENT + THREADS - 1) / THREADS;        // phase-3 entries per lane
  static constexpr int MAXCHUNK = 256;                                 // elements per workgroup
  static_assert(RV <= 2, "two rows per lane");
  static_assert(E * NSUB <= THREADS, "one subelement per lane");
  static_assert(NJ <= 64, "phase-3 mask");
};

// Resident workgroups per CU: as many as the LDS of one workgroup allows, up
// to two in FP64 (the integration needs ~250 VGPRs per lane) and three in
// FP32 (168 VGPRs per lane; the spills this costs are cheaper than the
// latency a third workgroup hides).
template <int P, typename R>
struct H1Occ {
  using C = H1Cfg<P>;
  static constexpr int SUBW = C::E * C::NSUB * 36;
  static constexpr int STGW = C::E * C::NENT;
  static constexpr int LDS = C::E * C::NLOC * 28 + C::E * C::NENTP +
                             (SUBW > STGW ? SUBW : STGW) * static_cast<int>(sizeof(R)) + 2 * C::MAXCHUNK * 4;
  static constexpr int WANT = sizeof(R) == 8 ? 2 : 3;
  static constexpr int FIT = 160 * 1024 / LDS;
  static constexpr int WPC = WANT < FIT ? WANT : (FIT > 0 ? FIT : 1);
};

// number of stencil offsets along one axis at lattice coordinate t, and the
// prefix sum of that count over coordinates < t
template <int P>
__device__ __forceinline__ int cnt1(int t) {
  return (t == 0 || t == P) ? 2 : 3;
}
template <int P>
__device__ __forceinline__ int pre1(int t) {
  return t == 0 ? 0 : 3 * t - 1;
}

// FP32 form, strongly curved subelement: FP64 geometry and quadrature, entries
// rounded to FP32.
template <int NSUB>
__device__ __forceinline__ bool h1_fp64_fallback(const double (&X)[8][3], double kap, double bet, float* out) {
  double dx[2][2][3], dy[2][2][3], dz[2][2][3];
  h1_edges<double>(X, dx, dy, dz);
  H1Factors<double> F;
  const bool ok = h1_factors<double>(dx, dy, dz, kap, bet, F);
#pragma unroll
  for (int u = 0; u < 8; ++u)
#pragma unroll
    for (int v = u; v < 8; ++v) out[pair_index(u, v) * NSUB] = static_cast<float>(h1_entry<double>(F, u, v));
  return ok;
}

template <int P, typename T, typename R>
__global__ __launch_bounds__(256, (H1Occ<P, R>::WPC)) void k_h1_assemble(
    const int32_t* __restrict__ order, const int32_t* __restrict__ order_class, int32_t ncol, int32_t chunk,
    const int32_t* __restrict__ elem_dofs,
    const double* __restrict__ coords, const T* __restrict__ kappa, T beta, const int32_t* __restrict__ row_ptr,
    const uint8_t* __restrict__ tables, int64_t tab_stride, const uint16_t* __restrict__ ent_row, int64_t nel,
    int64_t nnz, T* __restrict__ values, const T* __restrict__ zero, unsigned flags, R det_thresh,
    int32_t* __restrict__ diag) {
  using C = H1Cfg<P>;
  constexpr int Q = C::Q, NSUB = C::NSUB, NLOC = C::NLOC, NENT = C::NENT, NENTP = C::NENTP, E = C::E;
  constexpr int TH = C::THREADS, RV = C::RV, RW = C::RW, NJ = C::NJ, TWE = NENTP / 4;
  constexpr int SUBW = E * NSUB * 36;  // subelement entries, layout [E][36][NSUB]
  constexpr int STGW = E * NENT;       // finished local entries, [E][NENT]
  constexpr int REGW = SUBW > STGW ? SUBW : STGW;
  __shared__ double sX[E * NLOC * 3];
  __shared__ int32_t sRp[E * NLOC];
  __shared__ uint32_t sTabW[E * TWE];
  __shared__ R sSub[REGW];
  __shared__ int32_t sOrd[C::MAXCHUNK];
  __shared__ int32_t sCls[C::MAXCHUNK];
  T* sStg = reinterpret_cast<T*>(sSub);
  const uint8_t* sTab = reinterpret_cast<const uint8_t*>(sTabW);
  static_assert(sizeof(T) <= sizeof(R), "staging aliases the subelement region");

  const int tid = threadIdx.x;
  kappa += static_cast<int64_t>(blockIdx.y) * nel * NSUB;
  values += static_cast<int64_t>(blockIdx.y) * nnz;
  const int64_t cbeg = static_cast<int64_t>(blockIdx.x) * chunk;
  const int nce = static_cast<int>(ncol - cbeg < chunk ? ncol - cbeg : chunk);
  const int ngr = (nce + E - 1) / E;
  if (tid < nce) {
    sOrd[tid] = order[cbeg + tid];
    sCls[tid] = order_class[cbeg + tid];
  }
  __syncthreads();

  if (ngr == 0) return;
  auto group_size = [&](int g) { return nce - g * E < E ? nce - g * E : E; };
  // --- prefetch helpers (registers) ----------------------------------------
  // Every load is issued unconditionally: indices past the group, and groups
  // past the last, are clamped to valid ones whose values are never used.  A
  // register reset before a masked load, or a loaded value copied to another
  // register, makes the compiler wait for the load right there.
  auto load_dofs = [&](int g, int32_t (&d)[RV]) {
    const int gc = g < ngr ? g : ngr - 1;
    const int n = group_size(gc);
#pragma unroll
    for (int j = 0; j < RV; ++j) {
      const int i = tid + j * TH;
      const int i2 = i < n * NLOC ? i : 0;
      const int el = i2 / NLOC;
      d[j] = elem_dofs[static_cast<int64_t>(sOrd[gc * E + el]) * NLOC + (i2 - el * NLOC)];
    }
  };
  auto load_geo = [&](const int32_t (&d)[RV], double (&x)[RV][3], int32_t (&rp)[RV]) {
#pragma unroll
    for (int j = 0; j < RV; ++j) {
      const int64_t g3 = 3 * static_cast<int64_t>(d[j]);
      x[j][0] = coords[g3 + 0];
      x[j][1] = coords[g3 + 1];
      x[j][2] = coords[g3 + 2];
      rp[j] = row_ptr[d[j]];
    }
  };
  auto load_kap = [&](int g) {
    const int gc = g < ngr ? g : ngr - 1;
    const int t2 = tid < group_size(gc) * NSUB ? tid : 0;
    const int el = t2 / NSUB;
    return kappa[static_cast<int64_t>(sOrd[gc * E + el]) * NSUB + (t2 - el * NSUB)];
  };
  auto load_tab = [&](int g, uint32_t (&w)[RW]) {
    if constexpr (E == 1) {
      const uint32_t* row = reinterpret_cast<const uint32_t*>(tables + sCls[g] * tab_stride);
#pragma unroll
      for (int j = 0; j < RW; ++j) {
        const uint32_t i = static_cast<uint32_t>(threadIdx.x) + j * TH;
        w[j] = row[i < static_cast<uint32_t>(TWE) ? i : 0u];
      }
    } else {
#pragma unroll
      for (int j = 0; j < RW; ++j) {
        const int i = tid + j * TH;
        const int i2 = i < group_size(g) * TWE ? i : 0;
        const int el = i2 / TWE;
        const uint32_t* row = reinterpret_cast<const uint32_t*>(tables + sCls[g * E + el] * tab_stride);
        w[j] = row[i2 - el * TWE];
      }
    }
  };

  // Pipeline, in place: the geometry of group g is staged from registers at
  // the start of its step, then the registers receive group g + 1's (from the
  // element-map words loaded one step earlier), and the map words of g + 2;
  // the coefficient of group g is used by its integration, after which the
  // same register receives group g + 1's.
  int32_t dnext[RV];
  double xq[RV][3];
  int32_t rq[RV];
  T kq;
  {
    int32_t d0[RV];
    load_dofs(0, d0);
    load_geo(d0, xq, rq);
    load_dofs(1, dnext);
    kq = load_kap(0);
  }

  for (int g = 0; g < ngr; ++g) {
    const int ne = E == 1 ? 1 : group_size(g);
    // Index arithmetic below is cheap; an opaque copy of the lane id keeps the
    // compiler from hoisting it out of the loop into long-lived registers.
    int tid = threadIdx.x;
    __asm__ volatile("" : "+v"(tid));
    __builtin_assume(tid >= 0 && tid < TH);
    lds_barrier();  // the previous group is done with every LDS buffer
#pragma unroll
    for (int j = 0; j < RV; ++j) {
      const int i = tid + j * TH;
      if (i < ne * NLOC) {
        sX[3 * i + 0] = xq[j][0];
        sX[3 * i + 1] = xq[j][1];
        sX[3 * i + 2] = xq[j][2];
        sRp[i] = rq[j];
      }
    }
    // prefetch the next group; the loads complete while this group is computed
    load_geo(dnext, xq, rq);
    load_dofs(g + 2, dnext);
    lds_barrier();

    // phase 1: subelement matrices
    if (tid < ne * NSUB) {
      const int el = tid / NSUB;
      const int s = tid - el * NSUB;
      const int si = s % P, sj = (s / P) % P, sk = s / (P * P);
      auto load_X = [&](double (&X)[8][3]) {
#pragma unroll
        for (int v = 0; v < 8; ++v) {
          const int lv = (si + (v & 1)) + Q * ((sj + ((v >> 1) & 1)) + Q * (sk + (v >> 2)));
#pragma unroll
          for (int d = 0; d < 3; ++d) X[v][d] = sX[3 * (el * NLOC + lv) + d];
        }
      };
      const R kap = static_cast<R>(kq);
      R* out = sSub + el * 36 * NSUB + s;
      bool fallback = false;
      if constexpr (!std::is_same<R, double>::value) {
        if (flags & LOR_FP64_FALLBACK) {
          // corner-Jacobian test; the edge vectors are formed again below so
          // that they are not kept alive across the FP64 branch
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
        const bool ok = h1_factors<R>(ex, ey, ez, kap, static_cast<R>(beta), F);
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
          for (int v = u; v < 8; ++v) out[pair_index(u, v) * NSUB] = h1_entry<R>(F, u, v);
        if (!ok && diag) atomicAdd(&diag[1], 1);
      }
      if (fallback) {
        // FP32 form on a strongly curved subelement: FP64 geometry and
        // quadrature from the FP64 coordinates, entries rounded to FP32
        double X[8][3];
        load_X(X);
        const bool ok = h1_fp64_fallback<NSUB>(X, static_cast<double>(kap), static_cast<double>(beta),
                                               reinterpret_cast<float*>(out));
        if (diag) {
          atomicAdd(&diag[0], 1);
          if (!ok) atomicAdd(&diag[1], 1);
        }
      }
    }
    kq = load_kap(g + 1);  // the next group's coefficient, after this group's last use
    lds_barrier();

    // phase 2: local rows.  Lane owns rows tid and tid + 256.  The rank table
    // of the group is fetched meanwhile (needed in phase 3 only).
    uint32_t twq[RW];
    load_tab(g, twq);
    double acc[2][27];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
#pragma unroll
      for (int o = 0; o < 27; ++o) acc[h][o] = 0.0;
      const int r = tid + h * TH;
      if (r < ne * NLOC) {
        const int el = r / NLOC;
        const int l = r - el * NLOC;
        const int x = l % Q, y = (l / Q) % Q, z = l / (Q * Q);
        const R* base = sSub + el * 36 * NSUB;
        // corner u of the subelement s = (x,y,z) - u; s decreases as u grows
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int a = u & 1, bb = (u >> 1) & 1, c = u >> 2;
          const int sx = x - a, sy = y - bb, sz = z - c;
          if (sx >= 0 && sx < P && sy >= 0 && sy < P && sz >= 0 && sz < P) {
            const int s = sx + P * (sy + P * sz);
#pragma unroll
            for (int v = 0; v < 8; ++v) {
              const int o = ((v & 1) - a + 1) + 3 * ((((v >> 1) & 1) - bb + 1) + 3 * ((v >> 2) - c + 1));
              acc[h][o] += static_cast<double>(base[pair_index(u, v) * NSUB + s]);
            }
          }
        }
      }
    }
    lds_barrier();  // every lane has read sSub; now it becomes the staging area
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int r = tid + h * TH;
      if (r < ne * NLOC) {
        const int el = r / NLOC;
        const int l = r - el * NLOC;
        const int x = l % Q, y = (l / Q) % Q, z = l / (Q * Q);
        const int nx = cnt1<P>(x), ny = cnt1<P>(y), nxy = nx * ny;
        const int rbase = pre1<P>(z) * C::T1 * C::T1 + cnt1<P>(z) * pre1<P>(y) * C::T1 + cnt1<P>(z) * ny * pre1<P>(x);
        const int x0 = x > 0 ? 1 : 0, y0 = y > 0 ? 1 : 0, z0 = z > 0 ? 1 : 0;
        // entry (dx, dy, dz) of the row sits at c + dz * nxy + dy * nx + dx
        T* c = sStg + el * NENT + rbase + z0 * nxy + y0 * nx + x0;
        const bool vx[3] = {x > 0, true, x < P}, vy[3] = {y > 0, true, y < P}, vz[3] = {z > 0, true, z < P};
#pragma unroll
        for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
          for (int dy = -1; dy <= 1; ++dy) {
            T* line = c + dz * nxy + dy * nx;
            const bool vzy = vz[dz + 1] && vy[dy + 1];
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx)
              if (vzy && vx[dx + 1]) line[dx] = static_cast<T>(acc[h][(dx + 1) + 3 * (dy + 1) + 9 * (dz + 1)]);
          }
      }
    }
#pragma unroll
    for (int j = 0; j < RW; ++j) {
      const int i = tid + j * TH;
      if (i < ne * TWE) sTabW[i] = twq[j];
    }
    lds_barrier();

    // phase 3: store into the CSR values.  Every load is issued before any
    // store and the memory instructions sit in straight-line code (no branch
    // per entry), so each store waits only for its own operand.  A first
    // contributor reads its "old value" from a zero slot (one shared cache
    // line) instead of taking a branch; lanes past the end of the group
    // repeat their first store.
    if (tid < ne * NENT) {
      const uint32_t ut = static_cast<uint32_t>(tid);
      uint32_t erow[NJ];
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        const uint32_t i = ut + j * TH;
        const bool ok = i < static_cast<uint32_t>(ne * NENT);
        const uint32_t el = E == 1 ? 0u : i / NENT;
        erow[j] = ent_row[ok ? i - el * NENT : 0u];
      }
      uint32_t pos[NJ];
      T old[NJ];
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        const uint32_t i = ut + j * TH;
        const bool ok = i < static_cast<uint32_t>(ne * NENT);
        const uint32_t el = ok ? (E == 1 ? 0u : i / NENT) : 0u;
        const uint32_t k = ok ? i - el * NENT : 0u;
        const uint32_t t = sTab[el * NENTP + k];
        pos[j] = static_cast<uint32_t>(sRp[el * NLOC + erow[j]]) + (t & kRankMask);
        old[j] = *((t & kFirstBit) ? zero : values + pos[j]);
      }
      // non-temporal stores: the values are not re-read by this launch (later
      // colours read them back after the kernel boundary), and marking them
      // streaming measured about 4% faster in FP64
      const T v0 = sStg[ut] + old[0];
      __builtin_nontemporal_store(v0, values + pos[0]);
#pragma unroll
      for (int j = 1; j < NJ; ++j) {
        const uint32_t i = ut + j * TH;
        const bool ok = i < static_cast<uint32_t>(ne * NENT);
        const T v = sStg[ok ? i : ut] + old[j];
        __builtin_nontemporal_store(ok ? v : v0, values + (ok ? pos[j] : pos[0]));
      }
    }
  }
}

static int num_cus() {
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
static int launch_h1(const lor_sched* sched, int batch, const int32_t* elem_dofs, const double* coords,
                     const void* kappa, double beta, const int32_t* row_ptr, void* values, unsigned flags,
                     double thr, int32_t* diag, hipStream_t st) {
  using C = H1Cfg<P>;
  if (sched->tab_stride != C::NENTP || sched->nent != C::NENT)
    LOR_FAIL(LOR_EINVAL, "schedule tables do not match p = %d", P);
  const int32_t* order = dev_at<int32_t>(sched, sched->off_order);
  const int32_t* ocls = dev_at<int32_t>(sched, sched->off_order_class);
  const uint8_t* tab = dev_at<uint8_t>(sched, sched->off_tables);
  const uint16_t* ent_row = dev_at<uint16_t>(sched, sched->off_ent_row);
  const int wgs = H1Occ<P, R>::WPC * num_cus();  // resident workgroups
  for (int c = 0; c < sched->ncolors; ++c) {
    const int32_t n = sched->color_ptr[c + 1] - sched->color_ptr[c];
    if (n <= 0) continue;
    const int64_t groups = ceil_div(n, C::E);
    int64_t gpw = ceil_div(groups, wgs);  // groups per workgroup
    if (gpw * C::E > C::MAXCHUNK) gpw = C::MAXCHUNK / C::E;
    const int32_t chunk = static_cast<int32_t>(gpw * C::E);
    dim3 grid(static_cast<unsigned>(ceil_div(n, chunk)), static_cast<unsigned>(batch));
    k_h1_assemble<P, T, R><<<grid, C::THREADS, 0, st>>>(
        order + sched->color_ptr[c], ocls + sched->color_ptr[c], n, chunk, elem_dofs, coords, static_cast<const T*>(kappa), static_cast<T>(beta),
        row_ptr, tab, sched->tab_stride, ent_row, sched->nel, sched->nnz, static_cast<T*>(values),
        dev_at<T>(sched, sched->off_zero), flags, static_cast<R>(thr), diag);
    LOR_LAUNCHED("k_h1_assemble");
  }
  return LOR_OK;
}

template <typename T, typename R>
static int dispatch_h1(int p, const lor_sched* s, int batch, const int32_t* ed, const double* x, const void* k,
                       double beta, const int32_t* rp, void* v, unsigned f, double thr, int32_t* diag,
                       hipStream_t st) {
  switch (p) {
    case 1: return launch_h1<1, T, R>(s, batch, ed, x, k, beta, rp, v, f, thr, diag, st);
    case 2: return launch_h1<2, T, R>(s, batch, ed, x, k, beta, rp, v, f, thr, diag, st);
    case 3: return launch_h1<3, T, R>(s, batch, ed, x, k, beta, rp, v, f, thr, diag, st);
    case 4: return launch_h1<4, T, R>(s, batch, ed, x, k, beta, rp, v, f, thr, diag, st);
    case 5: return launch_h1<5, T, R>(s, batch, ed, x, k, beta, rp, v, f, thr, diag, st);
    case 6: return launch_h1<6, T, R>(s, batch, ed, x, k, beta, rp, v, f, thr, diag, st);
    default: LOR_FAIL(LOR_EUNSUPPORTED, "p = %d not compiled", p);
  }
}

template <typename T, typename R>
int dispatch_owner(int p, const lor_sched* s, int batch, const int32_t* ed, const double* x, const void* k,
                   double beta, const int32_t* rp, void* v, unsigned f, double thr, int32_t* diag, hipStream_t st);
bool owner_fits(const lor_sched* s, int tsize);

// Shared argument checks of the value calls.
int check_sched(const lor_sched* s, int space, int p, int64_t nel, int64_t nrows) {
  if (!s) LOR_FAIL(LOR_EINVAL, "sched is NULL");
  if (!s->dev) LOR_FAIL(LOR_EINVAL, "sched->dev is NULL (run lor_pattern phase 2 first)");
  if (s->space != space) LOR_FAIL(LOR_EINVAL, "sched was built for another space");
  if (s->p != p || s->nel != nel || s->nrows != nrows)
    LOR_FAIL(LOR_EINVAL, "sched (p=%d nel=%lld nrows=%lld) does not match the call (p=%d nel=%lld nrows=%lld)",
             s->p, (long long)s->nel, (long long)s->nrows, p, (long long)nel, (long long)nrows);
  if (s->ncolors < 0 || s->ncolors > LOR_MAX_COLORS) LOR_FAIL(LOR_EINVAL, "sched->ncolors out of range");
  if (s->color_ptr[s->ncolors] != nel) LOR_FAIL(LOR_EINVAL, "sched colour table does not cover the elements");
  return LOR_OK;
}

}  // namespace lor

using namespace lor;

extern "C" int lor_assemble_h1(int p, int64_t nel, int64_t ndofs, int batch, const int32_t* elem_dofs,
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
  int rc = check_sched(sched, LOR_H1, p, nel, ndofs);
  if (rc) return rc;
  if (static_cast<int64_t>(batch) * sched->nnz >= (int64_t(1) << 40)) LOR_FAIL(LOR_EOVERFLOW, "batch * nnz too large");
  if (nel == 0) return LOR_OK;
  if ((flags & LOR_OWNER) && !sched->owner)
    LOR_FAIL(LOR_EUNSUPPORTED, "LOR_OWNER: the mesh has no owner-computes schedule (its element lattices do not "
                               "continue across faces in one orientation, or a row is not a full lattice stencil)");
  hipStream_t st = as_stream(stream);
  // default: owner-computes wherever the schedule has it (faster in both
  // forms) and its buffer ranges allow
  const bool owner = sched->owner && !(flags & LOR_COLORED) &&
                     ((flags & LOR_OWNER) || owner_fits(sched, dtype == LOR_F64 ? 8 : 4));
  const unsigned fb = flags & LOR_FP64_FALLBACK;
  if (dtype == LOR_F64)
    return owner ? dispatch_owner<double, double>(p, sched, batch, elem_dofs, coords, kappa, beta, row_ptr, values,
                                                  0u, det_ratio_thresh, diag, st)
                 : dispatch_h1<double, double>(p, sched, batch, elem_dofs, coords, kappa, beta, row_ptr, values, 0u,
                                               det_ratio_thresh, diag, st);
  return owner ? dispatch_owner<float, float>(p, sched, batch, elem_dofs, coords, kappa, beta, row_ptr, values, fb,
                                              det_ratio_thresh, diag, st)
               : dispatch_h1<float, float>(p, sched, batch, elem_dofs, coords, kappa, beta, row_ptr, values, fb,
                                           det_ratio_thresh, diag, st);
}
