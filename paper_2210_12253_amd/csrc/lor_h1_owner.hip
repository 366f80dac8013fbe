// Values of the LOR H1 matrix, owner-computes form (Step S1.2, A1 + A2 fused,
// every row summed once, on the chip, and stored once, whole).
//
// The coloured kernel (lor_h1.hip) lets every element add into the rows it
// touches, so the rows on element faces are written piecewise by up to eight
// launches.  This kernel works on the global lattice of a box-shaped mesh
// instead (the pattern call checks that the mesh is one: lattice point
// (X, Y, Z) has vertex id base(Y, Z) + X, cell (X, Y, Z) belongs to element
// elem3d(X / p, Y / p, Z / p) at local subelement (X % p, Y % p, Z % p)):
//
//   * one wave = one worker, no workgroup barriers.  It takes a tile of 8 x 8
//     cells in x and y (tiles overlap by one cell layer, stride 7) and marches
//     along z over a segment of cell layers, one layer per step;
//   * each lane integrates one cell of the layer (one Q1 cell matrix, 36
//     unique entries) into the wave's LDS slab;
//   * the rows of the layer's lower lattice plane are finished in registers:
//     lane (x, y) sums, for row (x0 + x, y0 + y), the cells at the four
//     lanes (x - a, y - b), corners c = 1 (the layer below, carried in
//     registers from the previous step) before c = 0; the c = 1 corners of
//     this layer are the carry into the next plane.  Rows x, y in [1, 7] of a
//     tile are its own (also 0 on the box's lower faces), so the last cell
//     column and row of a tile are integrated twice (by this tile and its
//     neighbour): 64 cells per 49 rows;
//   * the finished rows of each x-line are consecutive rows of the matrix;
//     they are staged in LDS and stored as one contiguous span per line;
//   * a segment that starts above the bottom first integrates the layer below
//     it to build the carry; the topmost segment ends with the top plane,
//     whose rows only hold the carry.
//
// Every entry (i, j) is summed over the cells holding both vertices in one
// fixed order of the cell's corner at i (c = 1 before c = 0, then b, a); a
// cell holding i and j has the same corner at i and at j along every axis
// where i and j agree, so (j, i) takes the same cells in the same order, and
// a cell integrated by two tiles gives the same bits in both (same inputs,
// same code).  The matrix is therefore bitwise symmetric and deterministic.
// All sums are FP64, in the FP32 form too (each finished entry is rounded
// once).
#include <algorithm>

#include "lor_common.hpp"
#include "lor_h1_math.hpp"

namespace lor {

constexpr int kOwnTile = 8;                  // cells per tile side (one wave: 8 x 8)
constexpr int kOwnStride = kOwnTile - 1;     // tiles overlap by one cell
constexpr int kOwnPts = (kOwnTile + 1) * (kOwnTile + 1);  // lattice points of one tile plane

// Layers integrated per step and LDS slab of one wave.  The FP64 form runs
// one wave per SIMD: its integration wants ~250 VGPRs, and with the carry a
// second wave per SIMD spills (measured at the headline size: 1.10 ms at one
// wave, 1.28 ms at two with spills, 1.14 ms at two with the carry in LDS,
// 1.18 ms with two cells per lane and step).  The FP32 form runs two waves
// per SIMD.  LPS > 1 (several layers per lane and step) is supported but not
// used.
template <typename T, typename R>
struct OwnCfg {
  static constexpr int LPS = 1;                        // layers per step
  static constexpr int NPL = LPS + 1;                 // lattice planes in LDS (ring)
  static constexpr int WPE = sizeof(R) == 8 ? 1 : 2;  // waves per SIMD (second __launch_bounds__ argument)
  // cell matrices [pair][lane]; once the row sums have read them, the finished
  // rows of the plane staged per x-line
  static constexpr int CELLS = 36 * 64 * static_cast<int>(sizeof(R));
  static constexpr int ROWS = 64 * 27 * static_cast<int>(sizeof(T));
  static constexpr int SLAB = CELLS > ROWS ? CELLS : ROWS;
};

// FP32 form, strongly curved cell: FP64 geometry and quadrature from the FP64
// corner coordinates, entries rounded to FP32 (64 = distance between two
// entries of a cell in the slab).  Kept out of line: the branch is rare, and
// inlined its FP64 registers would be reserved for the whole kernel.
__device__ __noinline__ bool own_fp64_fallback(const double* __restrict__ pz0, const double* __restrict__ pz1,
                                               int lx, int ly, double kap, double bet, float* out) {
  double X[8][3];
#pragma unroll
  for (int v = 0; v < 8; ++v) {
    const double* pl = (v >> 2) ? pz1 : pz0;
    const int pidx = (lx + (v & 1)) + (kOwnTile + 1) * (ly + ((v >> 1) & 1));
#pragma unroll
    for (int d = 0; d < 3; ++d) X[v][d] = pl[3 * pidx + d];
  }
  double dx[2][2][3], dy[2][2][3], dz[2][2][3];
  h1_edges<double>(X, dx, dy, dz);
  H1Factors<double> F;
  const bool ok = h1_factors<double>(dx, dy, dz, kap, bet, F);
#pragma unroll
  for (int u = 0; u < 8; ++u)
#pragma unroll
    for (int v = u; v < 8; ++v) out[pair_index(u, v) * 64] = static_cast<float>(h1_entry<double>(F, u, v));
  return ok;
}

// Offset index (dx + 1) + 3 (dy + 1) + 9 (dz + 1) of the entry from corner u
// to corner v of a cell.
__host__ __device__ constexpr int own_off(int u, int v) {
  return ((v & 1) - (u & 1) + 1) + 3 * (((v >> 1) & 1) - ((u >> 1) & 1) + 1) + 9 * ((v >> 2) - (u >> 2) + 1);
}

template <int P, typename T, typename R>
__global__ __launch_bounds__(64, (OwnCfg<T, R>::WPE)) void k_h1_owner(
    int nex, int ney, int nez, int ntx, int seglen, const int32_t* __restrict__ elem3d,
    const int32_t* __restrict__ base, const double* __restrict__ coords, const T* __restrict__ kappa, T beta,
    const int32_t* __restrict__ row_ptr, int64_t nel, int64_t nnz, T* __restrict__ values, unsigned flags,
    R det_thresh, int32_t* __restrict__ diag) {
  using C = OwnCfg<T, R>;
  constexpr int NSUB = P * P * P, LPS = C::LPS, NPL = C::NPL;
  __shared__ __align__(16) unsigned char sSlab[C::SLAB];
  __shared__ double sPt[NPL][kOwnPts * 3];  // lattice planes, ring buffer indexed by Z % NPL
  __shared__ int32_t sRp[64];               // row pointers of the tile's rows in the plane being stored
  R* const sCell = reinterpret_cast<R*>(sSlab);
  T* const sStg = reinterpret_cast<T*>(sSlab);

  const int NXc = nex * P, NYc = ney * P, NZc = nez * P;  // cells per axis
  const int LY = NYc + 1;                                   // lattice points per plane along y
  const int lane = threadIdx.x;
  const int ti = blockIdx.x % ntx, tj = blockIdx.x / ntx;
  const int x0 = kOwnStride * ti, y0 = kOwnStride * tj;
  const int zs = blockIdx.y * seglen;
  const int ze = zs + seglen < NZc ? zs + seglen : NZc;
  kappa += static_cast<int64_t>(blockIdx.z) * nel * NSUB;
  values += static_cast<int64_t>(blockIdx.z) * nnz;

  const int lx = lane & 7, ly = lane >> 3;
  const int cX = x0 + lx, cY = y0 + ly;                // this lane's cell / row column (x, y)
  const bool cell_in = cX < NXc && cY < NYc;
  const bool row_in = cX <= NXc && cY <= NYc;           // row (cX, cY) exists in every plane
  const bool row_own = row_in && (lx > 0 || ti == 0) && (ly > 0 || tj == 0);
  // lattice points of a plane: slot j -> point lane + 64 j of the 9 x 9 grid
  auto pt_xy = [&](int j, int& X, int& Y) {
    const int pidx = lane + 64 * j;
    X = x0 + pidx % (kOwnTile + 1);
    Y = y0 + pidx / (kOwnTile + 1);
    return pidx < kOwnPts && X <= NXc && Y <= NYc;
  };
  // vertex ids of plane Z (-1 where absent)
  auto load_vid = [&](int Z, int32_t (&v)[2]) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      int X, Y;
      v[j] = -1;
      if (Z <= NZc && pt_xy(j, X, Y)) v[j] = base[static_cast<int64_t>(Z) * LY + Y] + X;
    }
  };
  auto load_xyz = [&](const int32_t (&v)[2], double (&xq)[2][3]) {
#pragma unroll
    for (int j = 0; j < 2; ++j)
      if (v[j] >= 0) {
        const int64_t g = 3 * static_cast<int64_t>(v[j]);
        xq[j][0] = coords[g + 0];
        xq[j][1] = coords[g + 1];
        xq[j][2] = coords[g + 2];
      }
  };
  // element of this lane's cell in layer Z (-1 where absent)
  auto load_elem = [&](int Z, int32_t& el) {
    el = -1;
    if (cell_in && Z < NZc) el = elem3d[(static_cast<int64_t>(Z / P) * ney + cY / P) * nex + cX / P];
  };
  auto load_kap = [&](int Z, int32_t el, T& k) {
    k = T(0);
    if (el >= 0) k = kappa[static_cast<int64_t>(el) * NSUB + (cX % P) + P * ((cY % P) + P * (Z % P))];
  };
  auto load_rp = [&](int Z, int32_t& rp) {
    rp = 0;
    if (row_in && Z <= NZc) rp = row_ptr[base[static_cast<int64_t>(Z) * LY + cY] + cX];
  };
  auto stage_plane = [&](int Z, const int32_t (&v)[2], const double (&xq)[2][3]) {
    double* pl = sPt[Z % NPL];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int pidx = lane + 64 * j;
      if (pidx < kOwnPts && v[j] >= 0) {
        pl[3 * pidx + 0] = xq[j][0];
        pl[3 * pidx + 1] = xq[j][1];
        pl[3 * pidx + 2] = xq[j][2];
      }
    }
  };

  const int zfirst = zs > 0 ? zs - 1 : zs;  // a segment above the bottom starts one layer lower
  // the segment writes planes zs .. ze - 1; the last one also writes the top
  // plane NZc, whose rows only hold the carry
  const int zend = ze == NZc ? NZc + 1 : ze;

  // Software pipeline, per step of LPS layers from Z: planes Z + 1 .. Z + LPS
  // are staged from registers, and loads for the next step are issued
  // (coordinates of its planes, vertex ids one step further, coefficients of
  // its layers, elements one step further, row pointers of its planes).
  int32_t vq[LPS][2], vnext[LPS][2];
  double xq[LPS][2][3] = {};
  int32_t elq[LPS], elnext[LPS], rpq[LPS];
  T kq[LPS];
  {
    int32_t v0[2];
    double xp[2][3] = {};
    load_vid(zfirst, v0);
    load_xyz(v0, xp);
    stage_plane(zfirst, v0, xp);
#pragma unroll
    for (int L = 0; L < LPS; ++L) {
      load_vid(zfirst + 1 + L, vq[L]);
      load_xyz(vq[L], xq[L]);
      load_vid(zfirst + 1 + LPS + L, vnext[L]);
      load_elem(zfirst + L, elq[L]);
      load_kap(zfirst + L, elq[L], kq[L]);
      load_rp(zfirst + L, rpq[L]);
      load_elem(zfirst + LPS + L, elnext[L]);
    }
  }

  double carry[18];
#pragma unroll
  for (int o = 0; o < 18; ++o) carry[o] = 0.0;

  for (int Z = zfirst; Z < zend; Z += LPS) {
#pragma unroll
    for (int L = 0; L < LPS; ++L) stage_plane(Z + 1 + L, vq[L], xq[L]);
    int32_t elcur[LPS], rpcur[LPS];
    T kcur[LPS];
#pragma unroll
    for (int L = 0; L < LPS; ++L) {
      elcur[L] = elq[L];
      kcur[L] = kq[L];
      rpcur[L] = rpq[L];
      load_xyz(vnext[L], xq[L]);
      vq[L][0] = vnext[L][0];
      vq[L][1] = vnext[L][1];
      load_vid(Z + 1 + 2 * LPS + L, vnext[L]);
      elq[L] = elnext[L];
      load_kap(Z + LPS + L, elq[L], kq[L]);
      load_elem(Z + 2 * LPS + L, elnext[L]);
      load_rp(Z + LPS + L, rpq[L]);
    }
    __builtin_amdgcn_wave_barrier();

    // the cells (cX, cY, Z + L): 36 entries each, straight into the slab for
    // one layer per step, in registers for several
    R ent[LPS > 1 ? LPS : 1][LPS > 1 ? 36 : 1];
#pragma unroll
    for (int L = 0; L < LPS; ++L) {
      const int Zl = Z + L;
      R* out = LPS > 1 ? &ent[L][0] : sCell + lane;
      constexpr int OS = LPS > 1 ? 1 : 64;  // distance between two entries of the cell
      if constexpr (LPS > 1) {
#pragma unroll
        for (int i = 0; i < 36; ++i) ent[L][i] = R(0);
      }
      if (elcur[L] < 0) continue;
      const double* pz0 = sPt[Zl % NPL];
      const double* pz1 = sPt[(Zl + 1) % NPL];
      auto load_X = [&](double (&X)[8][3]) {
#pragma unroll
        for (int v = 0; v < 8; ++v) {
          const double* pl = (v >> 2) ? pz1 : pz0;
          const int pidx = (lx + (v & 1)) + (kOwnTile + 1) * (ly + ((v >> 1) & 1));
#pragma unroll
          for (int d = 0; d < 3; ++d) X[v][d] = pl[3 * pidx + d];
        }
      };
      const R kap = static_cast<R>(kcur[L]);
      // counted once: a cell in a tile's last column (row) is also the first
      // column (row) of the next tile, which counts it
      const bool own = Zl >= zs && lx < kOwnStride && ly < kOwnStride;
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
        const bool ok = h1_factors<R>(ex, ey, ez, kap, static_cast<R>(beta), F);
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
          for (int v = u; v < 8; ++v) out[pair_index(u, v) * OS] = h1_entry<R>(F, u, v);
        if (!ok && own && diag) atomicAdd(&diag[1], 1);
      }
      if (fallback) {
        // FP32 only: computed in the slab (then read back for several layers)
        const bool ok = own_fp64_fallback(pz0, pz1, lx, ly, static_cast<double>(kap), static_cast<double>(beta),
                                          reinterpret_cast<float*>(sCell + lane));
        if constexpr (LPS > 1) {
#pragma unroll
          for (int i = 0; i < 36; ++i) ent[L][i] = sCell[i * 64 + lane];
        }
        if (own && diag) {
          atomicAdd(&diag[0], 1);
          if (!ok) atomicAdd(&diag[1], 1);
        }
      }
    }

#pragma unroll
    for (int L = 0; L < LPS; ++L) {
      const int Zl = Z + L;
      if (Zl >= zend) break;
      __builtin_amdgcn_wave_barrier();
      if constexpr (LPS > 1) {
#pragma unroll
        for (int i = 0; i < 36; ++i) sCell[i * 64 + lane] = ent[L][i];
      }
      sRp[lane] = rpcur[L];
      __builtin_amdgcn_wave_barrier();
      // row (cX, cY) of plane Zl: the carry (c = 1 corners, layer Zl - 1) +
      // this layer's c = 0 corners; this layer's c = 1 corners are the next carry
      double acc[27];
#pragma unroll
      for (int o = 0; o < 27; ++o) acc[o] = o < 18 ? carry[o] : 0.0;
#pragma unroll
      for (int o = 0; o < 18; ++o) carry[o] = 0.0;
      if (row_in && Zl < NZc) {
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
          for (int a = 0; a < 2; ++a) {
            const int sx = lx - a, sy = ly - b;
            if (sx >= 0 && sy >= 0 && x0 + sx < NXc && y0 + sy < NYc) {
              const R* cm = sCell + sx + 8 * sy;
              const int u0 = a + 2 * b, u1 = a + 2 * b + 4;
#pragma unroll
              for (int v = 0; v < 8; ++v) {
                acc[own_off(u0, v)] += static_cast<double>(cm[pair_index(u0, v) * 64]);
                carry[own_off(u1, v)] += static_cast<double>(cm[pair_index(u1, v) * 64]);
              }
            }
          }
      }
      __builtin_amdgcn_wave_barrier();
      if (Zl < zs) continue;  // the layer below the segment: carry only

      // stage the owned rows of each x-line in CSR order: a row holds
      // (x-offsets) x (y-offsets) x (z-offsets) entries, 2 per axis at a
      // lattice end and 3 elsewhere
      const int ylo = cY > 0, yhi = cY < NYc, zlo = Zl > 0, zhi = Zl < NZc;
      const int ny = 1 + ylo + yhi, nyz = ny * (1 + zlo + zhi);
      const int xfirst = ti == 0 ? 0 : 1;  // first owned row of the tile's x-lines
      if (row_own) {
        const int xlo = cX > 0, xhi = cX < NXc, nx = 1 + xlo + xhi;
        int before = 0;  // x-offset counts of the owned rows before this one in its line
        for (int x = xfirst; x < lx; ++x) before += 1 + (x0 + x > 0) + (x0 + x < NXc);
        T* row = sStg + 27 * 8 * ly + before * nyz + (zlo * ny + ylo) * nx + xlo;
#pragma unroll
        for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
          for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx) {
              const bool ok = (dx >= 0 || xlo) && (dx <= 0 || xhi) && (dy >= 0 || ylo) && (dy <= 0 || yhi) &&
                              (dz >= 0 || zlo) && (dz <= 0 || zhi);
              if (ok)
                row[dz * nx * ny + dy * nx + dx] = static_cast<T>(acc[(dx + 1) + 3 * (dy + 1) + 9 * (dz + 1)]);
            }
      }
      __builtin_amdgcn_wave_barrier();
      // one contiguous span per owned x-line
      const int xlast = x0 + 7 < NXc ? x0 + 7 : NXc;  // last owned row of the lines
      int span_x = 0;
      for (int X = x0 + xfirst; X <= xlast; ++X) span_x += 1 + (X > 0) + (X < NXc);
      for (int l = tj == 0 ? 0 : 1; l < 8; ++l) {
        const int Y = y0 + l;
        if (Y > NYc) break;
        const int span = span_x * (1 + (Y > 0) + (Y < NYc)) * (1 + zlo + zhi);
        T* dst = values + sRp[xfirst + 8 * l];
        const T* src = sStg + 27 * 8 * l;
        for (int t = lane; t < span; t += 64) __builtin_nontemporal_store(src[t], dst + t);
      }
    }
  }
}

template <int P, typename T, typename R>
static int launch_owner(const lor_sched* sched, int batch, const void* kappa, double beta, const double* coords,
                        const int32_t* row_ptr, void* values, unsigned flags, double thr, int32_t* diag,
                        hipStream_t st) {
  const int nex = sched->box[0], ney = sched->box[1], nez = sched->box[2];
  if (nex < 1 || ney < 1 || nez < 1 || static_cast<int64_t>(nex) * ney * nez != sched->nel)
    LOR_FAIL(LOR_EINVAL, "the owner-computes schedule does not describe the mesh");
  const int NXc = nex * P, NYc = ney * P, NZc = nez * P;
  const int64_t ntx = ceil_div(NXc, kOwnStride), nty = ceil_div(NYc, kOwnStride);
  const int64_t tiles = ntx * nty;
  if (tiles > INT32_MAX) LOR_FAIL(LOR_EOVERFLOW, "too many owner-computes tiles");
  // split the z-march into segments so that there are several waves per
  // SIMD slot of the chip; a segment costs one extra cell layer
  const int64_t want = 8192;
  int64_t nseg = std::min<int64_t>(NZc, std::max<int64_t>(1, ceil_div(want, tiles)));
  int64_t seglen = ceil_div(NZc, nseg);
  if (seglen < 8) seglen = std::min<int64_t>(8, NZc);
  nseg = ceil_div(NZc, seglen);
  dim3 grid(static_cast<unsigned>(tiles), static_cast<unsigned>(nseg), static_cast<unsigned>(batch));
  k_h1_owner<P, T, R><<<grid, 64, 0, st>>>(
      nex, ney, nez, static_cast<int>(ntx), static_cast<int>(seglen), dev_at<int32_t>(sched, sched->off_elem3d),
      dev_at<int32_t>(sched, sched->off_base), coords, static_cast<const T*>(kappa), static_cast<T>(beta), row_ptr,
      sched->nel, sched->nnz, static_cast<T*>(values), flags, static_cast<R>(thr), diag);
  LOR_LAUNCHED("k_h1_owner");
  return LOR_OK;
}

template <typename T, typename R>
int dispatch_owner(int p, const lor_sched* s, int batch, const int32_t* ed, const double* x, const void* k,
                   double beta, const int32_t* rp, void* v, unsigned f, double thr, int32_t* diag, hipStream_t st) {
  (void)ed;
  switch (p) {
    case 1: return launch_owner<1, T, R>(s, batch, k, beta, x, rp, v, f, thr, diag, st);
    case 2: return launch_owner<2, T, R>(s, batch, k, beta, x, rp, v, f, thr, diag, st);
    case 3: return launch_owner<3, T, R>(s, batch, k, beta, x, rp, v, f, thr, diag, st);
    case 4: return launch_owner<4, T, R>(s, batch, k, beta, x, rp, v, f, thr, diag, st);
    case 5: return launch_owner<5, T, R>(s, batch, k, beta, x, rp, v, f, thr, diag, st);
    case 6: return launch_owner<6, T, R>(s, batch, k, beta, x, rp, v, f, thr, diag, st);
    default: LOR_FAIL(LOR_EUNSUPPORTED, "p = %d not compiled", p);
  }
}

template int dispatch_owner<double, double>(int, const lor_sched*, int, const int32_t*, const double*, const void*,
                                            double, const int32_t*, void*, unsigned, double, int32_t*, hipStream_t);
template int dispatch_owner<float, float>(int, const lor_sched*, int, const int32_t*, const double*, const void*,
                                          double, const int32_t*, void*, unsigned, double, int32_t*, hipStream_t);

}  // namespace lor
