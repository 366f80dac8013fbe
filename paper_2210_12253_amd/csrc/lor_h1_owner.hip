// Values of the LOR H1 matrix, owner-computes form (Step S1.2, A1 + A2 fused,
// every row summed once, on the chip, and stored once, whole).
//
// The coloured kernel (lor_h1.hip) lets every element add into the rows it
// touches, so the rows on element faces are written piecewise by up to eight
// launches.  This kernel works on the global lattice of a box lattice instead
// (the pattern call checks that the mesh is one: lattice point (X, Y, Z) of
// the (LX, LY, LZ) points has vertex id X + LX (Y + LY Z), its row starts at
// box_row_start(X, Y, Z), and cell (X, Y, Z) belongs to element
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
//     they are staged in LDS and stored as one contiguous span per line, with
//     a fixed number of (predicated) store instructions per step: with a
//     data-dependent count the compiler cannot tell how many stores are still
//     in flight when a prefetched value is used, and waits for all of them;
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

// LDS slab of one wave and waves per SIMD.  The FP64 form runs one wave per
// SIMD: its integration wants ~250 VGPRs and the carry 36 more.  At two waves
// per SIMD it spills about 30 registers; measured at the headline size that
// was within 2% in time but wrote 15% more to HBM (the spills).  The FP32
// form runs two waves per SIMD.
template <typename T, typename R>
struct OwnCfg {
  static constexpr int LPS = 1;   // cell layers per step
  static constexpr int NPL = LPS + 1;  // lattice planes in LDS (ring)
  static constexpr int WPE = sizeof(R) == 8 ? 1 : 2;  // waves per SIMD (second __launch_bounds__ argument)
  // cell matrices [pair][lane]; once the row sums have read them, the finished
  // rows of the plane staged per x-line
  static constexpr int CELLS = 36 * 64 * static_cast<int>(sizeof(R));
  static constexpr int ROWS = 64 * 27 * static_cast<int>(sizeof(T));
  static constexpr int SLAB = CELLS > ROWS ? CELLS : ROWS;
  // one staged lattice plane (FP64 points), rounded to 16 bytes
  static constexpr int PLANE = ((kOwnTile + 1) * (kOwnTile + 1) * 3 * 8 + 15) / 16 * 16;
  // One buffer per wave: the slab at [0, SLAB), then the two planes (even Z,
  // odd Z).
  static constexpr int LDS = SLAB + 2 * PLANE;  // bytes per wave
  // resident waves per CU: registers allow 4 WPE, LDS (160 KB) may allow fewer
  static constexpr int WPC = 4 * WPE < 160 * 1024 / LDS ? 4 * WPE : 160 * 1024 / LDS;
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

// Whether term v of cell k = a + 2 b (in the order b, a of the row sums;
// lower corner k, or upper corner k + 4 if up) is the first term of its
// offset.  Such a term is assigned instead of added to 0 (which is not a
// no-op in IEEE arithmetic, so the compiler keeps it), except for the row
// entries below the carry's 18, which start from the carry.
__host__ __device__ constexpr bool own_first(int k, int v, int up) {
  const int o = own_off(k + 4 * up, v);
  for (int k2 = 0; k2 < k; ++k2)
    for (int v2 = 0; v2 < 8; ++v2)
      if (own_off(k2 + 4 * up, v2) == o) return false;
  return up == 1 || o >= 18;
}

// Most entries of one x-line's span (8 rows of 2 or 3 x-offsets, times 3 x 3),
// and the store instructions per lane that cover it.
constexpr int kOwnSpanMax = (2 + 3 * (kOwnTile - 1)) * 9;
constexpr int kOwnSpanIters = (kOwnSpanMax + 63) / 64;

// Memory is accessed through buffer resources (base, byte range): an access
// outside the range reads 0 or is dropped, so every load and store is issued
// unconditionally, in a fixed number per step, and no register is zeroed
// before a load.  A predicated (exec-masked) access would make the compiler
// wait for everything in flight before the register is reused or when the
// number of stores in flight is not known; with one wave per SIMD nothing
// hides those waits.
constexpr uint32_t kOwnOut = 0xFFFFFFFFu;  // byte offset outside every range (ranges end below 2^32 - 256)
constexpr int kOwnRsrcWord3 = 0x00020000;  // raw (untyped) buffer access on gfx9-family parts

__device__ __forceinline__ __amdgpu_buffer_rsrc_t own_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, static_cast<int>(bytes), kOwnRsrcWord3);
}
__device__ __forceinline__ double own_ld_f64(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, static_cast<int>(off), 0, 0));
}
__device__ __forceinline__ float own_ld_f32(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, static_cast<int>(off), 0, 0));
}
__device__ __forceinline__ int32_t own_ld_i32(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(int32_t, __builtin_amdgcn_raw_buffer_load_b32(r, static_cast<int>(off), 0, 0));
}
// non-temporal store (the values are not read again by this launch)
constexpr int kOwnStoreNT = 2;
__device__ __forceinline__ void own_st(double x, __amdgpu_buffer_rsrc_t r, uint32_t off) {
  using u2 = __attribute__((ext_vector_type(2))) unsigned;
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, x), r, static_cast<int>(off), 0, kOwnStoreNT);
}
__device__ __forceinline__ void own_st(float x, __amdgpu_buffer_rsrc_t r, uint32_t off) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, x), r, static_cast<int>(off), 0, kOwnStoreNT);
}

// Bijection of [0, n): workgroup b (on XCD b mod 8) -> tile, the tiles of
// one XCD consecutive.  With q = n / 8, r = n % 8, XCD x < r takes q + 1
// tiles and the others q.
constexpr int kXcds = 8;
__device__ __forceinline__ int own_xcd_tile(int b, int n) {
  const int q = n / kXcds, r = n % kXcds, x = b % kXcds, k = b / kXcds;
  return x < r ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

template <int P, typename T, typename R>
__global__ __launch_bounds__(64, (OwnCfg<T, R>::WPE)) void k_h1_owner(
    int nex, int ney, int nez, int ntx, int seglen, const int32_t* __restrict__ elem3d,
    const double* __restrict__ coords, const T* __restrict__ kappa, T beta, int64_t nel, int64_t nnz,
    T* __restrict__ values, unsigned flags, R det_thresh, int32_t* __restrict__ diag) {
  using C = OwnCfg<T, R>;
  constexpr int NSUB = P * P * P, NPL = C::NPL;
  static_assert(C::LPS == 1, "one cell layer per step");
  static_assert(NPL == 2, "two staged planes");
  __shared__ __align__(16) unsigned char sBuf[C::LDS];
  auto plane = [&](int Z) { return reinterpret_cast<double*>(sBuf + C::SLAB + (Z & 1) * C::PLANE); };
  R* const sCell = reinterpret_cast<R*>(sBuf);  // cell matrices of the layer
  T* const sStg = reinterpret_cast<T*>(sBuf);   // then the finished rows of its lower plane

  const int NXc = nex * P, NYc = ney * P, NZc = nez * P;  // cells per axis
  const int LX = NXc + 1, LY = NYc + 1, LZ = NZc + 1;     // lattice points per axis
  const int lane = threadIdx.x;
  // Workgroups are dealt to the 8 XCDs in turn (workgroup b to XCD b mod 8),
  // each with its own L2; tiles next to each other share a column or row of
  // lattice points.  So XCD k gets a contiguous run of tiles (about an eighth
  // of the tile rows) instead of every eighth tile.
  const int tile = own_xcd_tile(static_cast<int>(blockIdx.x), static_cast<int>(gridDim.x));
  const int ti = tile % ntx, tj = tile / ntx;
  const int x0 = kOwnStride * ti, y0 = kOwnStride * tj;
  const int zs = blockIdx.y * seglen;
  const int ze = zs + seglen < NZc ? zs + seglen : NZc;
  kappa += static_cast<int64_t>(blockIdx.z) * nel * NSUB;
  values += static_cast<int64_t>(blockIdx.z) * nnz;
  // byte ranges below 2^32: checked by the launch
  const auto rX = own_rsrc(coords, static_cast<uint32_t>(static_cast<int64_t>(LX) * LY * LZ * 24));
  const auto rK = own_rsrc(kappa, static_cast<uint32_t>(nel * NSUB * static_cast<int64_t>(sizeof(T))));
  const auto rE = own_rsrc(elem3d, static_cast<uint32_t>(nel * 4));

  const int lx = lane & 7, ly = lane >> 3;
  const int cX = x0 + lx, cY = y0 + ly;                // this lane's cell / row column (x, y)
  const bool cell_in = cX < NXc && cY < NYc;
  const bool row_in = cX <= NXc && cY <= NYc;           // row (cX, cY) exists in every plane
  const bool row_own = row_in && (lx > 0 || ti == 0) && (ly > 0 || tj == 0);
  // An inner tile (most of them): all 64 of its cells exist and, on an inner
  // plane (0 < Z < NZc), every row it owns (x, y in [1, 7]) has all 27
  // neighbours.  Its steps on inner planes take a path without per-lane
  // conditions: the row sums read all four cells (lanes x = 0 or y = 0 read
  // clamped cells and own no row), each owned row is one 27-entry copy, and
  // the seven owned lines of the plane are 7 rows x 27 entries each.
  const bool tile_inner = ti > 0 && tj > 0 && x0 + kOwnTile <= NXc && y0 + kOwnTile <= NYc;
  // lattice points of a plane: slot j -> point lane + 64 j of the 9 x 9 grid
  auto pt_xy = [&](int j, int& X, int& Y) {
    const int pidx = lane + 64 * j;
    X = x0 + pidx % (kOwnTile + 1);
    Y = y0 + pidx / (kOwnTile + 1);
    return pidx < kOwnPts && X <= NXc && Y <= NYc;
  };
  // coordinates of the tile's points of plane Z (vertex X + LX (Y + LY Z));
  // absent points read 0 and are never used
  auto load_xyz = [&](int Z, double (&xq)[2][3]) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      int X, Y;
      const bool in = Z <= NZc && pt_xy(j, X, Y);
      // absent points: three distinct offsets past the range (equal ones would
      // be merged into one load whose result is then copied, which waits)
      const uint32_t o =
          in ? static_cast<uint32_t>(24 * (X + LX * (Y + static_cast<int64_t>(LY) * Z))) : kOwnOut - 16u;
      xq[j][0] = own_ld_f64(rX, o);
      xq[j][1] = own_ld_f64(rX, o + 8u);
      xq[j][2] = own_ld_f64(rX, o + 16u);
    }
  };
  auto stage_plane = [&](int Z, const double (&xq)[2][3]) {
    double* pl = plane(Z);
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int pidx = lane + 64 * j;
      if (pidx < kOwnPts) {
        pl[3 * pidx + 0] = xq[j][0];
        pl[3 * pidx + 1] = xq[j][1];
        pl[3 * pidx + 2] = xq[j][2];
      }
    }
  };
  // element of this lane's cell in layer Z (0 where the cell is absent)
  auto load_elem = [&](int Z) {
    const bool in = cell_in && Z < NZc;
    return own_ld_i32(rE, in ? static_cast<uint32_t>(4 * ((static_cast<int64_t>(Z / P) * ney + cY / P) * nex + cX / P))
                             : kOwnOut);
  };
  // coefficient of the cell in layer Z of element el (0 where absent)
  auto load_kap = [&](int Z, int32_t el) {
    const bool in = cell_in && Z < NZc;
    const uint32_t o =
        in ? static_cast<uint32_t>(sizeof(T) * (static_cast<int64_t>(el) * NSUB + (cX % P) + P * ((cY % P) + P * (Z % P))))
           : kOwnOut;
    if constexpr (sizeof(T) == 8)
      return own_ld_f64(rK, o);
    else
      return own_ld_f32(rK, o);
  };

  const int zfirst = zs > 0 ? zs - 1 : zs;  // a segment above the bottom starts one layer lower
  // the segment writes planes zs .. ze - 1; the last one also writes the top
  // plane NZc, whose rows only hold the carry
  const int zend = ze == NZc ? NZc + 1 : ze;

  // Software pipeline, in place: at step Z the plane Z + 1 is staged from
  // registers loaded one step earlier and plane Z + 2 is loaded into them;
  // the coefficient of layer Z was loaded one step earlier, that of layer
  // Z + 1 is loaded after the integration from the element loaded one step
  // earlier, which is then replaced by the element of layer Z + 2.
  double xq[2][3];
  T kq;
  int32_t el;
  {
    double xp[2][3];
    load_xyz(zfirst, xp);
    stage_plane(zfirst, xp);
    load_xyz(zfirst + 1, xq);
    el = load_elem(zfirst);
    kq = load_kap(zfirst, el);
    el = load_elem(zfirst + 1);
    // as many stores as a step issues, all outside their (empty) range: the
    // loop is then entered with the same memory operations in flight after
    // each prefetch as on every later step, so the waits the compiler places
    // at the loop head (merged over both ways in) need not drain the prefetches
    const auto rNone = own_rsrc(values, 0u);
#pragma unroll
    for (int i = 0; i < 8 * kOwnSpanIters; ++i)  // distinct offsets, so that none is merged away
      own_st(T(0), rNone, static_cast<uint32_t>((64 * i + lane) * sizeof(T)));
  }

  double carry[18];
#pragma unroll
  for (int o = 0; o < 18; ++o) carry[o] = 0.0;

  for (int Z = zfirst; Z < zend; ++Z) {
    stage_plane(Z + 1, xq);
    load_xyz(Z + 2, xq);
    __builtin_amdgcn_wave_barrier();

    // the cell (cX, cY, Z): its 36 entries into the slab
    if (cell_in && Z < NZc) {
      const double* pz0 = plane(Z);
      const double* pz1 = plane(Z + 1);
      R* out = sCell + lane;
      auto load_X = [&](double (&X)[8][3]) {
#pragma unroll
        for (int v = 0; v < 8; ++v) {
          const double* pl = (v >> 2) ? pz1 : pz0;
          const int pidx = (lx + (v & 1)) + (kOwnTile + 1) * (ly + ((v >> 1) & 1));
#pragma unroll
          for (int d = 0; d < 3; ++d) X[v][d] = pl[3 * pidx + d];
        }
      };
      const R kap = static_cast<R>(kq);
      // counted once: a cell in a tile's last column (row) is also the first
      // column (row) of the next tile, which counts it
      const bool own = Z >= zs && lx < kOwnStride && ly < kOwnStride;
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
          for (int v = u; v < 8; ++v) out[pair_index(u, v) * 64] = h1_entry<R>(F, u, v);
        if (!ok && own && diag) atomicAdd(&diag[1], 1);
      } else {
        // FP32 only: FP64 geometry, written to the slab
        const bool ok = own_fp64_fallback(pz0, pz1, lx, ly, static_cast<double>(kap), static_cast<double>(beta),
                                          reinterpret_cast<float*>(out));
        if (own && diag) {
          atomicAdd(&diag[0], 1);
          if (!ok) atomicAdd(&diag[1], 1);
        }
      }
    }
    kq = load_kap(Z + 1, el);
    el = load_elem(Z + 2);
    __builtin_amdgcn_wave_barrier();

    // row (cX, cY) of plane Z: the carry (c = 1 corners, layer Z - 1) + this
    // layer's c = 0 corners; this layer's c = 1 corners are the next carry
    double acc[27];
#pragma unroll
    for (int o = 0; o < 27; ++o) acc[o] = o < 18 ? carry[o] : 0.0;
#pragma unroll
    for (int o = 0; o < 18; ++o) carry[o] = 0.0;
    const bool fast = tile_inner && Z > 0 && Z < NZc;  // the same for the whole wave
    if (fast) {
      // the 16 terms of two cells are read while the two before are summed
      // (each term in the same order as on the general path)
      R w[2][16];
      auto fetch = [&](int k, R(&wk)[16]) {
        const int a = k & 1, b = k >> 1;
        const R* cm = sCell + (lx > a ? lx - a : 0) + 8 * (ly > b ? ly - b : 0);
#pragma unroll
        for (int v = 0; v < 8; ++v) {
          wk[v] = cm[pair_index(k, v) * 64];
          wk[8 + v] = cm[pair_index(k + 4, v) * 64];
        }
      };
      auto sum = [&](int k, const R(&wk)[16]) {
#pragma unroll
        for (int v = 0; v < 8; ++v) {
          double& ea = acc[own_off(k, v)];
          double& ec = carry[own_off(k + 4, v)];
          ea = own_first(k, v, 0) ? static_cast<double>(wk[v]) : ea + static_cast<double>(wk[v]);
          ec = own_first(k, v, 1) ? static_cast<double>(wk[8 + v]) : ec + static_cast<double>(wk[8 + v]);
        }
      };
      fetch(0, w[0]);
      fetch(1, w[1]);
      __builtin_amdgcn_sched_barrier(0);
      sum(0, w[0]);
      fetch(2, w[0]);
      __builtin_amdgcn_sched_barrier(0);
      sum(1, w[1]);
      fetch(3, w[1]);
      __builtin_amdgcn_sched_barrier(0);
      sum(2, w[0]);
      sum(3, w[1]);
    } else if (row_in && Z < NZc) {
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
    if (Z < zs) continue;  // the layer below the segment: carry only

    // stage the owned rows of each x-line in CSR order: a row holds
    // (x-offsets) x (y-offsets) x (z-offsets) entries, 2 per axis at a
    // lattice end and 3 elsewhere
    const int ylo = cY > 0, yhi = cY < NYc, zlo = Z > 0, zhi = Z < NZc;
    const int ny = 1 + ylo + yhi, nyz = ny * (1 + zlo + zhi);
    const int xfirst = ti == 0 ? 0 : 1;  // first owned row of the tile's x-lines
    const int xa = x0 + xfirst;          // first owned row of the lines
    const int pxa = static_cast<int>(box_prefix(xa, LX));
    if (fast) {
      if (lx > 0 && ly > 0) {
        T* row = sStg + 27 * 8 * ly + 27 * (lx - 1);
#pragma unroll
        for (int k = 0; k < 27; ++k) row[k] = static_cast<T>(acc[k]);
      }
    } else if (row_own) {
      const int xlo = cX > 0, xhi = cX < NXc, nx = 1 + xlo + xhi;
      // x-offset counts of the owned rows before this one in its line
      const int before = static_cast<int>(box_prefix(cX, LX)) - pxa;
      T* row = sStg + 27 * 8 * ly + before * nyz + (zlo * ny + ylo) * nx + xlo;
#pragma unroll
      for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
          for (int dx = -1; dx <= 1; ++dx) {
            const bool ok = (dx >= 0 || xlo) && (dx <= 0 || xhi) && (dy >= 0 || ylo) && (dy <= 0 || yhi) &&
                            (dz >= 0 || zlo) && (dz <= 0 || zhi);
            if (ok) row[dz * nx * ny + dy * nx + dx] = static_cast<T>(acc[(dx + 1) + 3 * (dy + 1) + 9 * (dz + 1)]);
          }
    }
    __builtin_amdgcn_wave_barrier();
    // one contiguous span per owned x-line, through a buffer resource over
    // exactly that span (empty for the lines the tile does not own).  Row
    // starts are below nnz < 2^31; line Y of plane Z starts at lb and its
    // rows from xa on at lb + cy cz box_prefix(xa), and line Y + 1 starts
    // SX cy cz later
    const int SX = 3 * LX - 2;
    if (fast) {
      // lines 1..7: 7 rows x 27 entries, the owned rows of line y0 + l from
      // box_row_start(0, y0, Z) + 9 (SX l + box_prefix(xa)); line 0 empty
      const T* vb = values + (static_cast<int>(box_row_start(0, y0, Z, LX, LY, LZ)) + 9 * pxa);
      const int dl = 9 * SX;
      // all of the plane's staged values first, then the stores
      T sv[8][kOwnSpanIters];
#pragma unroll
      for (int l = 0; l < 8; ++l)
#pragma unroll
        for (int it = 0; it < kOwnSpanIters; ++it) {
          const int t = lane + 64 * it;
          sv[l][it] = sStg[27 * 8 * l + (t < kOwnSpanMax ? t : kOwnSpanMax - 1)];
        }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int l = 0; l < 8; ++l) {
        const auto rV = own_rsrc(vb + l * dl, l > 0 ? 7 * 27 * static_cast<uint32_t>(sizeof(T)) : 0u);
#pragma unroll
        for (int it = 0; it < kOwnSpanIters; ++it)
          own_st(sv[l][it], rV, static_cast<uint32_t>((lane + 64 * it) * sizeof(T)));
      }
      continue;
    }
    const int xlast = x0 + 7 < NXc ? x0 + 7 : NXc;  // last owned row of the lines
    const int span_x = static_cast<int>(box_prefix(xlast + 1, LX)) - pxa;
    const int cz = 1 + zlo + zhi;
    int lb = static_cast<int>(box_row_start(0, y0, Z, LX, LY, LZ));
#pragma unroll
    for (int l = 0; l < 8; ++l) {
      const int Y = y0 + l;
      const int cyz = box_count(Y, LY) * cz;
      const bool line = (l > 0 || tj == 0) && Y <= NYc;
      const int span = line ? span_x * cyz : 0;
      const auto rV = own_rsrc(values + (line ? lb + cyz * pxa : 0), static_cast<uint32_t>(span * sizeof(T)));
      lb += SX * cyz;
      const T* src = sStg + 27 * 8 * l;
#pragma unroll
      for (int it = 0; it < kOwnSpanIters; ++it) {
        const int t = lane + 64 * it;
        own_st(src[t < kOwnSpanMax ? t : kOwnSpanMax - 1], rV, static_cast<uint32_t>(t * sizeof(T)));
      }
    }
  }
}

// Whether the owner-computes kernel's buffer ranges (coordinates, one batch
// entry's coefficients, the element grid) stay below 2^32 bytes.
bool owner_fits(const lor_sched* s, int tsize) {
  const int64_t nsub = static_cast<int64_t>(s->p) * s->p * s->p;
  const int64_t lim = (int64_t(1) << 32) - 256;
  return s->nrows * 24 < lim && s->nel * nsub * tsize < lim && s->nel * 4 < lim;
}

// Compute units of the current device (cached per device).
static int owner_num_cus() {
  static int cus[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (cus[dev] == 0) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
    cus[dev] = n;
  }
  return cus[dev];
}

template <int P, typename T, typename R>
static int launch_owner(const lor_sched* sched, int batch, const void* kappa, double beta, const double* coords,
                        const int32_t* row_ptr, void* values, unsigned flags, double thr, int32_t* diag,
                        hipStream_t st) {
  const int nex = sched->box[0], ney = sched->box[1], nez = sched->box[2];
  if (nex < 1 || ney < 1 || nez < 1 || static_cast<int64_t>(nex) * ney * nez != sched->nel ||
      (static_cast<int64_t>(nex) * P + 1) * (static_cast<int64_t>(ney) * P + 1) * (static_cast<int64_t>(nez) * P + 1) !=
          sched->nrows)
    LOR_FAIL(LOR_EINVAL, "the owner-computes schedule does not describe the mesh");
  if (!owner_fits(sched, static_cast<int>(sizeof(T))))
    LOR_FAIL(LOR_EUNSUPPORTED, "owner-computes kernel: coordinates or coefficients span 4 GiB or more");
  const int NXc = nex * P, NYc = ney * P, NZc = nez * P;
  const int64_t ntx = ceil_div(NXc, kOwnStride), nty = ceil_div(NYc, kOwnStride);
  const int64_t tiles = ntx * nty;
  if (tiles > INT32_MAX) LOR_FAIL(LOR_EOVERFLOW, "too many owner-computes tiles");
  // Split the z-march into segments (a segment above the bottom costs one
  // extra cell layer).  The waves run in rounds over the chip's wave slots
  // (CUs x resident waves per CU), so the launch takes about
  // ceil(waves / slots) x (layers per wave + 1) layer steps: pick the segment
  // length (at least 8 layers) that minimises it, so that the last round is
  // not left mostly idle.
  const int64_t slots = static_cast<int64_t>(owner_num_cus()) * OwnCfg<T, R>::WPC;
  int64_t seglen = NZc, best = -1;
  for (int64_t len = std::min<int64_t>(8, NZc); len <= NZc; ++len) {
    const int64_t ns = ceil_div(NZc, len);
    if (ns > 1 && ceil_div(NZc, ns) != len) continue;  // same split as a shorter length
    const int64_t cost = ceil_div(tiles * ns * batch, slots) * (len + 1);
    if (best < 0 || cost < best) {
      best = cost;
      seglen = len;
    }
  }
  const int64_t nseg = ceil_div(NZc, seglen);
  dim3 grid(static_cast<unsigned>(tiles), static_cast<unsigned>(nseg), static_cast<unsigned>(batch));
  (void)row_ptr;  // the rows start where the lattice puts them (the pattern call checked row_ptr)
  k_h1_owner<P, T, R><<<grid, 64, 0, st>>>(
      nex, ney, nez, static_cast<int>(ntx), static_cast<int>(seglen), dev_at<int32_t>(sched, sched->off_elem3d),
      coords, static_cast<const T*>(kappa), static_cast<T>(beta), sched->nel, sched->nnz, static_cast<T*>(values),
      flags, static_cast<R>(thr), diag);
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
