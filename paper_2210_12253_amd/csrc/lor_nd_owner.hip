// Values of the LOR H(curl) matrix, owner-computes form (Step S1.2 for the
// lowest-order Nedelec space of Section 2.3: every row summed once, on the
// chip, and stored once, whole).
//
// On an edge lattice (the pattern call checks that the mesh is one: with
// (MX, MY, MZ) cells per axis, the x-edge from lattice point (X, Y, Z) has id
// X + MX (Y + (MY + 1) Z), the y-edges and z-edges follow at
// OY = MX (MY + 1) (MZ + 1) and OZ = OY + (MX + 1) MY (MZ + 1) in the same
// way, the element at every box position is known, and the CSR pattern is
// the closed form below) the row of an edge along axis m holds the edges of
// the <= 4 cells around it, at most 33:
//
//   * one launch per edge direction m.  A wave takes a tile of 8 x 8 cells in
//     the two other axes (tiles overlap by one cell, stride 7) and marches
//     along m over a segment of cell layers; the rows of the edges along m
//     in a layer need only that layer's cells, so the steps carry nothing;
//   * lane (i, j) integrates its cell (the 4 rows of its edges along m, 12
//     columns each, times the orientation signs from its element's edge map)
//     into the wave's LDS slab (FP64: 2 rows at a time, in two passes, so
//     that LDS does not limit the waves per CU), then sums the row of the
//     edge along m at its tile node from the cells at lanes (i - a, j - b),
//     a, b in {0, 1}, in one fixed order of the cells (increasing z, then y,
//     then x) that every direction's launch shares, so the matrix is bitwise
//     symmetric;
//   * a row's columns are sorted by id: the x-edges, then the y-edges, then
//     the z-edges, each group in (z, y, x) order over per-axis ranges (a
//     node axis has 3 values inside the box and 2 on its faces, a cell axis
//     2 and 1, the edge's own axis 1 or 2), so an entry's position is a
//     mixed-radix number; the sums run in the 33 inside positions and are
//     compacted on the box faces;
//   * the finished rows are staged in LDS and stored row after row (64 lanes
//     over consecutive entries), each at its row pointer.
// Every cell is integrated once per direction (3x the work of one pass, plus
// the one-cell tile overlap); all sums are FP64, in the FP32 form too.  The
// cell corners are gathered through the vertex map, so the vertex numbering
// can be anything.
#include <algorithm>

#include "lor_common.hpp"
#include "lor_nd_math.hpp"

namespace lor {

constexpr int kNdTile = 8;               // cells per tile side (one wave: 8 x 8)
constexpr int kNdStride = kNdTile - 1;   // tiles overlap by one cell
constexpr int kNdRow = 33;               // entries of an inside row
constexpr int kNdStoreIters = 64 * kNdRow / 64;

// Local edge v of a cell (numbering of the ND integration): its direction
// and its offset from the cell's lowest corner.
//   x-edges (b, c) -> b + 2c at (0, b, c); y-edges (a, c) -> 4 + a + 2c at
//   (a, 0, c); z-edges (a, b) -> 8 + a + 2b at (a, b, 0).
__host__ __device__ constexpr int nd_dir(int v) { return v >> 2; }
__host__ __device__ constexpr int nd_off(int v, int d) {
  const int e = v >> 2, s = v & 3, lo = s & 1, hi = s >> 1;
  // the two non-zero offsets are along the two axes other than e, lower axis first
  return d == e ? 0 : (d == (e == 0 ? 1 : 0) ? lo : hi);
}

// Inside position (full per-axis ranges) of column v of the cell at offsets
// (a, b) below the row's edge along m in its two other axes t1 < t2.
__host__ __device__ constexpr int nd_slot(int m, int a, int b, int v) {
  const int t1 = m == 0 ? 1 : 0, t2 = m == 2 ? 1 : 2;
  const int g = nd_dir(v);
  int rel[3] = {0, 0, 0};
  rel[t1] = -a;
  rel[t2] = -b;
  for (int d = 0; d < 3; ++d) rel[d] += nd_off(v, d);
  int cnt[3] = {0, 0, 0}, idx[3] = {0, 0, 0};
  for (int d = 0; d < 3; ++d) {
    if (d == m) {
      cnt[d] = g == m ? 1 : 2;
      idx[d] = rel[d];
    } else {
      cnt[d] = d == g ? 2 : 3;
      idx[d] = rel[d] + 1;
    }
  }
  int off = 0;
  for (int h = 0; h < g; ++h) off += (h == m ? 1 * 3 * 3 : 2 * 2 * 3);
  return off + (idx[2] * cnt[1] + idx[1]) * cnt[0] + idx[0];
}

// Group, and per-axis inside index, of inside position k of a row along m.
struct NdSlot {
  int g, idx[3];
};
__host__ __device__ constexpr NdSlot nd_slot_decode(int m, int k) {
  NdSlot s{0, {0, 0, 0}};
  int off = 0;
  for (int h = 0; h < 3; ++h) {
    const int size = h == m ? 9 : 12;
    if (k < off + size) {
      s.g = h;
      int cnt[3] = {0, 0, 0};
      for (int d = 0; d < 3; ++d) cnt[d] = d == m ? (h == m ? 1 : 2) : (d == h ? 2 : 3);
      int r = k - off;
      s.idx[0] = r % cnt[0];
      r /= cnt[0];
      s.idx[1] = r % cnt[1];
      s.idx[2] = r / cnt[1];
      return s;
    }
    off += size;
  }
  return s;
}

constexpr bool nd_slots_ok() {
  // the 4 cells' 48 columns land in the 33 inside positions, each position
  // reached, and the decode inverts the encode
  for (int m = 0; m < 3; ++m) {
    bool hit[kNdRow] = {};
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b)
        for (int v = 0; v < 12; ++v) {
          const int k = nd_slot(m, a, b, v);
          if (k < 0 || k >= kNdRow) return false;
          hit[k] = true;
        }
    for (int k = 0; k < kNdRow; ++k)
      if (!hit[k]) return false;
  }
  return true;
}
static_assert(nd_slots_ok(), "ND row layout");

// Global id of the edge along e from lattice point c (edge lattice above).
__host__ __device__ __forceinline__ int64_t nd_edge_id(int e, int64_t x, int64_t y, int64_t z, int64_t MX, int64_t MY,
                                                      int64_t MZ) {
  const int64_t OY = MX * (MY + 1) * (MZ + 1), OZ = OY + (MX + 1) * MY * (MZ + 1);
  if (e == 0) return x + MX * (y + (MY + 1) * z);
  if (e == 1) return OY + x + (MX + 1) * (y + MY * z);
  return OZ + x + (MX + 1) * (y + (MY + 1) * z);
}

// FP32 form, strongly distorted cell: FP64 integration from the FP64 corners
// (gathered again; lv0 = local vertex of corner 0), the rows of the cell's
// edges along m (local r0 + a + 2 b) signed by negmask (bit v: edge v
// reversed) and rounded to FP32 into the slab ([row][col][lane]).
template <int P>
__device__ __forceinline__ bool nd_owner_fp64_fallback(const int32_t* __restrict__ elem_dofs,
                                                    const double* __restrict__ coords, int32_t el, int lv0, int r0,
                                                    double kap, double bet, unsigned negmask, float* out) {
  constexpr int Q = P + 1, NLOCV = Q * Q * Q;
  double X[8][3];
#pragma unroll
  for (int v = 0; v < 8; ++v) {
    const int64_t g = elem_dofs[static_cast<int64_t>(el) * NLOCV + lv0 + (v & 1) + Q * (((v >> 1) & 1) + Q * (v >> 2))];
#pragma unroll
    for (int d = 0; d < 3; ++d) X[v][d] = coords[3 * g + d];
  }
  double ex[2][2][3], ey[2][2][3], ez[2][2][3];
  h1_edges<double>(X, ex, ey, ez);
  H1Factors<double> F;
  NDCurl<double> W;
  const bool ok = nd_factors<double>(ex, ey, ez, kap, bet, F, W);
  for (int j = 0; j < 4; ++j) {
    const int r = r0 + (j & 1) + 2 * (j >> 1);
#pragma unroll
    for (int v = 0; v < 12; ++v) {
      const float e = static_cast<float>(nd_entry<double>(F, W, r < v ? r : v, r < v ? v : r));
      out[(j * 12 + v) * 64] = (((negmask >> r) ^ (negmask >> v)) & 1u) ? -e : e;
    }
  }
  return ok;
}

// Two waves per SIMD at most registers: the FP32 form's FP64 fallback is
// inlined (a call would make the kernel reserve the callee's registers too).
template <int P, typename T, typename R, int M>
__global__ __launch_bounds__(64, 2) void k_nd_owner(int nex, int ney, int nez, int nt1, int seglen,
                                                const int32_t* __restrict__ elem3d,
                                                const int32_t* __restrict__ elem_dofs,
                                                const int32_t* __restrict__ elem_edges,
                                                const double* __restrict__ coords, const T* __restrict__ kappa, T beta,
                                                const int32_t* __restrict__ row_ptr, int64_t nel, int64_t nnz,
                                                T* __restrict__ values, unsigned flags, R det_thresh,
                                                int32_t* __restrict__ diag) {
  constexpr int Q = P + 1, NSUB = P * P * P, NLOCV = Q * Q * Q, NLOCE = 3 * P * Q * Q;
  constexpr int T1 = M == 0 ? 1 : 0, T2 = M == 2 ? 1 : 2;  // the tile axes
  constexpr int RBASE = 4 * M;                              // first local edge along M
  // FP64: the cell's 4 rows go through the slab in two passes (b = 1, then
  // b = 0), so that the slab takes half the LDS and does not limit the waves
  // per CU
  constexpr int NH = sizeof(R) == 8 ? 2 : 1;
  constexpr int RPP = 4 / NH;  // rows per pass
  constexpr int SLAB = RPP * 12 * 64 * static_cast<int>(sizeof(R));
  constexpr int STG = 64 * kNdRow * static_cast<int>(sizeof(T));
  __shared__ __align__(16) unsigned char sBuf[SLAB > STG ? SLAB : STG];
  __shared__ int64_t sStart[64];
  __shared__ int32_t sLen[64];
  R* const sCell = reinterpret_cast<R*>(sBuf);  // the 4 rows along M of each cell: [row a + 2b][col][lane]
  T* const sStg = reinterpret_cast<T*>(sBuf);   // then the finished rows: [lane][kNdRow]

  const int L[3] = {nex * P, ney * P, nez * P};
  const int lane = threadIdx.x;
  // XCD-aware order: workgroups go to the 8 XCDs round-robin by linear id, so
  // linear id g runs (tile, segment) number (g mod 8) * (n / 8) + g / 8 of
  // the tile-fastest order: each XCD walks a contiguous run of layers, tile
  // after tile, and finds the corners and edge words its neighbours loaded
  // in its own L2 (the last n mod 8 ids keep their place)
  const int64_t ntile = gridDim.x, nlin = ntile * gridDim.y;
  const int64_t glin = blockIdx.x + ntile * blockIdx.y, gfull = nlin & ~int64_t(7);
  const int64_t hlin = glin < gfull ? (glin & 7) * (gfull >> 3) + (glin >> 3) : glin;
  const int tile = static_cast<int>(hlin % ntile), seg = static_cast<int>(hlin / ntile);
  const int i1 = tile % nt1, i2 = tile / nt1;
  const int l1 = lane & 7, l2 = lane >> 3;
  const int c1 = kNdStride * i1 + l1, c2 = kNdStride * i2 + l2;  // this lane's cell / node along T1, T2
  const int ms = seg * seglen;
  const int me = ms + seglen < L[M] ? ms + seglen : L[M];
  kappa += static_cast<int64_t>(blockIdx.z) * nel * NSUB;
  values += static_cast<int64_t>(blockIdx.z) * nnz;

  const bool cell_col = c1 < L[T1] && c2 < L[T2];
  const bool row_own = c1 <= L[T1] && c2 <= L[T2] && (l1 > 0 || i1 == 0) && (l2 > 0 || i2 == 0);
  const int c1c = c1 < L[T1] ? c1 : L[T1] - 1, c2c = c2 < L[T2] ? c2 : L[T2] - 1;
  // the row's per-axis ranges along T1 and T2 (nodes; cells for the group
  // along that axis): lower end and whether the lower / upper neighbour exists
  const int lo1 = c1 > 0, hi1 = c1 < L[T1], lo2 = c2 > 0, hi2 = c2 < L[T2];
  const bool inside = lo1 && hi1 && lo2 && hi2;
  // counted once: cells in a tile's last column or row are the next tile's
  // first; only the x-edge launch counts
  const bool count = M == 0 && l1 < kNdStride && l2 < kNdStride;

  // the cell's rows RBASE + jb .. RBASE + jb + RPP - 1 into the slab, signed
  auto write_rows = [&](const H1Factors<R>& F, const NDCurl<R>& W, unsigned negmask, int jb) {
#pragma unroll
    for (int jj = 0; jj < RPP; ++jj) {
      const int r = RBASE + jb + jj;
#pragma unroll
      for (int v = 0; v < 12; ++v) {
        const R e = nd_entry<R>(F, W, r < v ? r : v, r < v ? v : r);
        sCell[(jj * 12 + v) * 64 + lane] = (((negmask >> r) ^ (negmask >> v)) & 1u) ? -e : e;
      }
    }
  };
  // the cell's element, coefficient, corners and edge orientations (bit v of
  // negmask: local edge v reversed; local edges of the element: x-edges
  // i + p (j + q k), y-edges p q^2 + i + q (j + p k), z-edges
  // 2 p q^2 + i + q (j + q k))
  auto load_cell = [&](const int (&C)[3], int32_t& el, int& lv0, R& kap, double (&Xv)[8][3], unsigned& negmask) {
    el = elem3d[(static_cast<int64_t>(C[2] / P) * ney + C[1] / P) * nex + C[0] / P];
    const int sx = C[0] % P, sy = C[1] % P, sz = C[2] % P;
    lv0 = sx + Q * (sy + Q * sz);
    kap = static_cast<R>(kappa[static_cast<int64_t>(el) * NSUB + sx + P * (sy + P * sz)]);
#pragma unroll
    for (int v = 0; v < 8; ++v) {
      const int64_t g = elem_dofs[static_cast<int64_t>(el) * NLOCV + (sx + (v & 1)) +
                                  Q * ((sy + ((v >> 1) & 1)) + Q * (sz + (v >> 2)))];
#pragma unroll
      for (int d = 0; d < 3; ++d) Xv[v][d] = coords[3 * g + d];
    }
    const int32_t* em = elem_edges + static_cast<int64_t>(el) * NLOCE;
    negmask = 0;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int lo = s & 1, hi = s >> 1;
      negmask |= (em[sx + P * ((sy + lo) + Q * (sz + hi))] < 0 ? 1u : 0u) << s;
      negmask |= (em[P * Q * Q + (sx + lo) + Q * (sy + P * (sz + hi))] < 0 ? 1u : 0u) << (4 + s);
      negmask |= (em[2 * P * Q * Q + (sx + lo) + Q * ((sy + hi) + Q * sz)] < 0 ? 1u : 0u) << (8 + s);
    }
  };
  // add the slab's rows of the cells at lanes (l1 - a, l2 - b), b in
  // [b_hi, b_lo] downwards and a = 1 before a = 0, to the row of the edge
  // along M at this lane's node (the edge is the cell's local edge
  // RBASE + a + 2b; the slab holds rows from RBASE + jb)
  auto sum_rows = [&](double (&acc)[kNdRow], int b_hi, int b_lo, int jb) {
#pragma unroll
    for (int b = 1; b >= 0; --b) {
      if (b > b_hi || b < b_lo) continue;
#pragma unroll
      for (int a = 1; a >= 0; --a) {
        if ((a == 0 || lo1) && (b == 0 || lo2) && (a == 1 || hi1) && (b == 1 || hi2)) {
          const R* cm_ = sCell + (lane - a - 8 * b) + (a + 2 * b - jb) * 12 * 64;
#pragma unroll
          for (int v = 0; v < 12; ++v) acc[nd_slot(M, a, b, v)] += static_cast<double>(cm_[v * 64]);
        }
      }
    }
  };

  for (int cm = ms; cm < me; ++cm) {
    double acc[kNdRow];
    if constexpr (NH == 1) {
      // all 4 rows through the slab at once; in the FP32 form strongly
      // distorted cells take the FP64 fallback (the gathers written out here:
      // through load_cell this form compiles to a slower schedule)
      int C[3];
      C[M] = cm;
      C[T1] = c1c;
      C[T2] = c2c;
      if (cell_col) {
        const int32_t el = elem3d[(static_cast<int64_t>(C[2] / P) * ney + C[1] / P) * nex + C[0] / P];
        const int sx = C[0] % P, sy = C[1] % P, sz = C[2] % P;
        const R kap = static_cast<R>(kappa[static_cast<int64_t>(el) * NSUB + sx + P * (sy + P * sz)]);
        double Xv[8][3];
#pragma unroll
        for (int v = 0; v < 8; ++v) {
          const int64_t g = elem_dofs[static_cast<int64_t>(el) * NLOCV + (sx + (v & 1)) +
                                      Q * ((sy + ((v >> 1) & 1)) + Q * (sz + (v >> 2)))];
#pragma unroll
          for (int d = 0; d < 3; ++d) Xv[v][d] = coords[3 * g + d];
        }
        // orientation of the cell's 12 edges in its element's edge map (local
        // edges: x-edges i + p (j + q k), y-edges p q^2 + i + q (j + p k),
        // z-edges 2 p q^2 + i + q (j + q k))
        unsigned negmask = 0;
        const int32_t* em = elem_edges + static_cast<int64_t>(el) * NLOCE;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int lo = s & 1, hi = s >> 1;
          negmask |= (em[sx + P * ((sy + lo) + Q * (sz + hi))] < 0 ? 1u : 0u) << s;
          negmask |= (em[P * Q * Q + (sx + lo) + Q * (sy + P * (sz + hi))] < 0 ? 1u : 0u) << (4 + s);
          negmask |= (em[2 * P * Q * Q + (sx + lo) + Q * ((sy + hi) + Q * sz)] < 0 ? 1u : 0u) << (8 + s);
        }
        bool fallback = false;
        if constexpr (!std::is_same<R, double>::value) {
          if (flags & LOR_FP64_FALLBACK) {
            R ex[2][2][3], ey[2][2][3], ez[2][2][3];
            h1_edges<R>(Xv, ex, ey, ez);
            R dmin, dmax;
            h1_corner_det_range<R>(ex, ey, ez, dmin, dmax);
            fallback = !(dmin > R(0)) || dmax > det_thresh * dmin;
          }
        }
        if (!fallback) {
          R ex[2][2][3], ey[2][2][3], ez[2][2][3];
          h1_edges<R>(Xv, ex, ey, ez);
          H1Factors<R> F;
          NDCurl<R> W;
          const bool ok = nd_factors<R>(ex, ey, ez, kap, static_cast<R>(beta), F, W);
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int r = RBASE + j;
#pragma unroll
            for (int v = 0; v < 12; ++v) {
              const R e = nd_entry<R>(F, W, r < v ? r : v, r < v ? v : r);
              sCell[(j * 12 + v) * 64 + lane] = (((negmask >> r) ^ (negmask >> v)) & 1u) ? -e : e;
            }
          }
          if (!ok && count && diag) atomicAdd(&diag[1], 1);
        } else {
          const bool ok = nd_owner_fp64_fallback<P>(elem_dofs, coords, el, sx + Q * (sy + Q * sz), RBASE,
                                                    static_cast<double>(kap), static_cast<double>(beta), negmask,
                                                    reinterpret_cast<float*>(sCell) + lane);
          if (count && diag) {
            atomicAdd(&diag[0], 1);
            if (!ok) atomicAdd(&diag[1], 1);
          }
        }
      }
      __syncthreads();

      // the row of the edge along M at (cm, c1, c2): the cells at lanes
      // (l1 - a, l2 - b) in increasing (z, y, x), i.e. b = 1 before b = 0 and a
      // = 1 before a = 0 (the edge is the cell's local edge RBASE + a + 2b)
#pragma unroll
      for (int k = 0; k < kNdRow; ++k) acc[k] = 0.0;
      if (row_own) {
#pragma unroll
        for (int b = 1; b >= 0; --b)
#pragma unroll
          for (int a = 1; a >= 0; --a) {
            if ((a == 0 || lo1) && (b == 0 || lo2) && (a == 1 || hi1) && (b == 1 || hi2)) {
              const R* cm_ = sCell + (lane - a - 8 * b) + (a + 2 * b) * 12 * 64;
#pragma unroll
              for (int v = 0; v < 12; ++v) acc[nd_slot(M, a, b, v)] += static_cast<double>(cm_[v * 64]);
            }
          }
      }
      __syncthreads();  // the staging area is the slab
    } else {
      // FP64 form: the rows of b = 1 (local edges RBASE + 2, + 3), then those
      // of b = 0, each pass through the half-size slab
      int C[3];
      C[M] = cm;
      C[T1] = c1c;
      C[T2] = c2c;
      H1Factors<R> F;
      NDCurl<R> W;
      unsigned negmask = 0;
      if (cell_col) {
        int32_t el;
        int lv0;
        R kap;
        double Xv[8][3];
        load_cell(C, el, lv0, kap, Xv, negmask);
        R ex[2][2][3], ey[2][2][3], ez[2][2][3];
        h1_edges<R>(Xv, ex, ey, ez);
        const bool ok = nd_factors<R>(ex, ey, ez, kap, static_cast<R>(beta), F, W);
        if (!ok && count && diag) atomicAdd(&diag[1], 1);
      }
#pragma unroll
      for (int k = 0; k < kNdRow; ++k) acc[k] = 0.0;
#pragma unroll
      for (int b = 1; b >= 0; --b) {
        if (cell_col) write_rows(F, W, negmask, 2 * b);
        __syncthreads();
        if (row_own) sum_rows(acc, b, b, 2 * b);
        __syncthreads();  // the slab is written again, or is the staging area
      }
    }

    // stage the row, compacted on the box faces, and its start and length
    if (row_own) {
      int R3[3];
      R3[M] = cm;
      R3[T1] = c1;
      R3[T2] = c2;
      const int64_t row = nd_edge_id(M, R3[0], R3[1], R3[2], L[0], L[1], L[2]);
      T* dst = sStg + lane * kNdRow;
      int len = 0;
      if (inside) {
#pragma unroll
        for (int k = 0; k < kNdRow; ++k) dst[k] = static_cast<T>(acc[k]);
        len = kNdRow;
      } else {
        // per group g and axis d: the count and the inside index of the
        // range's lower end (0, or 1 where the lower neighbour is missing)
        auto cnt = [&](int g, int d) -> int {
          if (d == M) return g == M ? 1 : 2;
          const int lo = d == T1 ? lo1 : lo2, hi = d == T1 ? hi1 : hi2;
          return d == g ? lo + hi : 1 + lo + hi;
        };
        auto skip = [&](int d) -> int { return d == M ? 0 : (d == T1 ? 1 - lo1 : 1 - lo2); };
        int off[3];
        off[0] = 0;
        off[1] = cnt(0, 0) * cnt(0, 1) * cnt(0, 2);
        off[2] = off[1] + cnt(1, 0) * cnt(1, 1) * cnt(1, 2);
        len = off[2] + cnt(2, 0) * cnt(2, 1) * cnt(2, 2);
#pragma unroll
        for (int k = 0; k < kNdRow; ++k) {
          const NdSlot s = nd_slot_decode(M, k);
          int pos = off[s.g], mul = 1;
          bool ok = true;
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            const int i = s.idx[d] - skip(d);
            const int c = cnt(s.g, d);
            ok = ok && i >= 0 && i < c;
            pos += i * mul;
            mul *= c;
          }
          if (ok) dst[pos] = static_cast<T>(acc[k]);
        }
      }
      sStart[lane] = static_cast<int64_t>(row_ptr[row]);
      sLen[lane] = len;
    } else {
      sLen[lane] = 0;
    }
    __syncthreads();
    // rows one after another: entry t of the staging area is entry t % 33 of
    // the row of lane t / 33
#pragma unroll 4
    for (int it = 0; it < kNdStoreIters; ++it) {
      const int t = lane + 64 * it;
      const int r = t / kNdRow, k = t - r * kNdRow;
      if (k < sLen[r]) values[sStart[r] + k] = sStg[t];
    }
    __syncthreads();
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

template <int P, typename T, typename R, int M>
static int launch_nd_owner_dir(const lor_sched* s, int batch, const int32_t* elem_dofs, const int32_t* elem_edges,
                               const double* coords, const void* kappa, double beta, const int32_t* row_ptr,
                               void* values, unsigned flags, double thr, int32_t* diag, hipStream_t st) {
  const int nex = s->box[0], ney = s->box[1], nez = s->box[2];
  const int L[3] = {nex * P, ney * P, nez * P};
  constexpr int T1 = M == 0 ? 1 : 0, T2 = M == 2 ? 1 : 2;
  // tiles so that the last one reaches the last node: 7 (nt - 1) + 7 >= L
  const int nt1 = static_cast<int>(ceil_div(L[T1], kNdStride)), nt2 = static_cast<int>(ceil_div(L[T2], kNdStride));
  // segments along M (independent: no carry): as many waves as the chip's
  // wave slots hold, from the kernel's occupancy
  static int wpc[64] = {};
  int dev = 0;
  LOR_HIP(hipGetDevice(&dev));
  if (dev >= 0 && dev < 64 && wpc[dev] == 0) {
    int n = 0;
    LOR_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_nd_owner<P, T, R, M>, 64, 0));
    wpc[dev] = n > 0 ? n : 1;
  }
  const int64_t slots = static_cast<int64_t>(num_cus_nd()) * ((dev >= 0 && dev < 64) ? wpc[dev] : 1);
  const int64_t tiles = static_cast<int64_t>(nt1) * nt2;
  int64_t seglen = L[M], best = -1;
  for (int64_t len = 1; len <= L[M]; ++len) {
    const int64_t ns = ceil_div(L[M], len);
    if (ns > 1 && ceil_div(L[M], ns) != len) continue;  // same split as a shorter length
    const int64_t cost = ceil_div(tiles * ns * batch, slots) * len;
    if (best < 0 || cost < best) {
      best = cost;
      seglen = len;
    }
  }
  const int nseg = static_cast<int>(ceil_div(L[M], seglen));
  dim3 grid(static_cast<unsigned>(tiles), static_cast<unsigned>(nseg), static_cast<unsigned>(batch));
  k_nd_owner<P, T, R, M><<<grid, 64, 0, st>>>(nex, ney, nez, nt1, static_cast<int>(seglen),
                                             dev_at<int32_t>(s, s->off_elem3d), elem_dofs, elem_edges, coords,
                                             static_cast<const T*>(kappa), static_cast<T>(beta), row_ptr, s->nel,
                                             s->nnz, static_cast<T*>(values), flags, static_cast<R>(thr), diag);
  LOR_LAUNCHED("k_nd_owner");
  return LOR_OK;
}

template <int P, typename T, typename R>
static int launch_nd_owner(const lor_sched* s, int batch, const int32_t* ed, const int32_t* em, const double* x,
                           const void* k, double beta, const int32_t* rp, void* v, unsigned f, double thr,
                           int32_t* diag, hipStream_t st) {
  int rc = launch_nd_owner_dir<P, T, R, 0>(s, batch, ed, em, x, k, beta, rp, v, f, thr, diag, st);
  if (rc) return rc;
  rc = launch_nd_owner_dir<P, T, R, 1>(s, batch, ed, em, x, k, beta, rp, v, f, thr, diag, st);
  if (rc) return rc;
  return launch_nd_owner_dir<P, T, R, 2>(s, batch, ed, em, x, k, beta, rp, v, f, thr, diag, st);
}

template <typename T, typename R>
int dispatch_nd_owner(int p, const lor_sched* s, int batch, const int32_t* ed, const int32_t* em, const double* x,
                      const void* k, double beta, const int32_t* rp, void* v, unsigned f, double thr, int32_t* diag,
                      hipStream_t st) {
  if (s->box[0] < 1 || s->box[1] < 1 || s->box[2] < 1 ||
      static_cast<int64_t>(s->box[0]) * s->box[1] * s->box[2] != s->nel)
    LOR_FAIL(LOR_EINVAL, "schedule has no edge lattice");
  switch (p) {
    case 1: return launch_nd_owner<1, T, R>(s, batch, ed, em, x, k, beta, rp, v, f, thr, diag, st);
    case 2: return launch_nd_owner<2, T, R>(s, batch, ed, em, x, k, beta, rp, v, f, thr, diag, st);
    case 3: return launch_nd_owner<3, T, R>(s, batch, ed, em, x, k, beta, rp, v, f, thr, diag, st);
    case 4: return launch_nd_owner<4, T, R>(s, batch, ed, em, x, k, beta, rp, v, f, thr, diag, st);
    case 5: return launch_nd_owner<5, T, R>(s, batch, ed, em, x, k, beta, rp, v, f, thr, diag, st);
    case 6: return launch_nd_owner<6, T, R>(s, batch, ed, em, x, k, beta, rp, v, f, thr, diag, st);
    default: LOR_FAIL(LOR_EUNSUPPORTED, "lor_assemble_nd: p = %d not supported", p);
  }
}

template int dispatch_nd_owner<double, double>(int, const lor_sched*, int, const int32_t*, const int32_t*,
                                               const double*, const void*, double, const int32_t*, void*, unsigned,
                                               double, int32_t*, hipStream_t);
template int dispatch_nd_owner<float, float>(int, const lor_sched*, int, const int32_t*, const int32_t*, const double*,
                                             const void*, double, const int32_t*, void*, unsigned, double, int32_t*,
                                             hipStream_t);

}  // namespace lor
