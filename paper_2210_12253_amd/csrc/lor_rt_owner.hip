// Values of the LOR H(div) matrix, owner-computes form (Step S1.2 for the
// lowest-order Raviart-Thomas space of Section 2.3: every row summed once, on
// the chip, and stored once, whole).
//
// On a face lattice (the pattern call checks that the mesh is one: with
// (MX, MY, MZ) cells per axis, the x-face at lattice x = X bounding cell row
// (Y, Z) has id X + (MX + 1)(Y + MY Z), the y-faces and z-faces follow at
// OY = (MX + 1) MY MZ and OZ = OY + MX (MY + 1) MZ in the same way, the
// element at every box position is known, and row_ptr matches the closed
// form below) a face row has 11 entries from the two cells it bounds (6 on
// the boundary of the box):
//
//   * one wave takes a tile of 8 x 8 cells in x and y (tiles overlap by one
//     cell, stride 7) and marches along z over a segment of cell layers;
//   * lane (x, y) integrates cell (X, Y, Z) (21 unique entries of its 6 x 6
//     matrix, times the orientation signs of its faces in its element's face
//     map) into the wave's LDS slab, then sums three rows: the x-face at X
//     (cells at lanes x - 1 and x), the y-face at Y (lanes y - 8 and y) and
//     the z-face at Z (the cell below, carried in registers from the previous
//     step, then this cell);
//   * every row type's finished rows of a line (X consecutive) are
//     consecutive rows of the matrix: staged in LDS and stored as one span.
//
// Two distinct faces share at most one cell, so every off-diagonal entry has
// one term and the matrix is bitwise symmetric; a diagonal entry takes its
// two cells in a fixed order.  All sums are FP64, in the FP32 form too.  The
// cell corners are gathered through the vertex map (the vertex numbering can
// be anything), the element and its coefficient through the element grid.
#include <algorithm>

#include "lor_common.hpp"
#include "lor_rt_math.hpp"

namespace lor {

constexpr int kRtTile = 8;               // cells per tile side (one wave: 8 x 8)
constexpr int kRtStride = kRtTile - 1;   // tiles overlap by one cell
constexpr int kRtLine = kRtTile * 11;    // entries of one staged line at most
constexpr int kRtLineIters = (kRtLine + 63) / 64;

// Entries before face X of a row of faces 0 .. M (the faces at 0 and M have 6
// entries, the others 11), X in [0, M + 1].
__host__ __device__ __forceinline__ int64_t rt_prefix(int64_t X, int64_t M) {
  if (X <= 0) return 0;
  if (X <= M) return 6 + 11 * (X - 1);
  return 12 + 11 * (M - 1);
}
__host__ __device__ __forceinline__ int rt_len(int64_t X, int64_t M) { return (X == 0 || X == M) ? 6 : 11; }

// Row starts of the face-lattice pattern (x-face rows, then y-face rows, then
// z-face rows, each in face-id order).
struct RtLattice {
  int64_t MX, MY, MZ;
  __host__ __device__ int64_t nnz_x() const { return MY * MZ * rt_prefix(MX + 1, MX); }
  __host__ __device__ int64_t nnz_y() const { return MZ * MX * rt_prefix(MY + 1, MY); }
  __host__ __device__ int64_t row_x(int64_t X, int64_t Y, int64_t Z) const {
    return (Y + MY * Z) * rt_prefix(MX + 1, MX) + rt_prefix(X, MX);
  }
  __host__ __device__ int64_t row_y(int64_t X, int64_t Y, int64_t Z) const {
    return nnz_x() + Z * MX * rt_prefix(MY + 1, MY) + MX * rt_prefix(Y, MY) + X * rt_len(Y, MY);
  }
  __host__ __device__ int64_t row_z(int64_t X, int64_t Y, int64_t Z) const {
    return nnz_x() + nnz_y() + MX * MY * rt_prefix(Z, MZ) + (X + MX * Y) * rt_len(Z, MZ);
  }
};

// Positions in an 11-entry row of the 6 faces (x-, x+, y-, y+, z-, z+) of the
// cell before the row's face along its axis ("lo") and of the cell after it
// ("hi"); a row with one cell keeps its 6 entries in the cell's face order.
// x-row: [x: X-1, X, X+1] [y: (Y, X-1), (Y, X), (Y+1, X-1), (Y+1, X)] [z: (Z, X-1), (Z, X), (Z+1, X-1), (Z+1, X)]
// y-row: [x: (Y-1, X), (Y-1, X+1), (Y, X), (Y, X+1)] [y: Y-1, Y, Y+1] [z: (Z, Y-1), (Z, Y), (Z+1, Y-1), (Z+1, Y)]
// z-row: [x: (Z-1, X), (Z-1, X+1), (Z, X), (Z, X+1)] [y: (Z-1, Y), (Z-1, Y+1), (Z, Y), (Z, Y+1)] [z: Z-1, Z, Z+1]
__host__ __device__ constexpr int rt_pos(int axis, int hi, int v) {
  constexpr int P[3][2][6] = {{{0, 1, 3, 5, 7, 9}, {1, 2, 4, 6, 8, 10}},
                              {{0, 1, 4, 5, 7, 9}, {2, 3, 5, 6, 8, 10}},
                              {{0, 1, 4, 5, 8, 9}, {2, 3, 6, 7, 9, 10}}};
  return P[axis][hi][v];
}

// FP32 form, strongly distorted cell: the FP64 integration from the FP64
// corners (gathered again through the vertex map; lv0 is the local vertex of
// corner 0), entries signed by negmask (bit u: face u reversed) and rounded
// to FP32 into the slab (64 = distance between two entries of a cell).
template <int P>
__device__ __noinline__ bool rt_owner_fp64_fallback(const int32_t* __restrict__ elem_dofs,
                                                    const double* __restrict__ coords, int32_t el, int lv0, double kap,
                                                    double bet, unsigned negmask, float* out) {
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
  RTFactors<double> F;
  const bool ok = rt_factors<double>(ex, ey, ez, kap, bet, F);
#pragma unroll
  for (int u = 0; u < 6; ++u)
#pragma unroll
    for (int v = u; v < 6; ++v) {
      const float e = static_cast<float>(rt_entry<double>(F, u, v));
      out[pair_index6(u, v) * 64] = (((negmask >> u) ^ (negmask >> v)) & 1u) ? -e : e;
    }
  return ok;
}

template <int P, typename T, typename R>
__global__ __launch_bounds__(64) void k_rt_owner(int nex, int ney, int nez, int ntx, int seglen,
                                                const int32_t* __restrict__ elem3d,
                                                const int32_t* __restrict__ elem_dofs,
                                                const int32_t* __restrict__ elem_faces,
                                                const double* __restrict__ coords, const T* __restrict__ kappa, T beta,
                                                int64_t nel, int64_t nnz, T* __restrict__ values, unsigned flags,
                                                R det_thresh, int32_t* __restrict__ diag) {
  constexpr int Q = P + 1, NSUB = P * P * P, NLOCV = Q * Q * Q, NLOCF = 3 * P * P * Q;
  __shared__ R sCell[21 * 64];                 // cell matrices [pair][lane]
  __shared__ T sStg[kRtTile * kRtLine];        // one row type's finished lines

  const int MX = nex * P, MY = ney * P, MZ = nez * P;
  const RtLattice lat{MX, MY, MZ};
  const int lane = threadIdx.x;
  const int ti = blockIdx.x % ntx, tj = blockIdx.x / ntx;
  const int x0 = kRtStride * ti, y0 = kRtStride * tj;
  const int zs = blockIdx.y * seglen;
  const int ze = zs + seglen < MZ ? zs + seglen : MZ;
  kappa += static_cast<int64_t>(blockIdx.z) * nel * NSUB;
  values += static_cast<int64_t>(blockIdx.z) * nnz;

  const int lx = lane & 7, ly = lane >> 3;
  const int X = x0 + lx, Y = y0 + ly;
  const bool cell_col = X < MX && Y < MY;  // this lane's cell column exists
  const int Xc = X < MX ? X : MX - 1, Yc = Y < MY ? Y : MY - 1;

  const int zfirst = zs > 0 ? zs - 1 : zs;  // a segment above the bottom starts one layer lower
  const int zend = ze == MZ ? MZ + 1 : ze;  // the top segment also writes the top z-faces

  // owned rows: x-faces X in [xa, xe], y-faces Y in [ya, ye] (X a cell
  // column), z-faces of the cell columns [xca, xce] x [yca, yce]
  const int xa = x0 + (ti > 0), xe = x0 + kRtStride < MX ? x0 + kRtStride : MX;
  const int ya = y0 + (tj > 0), ye2 = y0 + kRtStride < MY ? y0 + kRtStride : MY;
  const int xce = x0 + kRtStride < MX - 1 ? x0 + kRtStride : MX - 1;
  const int yce = y0 + kRtStride < MY - 1 ? y0 + kRtStride : MY - 1;

  double carry[6];  // z+ row of the cell below (at the "lo" positions of the z-row)
#pragma unroll
  for (int v = 0; v < 6; ++v) carry[v] = 0.0;

  // Loads of the cell column, layer Zl clamped to the mesh (a lane without a
  // cell reads the last one and never uses it).
  const int sx = Xc % P, sy = Yc % P;
  auto elem_of = [&](int Zl) {
    const int zc = Zl < MZ ? Zl : MZ - 1;
    return elem3d[(static_cast<int64_t>(zc / P) * ney + Yc / P) * nex + Xc / P];
  };
  // vertex ids of the 4 corners of the cell of layer Zl on its lower (c = 0)
  // or upper (c = 1) face, corner a + 2 b
  auto corner_ids = [&](int32_t el, int Zl, int c, int32_t(&ids)[4]) {
    const int sz = (Zl < MZ ? Zl : MZ - 1) % P + c;
#pragma unroll
    for (int v = 0; v < 4; ++v)
      ids[v] = elem_dofs[static_cast<int64_t>(el) * NLOCV + (sx + (v & 1)) + Q * ((sy + (v >> 1)) + Q * sz)];
  };
  auto corner_xyz = [&](const int32_t(&ids)[4], double(&c)[4][3]) {
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int d = 0; d < 3; ++d) c[v][d] = coords[3 * static_cast<int64_t>(ids[v]) + d];
  };
  // the face-map words of the cell's faces x-, x+, y-, y+, z-, z+ (local face
  // numbering of the element: x-faces i + q (j + p k), y-faces
  // p^2 q + i + p (j + q k), z-faces 2 p^2 q + i + p (j + p k)); their signs
  // are the orientations
  auto face_words = [&](int32_t el, int Zl, int32_t(&fw)[6]) {
    const int sz = (Zl < MZ ? Zl : MZ - 1) % P;
    const int32_t* fm = elem_faces + static_cast<int64_t>(el) * NLOCF;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      fw[0 + t] = fm[(sx + t) + Q * (sy + P * sz)];
      fw[2 + t] = fm[P * P * Q + sx + P * ((sy + t) + Q * sz)];
      fw[4 + t] = fm[2 * P * P * Q + sx + P * (sy + P * (sz + t))];
    }
  };
  auto kap_of = [&](int32_t el, int Zl) {
    const int sz = (Zl < MZ ? Zl : MZ - 1) % P;
    return kappa[static_cast<int64_t>(el) * NSUB + sx + P * (sy + P * sz)];
  };

  // Pipeline: the step of layer Z holds the corners of its cell (lower =
  // upper of the cell below), its face words and coefficient, the element
  // of layer Z + 1 and the upper-corner ids of the cell of layer Z + 1.  It
  // loads, before its integration, the face words and coefficient of the next
  // cell and the element two layers up, and after it the next cell's upper
  // corners and the upper-corner ids of the cell after that, so that no step
  // waits on a chain of dependent loads (and the integration, the register
  // peak, holds no prefetched corners).
  double lo[4][3], hi[4][3];
  int32_t fw[6], idn[4];
  T kq;
  int32_t el1, elc;  // elements of layers Z + 1 and Z
  {
    const int32_t el0 = elem_of(zfirst);
    elc = el0;
    int32_t ids[4];
    corner_ids(el0, zfirst, 0, ids);
    corner_xyz(ids, lo);
    corner_ids(el0, zfirst, 1, ids);
    corner_xyz(ids, hi);
    face_words(el0, zfirst, fw);
    kq = kap_of(el0, zfirst);
    el1 = elem_of(zfirst + 1);
    corner_ids(el1, zfirst + 1, 1, idn);
  }

  for (int Z = zfirst; Z < zend; ++Z) {
    const bool cell = cell_col && Z < MZ;
    int32_t fwn[6];
    face_words(el1, Z + 1, fwn);
    const T kn = kap_of(el1, Z + 1);
    const int32_t el2 = elem_of(Z + 2);
    if (cell) {
      const R kap = static_cast<R>(kq);
      double Xv[8][3];
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          Xv[v][d] = lo[v][d];
          Xv[4 + v][d] = hi[v][d];
        }
      bool neg[6];
#pragma unroll
      for (int u = 0; u < 6; ++u) neg[u] = fw[u] < 0;
      // counted once: a cell in a tile's last column (row) is the first of
      // the next tile, which counts it
      const bool own = Z >= zs && lx < kRtStride && ly < kRtStride;
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
        RTFactors<R> F;
        const bool ok = rt_factors<R>(ex, ey, ez, kap, static_cast<R>(beta), F);
#pragma unroll
        for (int u = 0; u < 6; ++u)
#pragma unroll
          for (int v = u; v < 6; ++v) {
            const R e = rt_entry<R>(F, u, v);
            sCell[pair_index6(u, v) * 64 + lane] = (neg[u] != neg[v]) ? -e : e;
          }
        if (!ok && own && diag) atomicAdd(&diag[1], 1);
      } else {
        // FP32 only, rare: FP64 geometry and quadrature out of line (inlined,
        // its FP64 registers would be reserved for the whole kernel)
        unsigned negmask = 0;
#pragma unroll
        for (int u = 0; u < 6; ++u) negmask |= neg[u] ? 1u << u : 0u;
        const bool ok = rt_owner_fp64_fallback<P>(elem_dofs, coords, elc, sx + Q * (sy + Q * (Z % P)),
                                               static_cast<double>(kap), static_cast<double>(beta), negmask,
                                               reinterpret_cast<float*>(sCell) + lane);
        if (own && diag) {
          atomicAdd(&diag[0], 1);
          if (!ok) atomicAdd(&diag[1], 1);
        }
      }
    }
    // the next cell's upper corners (their ids arrived during the
    // integration) and the ids of the one after it
    double hin[4][3];
    corner_xyz(idn, hin);
    int32_t idn2[4];
    corner_ids(el2, Z + 2, 1, idn2);
    __syncthreads();

    // the three rows of this lane, each at the interior positions; the terms
    // of a missing cell are absent (0)
    double rx[11], ry[11], rz[11];
#pragma unroll
    for (int k = 0; k < 11; ++k) {
      rx[k] = 0.0;
      ry[k] = 0.0;
      rz[k] = 0.0;
    }
#pragma unroll
    for (int v = 0; v < 6; ++v) rz[rt_pos(2, 0, v)] = carry[v];
    if (Z < MZ) {
      // x-face at X: the cell X - 1 (lane x - 1, its x+ face) then the cell X
      if (lx > 0 && X - 1 < MX && Y < MY) {
        const R* cm = sCell + lane - 1;
#pragma unroll
        for (int v = 0; v < 6; ++v) rx[rt_pos(0, 0, v)] += static_cast<double>(cm[pair_index6(1, v) * 64]);
      }
      if (cell) {
#pragma unroll
        for (int v = 0; v < 6; ++v)
          rx[rt_pos(0, 1, v)] += static_cast<double>(sCell[pair_index6(0, v) * 64 + lane]);
      }
      // y-face at Y: the cell Y - 1 (lane y - 1, its y+ face) then the cell Y
      if (ly > 0 && X < MX && Y - 1 < MY) {
        const R* cm = sCell + lane - 8;
#pragma unroll
        for (int v = 0; v < 6; ++v) ry[rt_pos(1, 0, v)] += static_cast<double>(cm[pair_index6(3, v) * 64]);
      }
      if (cell) {
#pragma unroll
        for (int v = 0; v < 6; ++v)
          ry[rt_pos(1, 1, v)] += static_cast<double>(sCell[pair_index6(2, v) * 64 + lane]);
        // z-face at Z: the carry (cell Z - 1), then this cell's z- face; its
        // z+ face is the next carry
#pragma unroll
        for (int v = 0; v < 6; ++v) {
          rz[rt_pos(2, 1, v)] += static_cast<double>(sCell[pair_index6(4, v) * 64 + lane]);
          carry[v] = static_cast<double>(sCell[pair_index6(5, v) * 64 + lane]);
        }
      }
    }
    __syncthreads();
    // the next layer's cell: its lower corners are this cell's upper ones
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        lo[v][d] = hi[v][d];
        hi[v][d] = hin[v][d];
      }
#pragma unroll
    for (int u = 0; u < 6; ++u) fw[u] = fwn[u];
#pragma unroll
    for (int v = 0; v < 4; ++v) idn[v] = idn2[v];
    kq = kn;
    elc = el1;
    el1 = el2;
    if (Z < zs) continue;  // the layer below the segment: carry only

    // stage and store one row type at a time: line l of the tile holds the
    // owned rows of that line in face-id order (X consecutive)
    for (int axis = 0; axis < 3; ++axis) {
      // this lane's row of this type, its line and its first owned row
      bool mine;
      int len, before, first, last;
      if (axis == 0) {  // x-face (X, Y, Z): Y < MY, Z < MZ, X in [xa, xe]
        mine = Z < MZ && Y < MY && ly >= (tj > 0) && X >= xa && X <= xe;
        len = rt_len(X, MX);
        before = static_cast<int>(rt_prefix(X, MX) - rt_prefix(xa, MX));
        first = xa;
        last = xe;
      } else if (axis == 1) {  // y-face (X, Y, Z): X a cell column, Y in [ya, ye2], Z < MZ
        mine = Z < MZ && X < MX && lx >= (ti > 0) && X <= xce && Y >= ya && Y <= ye2;
        len = rt_len(Y, MY);
        before = (X - xa) * len;
        first = xa;
        last = xce;
      } else {  // z-face (X, Y, Z): a cell column, Z <= MZ
        mine = X < MX && Y < MY && lx >= (ti > 0) && ly >= (tj > 0) && X <= xce && Y <= yce;
        len = rt_len(Z, MZ);
        before = (X - xa) * len;
        first = xa;
        last = xce;
      }
      if (mine) {
        const double* r = axis == 0 ? rx : axis == 1 ? ry : rz;
        T* dst = sStg + kRtLine * ly + before;
        const int A = axis == 0 ? X : axis == 1 ? Y : Z;
        const int M = axis == 0 ? MX : axis == 1 ? MY : MZ;
        if (A > 0 && A < M) {
#pragma unroll
          for (int k = 0; k < 11; ++k) dst[k] = static_cast<T>(r[k]);
        } else if (A == 0) {  // only the cell after the face
#pragma unroll
          for (int v = 0; v < 6; ++v) dst[v] = static_cast<T>(r[rt_pos(axis, 1, v)]);
        } else {  // only the cell before it
#pragma unroll
          for (int v = 0; v < 6; ++v) dst[v] = static_cast<T>(r[rt_pos(axis, 0, v)]);
        }
      }
      __syncthreads();
      // line l: the rows [first, last] of line y0 + l (the same for every lane)
#pragma unroll
      for (int l = 0; l < kRtTile; ++l) {
        const int Yl = y0 + l;
        bool line;
        int64_t ls = 0;
        int span = 0;
        if (axis == 0) {
          line = Z < MZ && Yl < MY && (l > 0 || tj == 0);
          if (line) {
            ls = lat.row_x(first, Yl, Z);
            span = static_cast<int>(rt_prefix(last + 1, MX) - rt_prefix(first, MX));
          }
        } else if (axis == 1) {
          line = Z < MZ && Yl <= MY && (l > 0 || tj == 0) && last >= first;
          if (line) {
            ls = lat.row_y(first, Yl, Z);
            span = (last - first + 1) * rt_len(Yl, MY);
          }
        } else {
          line = Yl < MY && (l > 0 || tj == 0) && last >= first;
          if (line) {
            ls = lat.row_z(first, Yl, Z);
            span = (last - first + 1) * rt_len(Z, MZ);
          }
        }
        T* dst = values + ls;
#pragma unroll
        for (int it = 0; it < kRtLineIters; ++it) {
          const int t = lane + 64 * it;
          if (t < span) dst[t] = sStg[kRtLine * l + t];
        }
      }
      __syncthreads();
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
static int launch_rt_owner(const lor_sched* s, int batch, const int32_t* elem_dofs, const int32_t* elem_faces,
                           const double* coords, const void* kappa, double beta, void* values, unsigned flags,
                           double thr, int32_t* diag, hipStream_t st) {
  const int nex = s->box[0], ney = s->box[1], nez = s->box[2];
  const int MX = nex * P, MY = ney * P, MZ = nez * P;
  // tiles so that the last one reaches the last face: 7 (ntx - 1) + 7 >= MX
  const int ntx = static_cast<int>(ceil_div(MX, kRtStride)), nty = static_cast<int>(ceil_div(MY, kRtStride));
  // Segments along z (a segment above the bottom integrates one extra layer
  // to build its carry).  The waves run in rounds over the chip's wave slots
  // (CUs x resident waves per CU, from the kernel's register use), so the
  // launch takes about ceil(waves / slots) x (layers per wave + 1) layer
  // steps: pick the segment length that minimises it.
  static int wpc[64] = {};
  int dev = 0;
  LOR_HIP(hipGetDevice(&dev));
  if (dev >= 0 && dev < 64 && wpc[dev] == 0) {
    int n = 0;
    LOR_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_rt_owner<P, T, R>, 64, 0));
    wpc[dev] = n > 0 ? n : 1;
  }
  const int64_t slots = static_cast<int64_t>(num_cus_rt()) * ((dev >= 0 && dev < 64) ? wpc[dev] : 1);
  const int64_t tiles = static_cast<int64_t>(ntx) * nty;
  int64_t seglen = MZ, best = -1;
  for (int64_t len = std::min<int64_t>(2, MZ); len <= MZ; ++len) {
    const int64_t ns = ceil_div(MZ, len);
    if (ns > 1 && ceil_div(MZ, ns) != len) continue;  // same split as a shorter length
    const int64_t cost = ceil_div(tiles * ns * batch, slots) * (len + (ns > 1));
    if (best < 0 || cost < best) {
      best = cost;
      seglen = len;
    }
  }
  const int nseg = static_cast<int>(ceil_div(MZ, seglen));
  dim3 grid(static_cast<unsigned>(ntx * nty), static_cast<unsigned>(nseg), static_cast<unsigned>(batch));
  k_rt_owner<P, T, R><<<grid, 64, 0, st>>>(nex, ney, nez, ntx, static_cast<int>(seglen), dev_at<int32_t>(s, s->off_elem3d), elem_dofs,
                                          elem_faces, coords, static_cast<const T*>(kappa), static_cast<T>(beta),
                                          s->nel, s->nnz, static_cast<T*>(values), flags, static_cast<R>(thr), diag);
  LOR_LAUNCHED("k_rt_owner");
  return LOR_OK;
}

template <typename T, typename R>
int dispatch_rt_owner(int p, const lor_sched* s, int batch, const int32_t* ed, const int32_t* fm, const double* x,
                      const void* k, double beta, void* v, unsigned f, double thr, int32_t* diag, hipStream_t st) {
  if (s->box[0] < 1 || s->box[1] < 1 || s->box[2] < 1 ||
      static_cast<int64_t>(s->box[0]) * s->box[1] * s->box[2] != s->nel)
    LOR_FAIL(LOR_EINVAL, "schedule has no face lattice");
  switch (p) {
    case 1: return launch_rt_owner<1, T, R>(s, batch, ed, fm, x, k, beta, v, f, thr, diag, st);
    case 2: return launch_rt_owner<2, T, R>(s, batch, ed, fm, x, k, beta, v, f, thr, diag, st);
    case 3: return launch_rt_owner<3, T, R>(s, batch, ed, fm, x, k, beta, v, f, thr, diag, st);
    case 4: return launch_rt_owner<4, T, R>(s, batch, ed, fm, x, k, beta, v, f, thr, diag, st);
    case 5: return launch_rt_owner<5, T, R>(s, batch, ed, fm, x, k, beta, v, f, thr, diag, st);
    case 6: return launch_rt_owner<6, T, R>(s, batch, ed, fm, x, k, beta, v, f, thr, diag, st);
    default: LOR_FAIL(LOR_EUNSUPPORTED, "lor_assemble_rt: p = %d not supported", p);
  }
}

template int dispatch_rt_owner<double, double>(int, const lor_sched*, int, const int32_t*, const int32_t*,
                                               const double*, const void*, double, void*, unsigned, double, int32_t*,
                                               hipStream_t);
template int dispatch_rt_owner<float, float>(int, const lor_sched*, int, const int32_t*, const int32_t*, const double*,
                                             const void*, double, void*, unsigned, double, int32_t*, hipStream_t);

}  // namespace lor
