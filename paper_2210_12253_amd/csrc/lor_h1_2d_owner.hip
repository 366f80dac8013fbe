// Values of the 2D LOR H1 matrix, owner-computes form (the 2D variant of
// Step S1.2: every row summed once, on the chip, and stored once, whole).
//
// On a 2D box lattice (the pattern call checks that the mesh is one: lattice
// point (X, Y) of the LX x LY points has vertex id X + LX Y, its row starts
// at the closed form below, and cell (X, Y) belongs to element
// elem2d[(Y / p) nx + X / p] at local subelement (X % p, Y % p)):
//
//   * one wave = one worker.  It takes a strip of 64 cells along x (strips
//     overlap by one cell, stride 63) and marches along y over a segment of
//     cell rows, one row per step;
//   * lane x integrates cell (x0 + x, Y) (10 unique entries of the Q1 cell
//     matrix) into the wave's LDS slab;
//   * lane x then sums row (x0 + x, Y) of the lower lattice line: the carry
//     (the corners b = 1 of the cells of row Y - 1, kept in registers) first,
//     then the corners b = 0 of the cells at lanes x - a, a = 0 then 1; the
//     corners b = 1 of this row's cells are the next carry.  So an entry
//     (i, j) takes the cells holding both in the same order from row i and
//     from row j, and the matrix is bitwise symmetric;
//   * the finished rows of the line are consecutive rows of the matrix: they
//     are staged in LDS and stored as one contiguous span.
// A segment that starts above the bottom first integrates the row below it
// to build the carry; the topmost segment ends with the top line, whose rows
// only hold the carry.  All sums are FP64, in the FP32 form too (each
// finished entry is rounded once).  The loads of a step (the upper line's
// corners, the element and then its coefficient) are issued one or two steps
// ahead: the element-to-coefficient chain would otherwise put two memory
// latencies on every step.
#include "lor_common.hpp"
#include "lor_h1_2d_math.hpp"

namespace lor {

constexpr int kOwn2Strip = 64;                     // cells per strip (one wave)
constexpr int kOwn2Stride = kOwn2Strip - 1;         // strips overlap by one cell
constexpr int kOwn2SpanMax = kOwn2Strip * 9;        // entries of one line's span at most
constexpr int kOwn2SpanIters = kOwn2SpanMax / 64;   // store instructions per lane

// Row-pointer closed form of the 2D lattice pattern: a point has 1 + [X > 0]
// + [X < L - 1] neighbours along an axis; the row of (X, Y) holds the in-box
// points of its 3 x 3 neighbourhood in (dy, dx) order.
__host__ __device__ __forceinline__ int64_t box2d_row_start(int64_t X, int64_t Y, int64_t LX, int64_t LY) {
  return box_prefix(Y, LY) * (3 * LX - 2) + box_count(Y, LY) * box_prefix(X, LX);
}

// Registers for four waves per SIMD (128 VGPRs): the FP64 form needs 126;
// the FP32 form would take 146 (three waves) with its FP64 fallback inlined,
// and at 128 keeps a few loop-invariant values in scratch (stored once,
// reloaded per step), which costs less than the fourth wave gains.
template <int P, typename T, typename R>
__global__ __launch_bounds__(64, 4) void k_h1_2d_owner(int nex, int ney, int seglen, const int32_t* __restrict__ elem2d,
                                                   const double* __restrict__ coords, const T* __restrict__ kappa,
                                                   T beta, int64_t nel, int64_t nnz, T* __restrict__ values,
                                                   unsigned flags, R det_thresh, int32_t* __restrict__ diag) {
  constexpr int NSUB = P * P;
  __shared__ R sCell[10 * 64];        // cell matrices [pair][lane]
  __shared__ T sStg[kOwn2SpanMax];    // the finished rows of the line, in CSR order

  const int NXc = nex * P, NYc = ney * P;
  const int LX = NXc + 1, LY = NYc + 1;
  const int lane = threadIdx.x;
  const int ti = blockIdx.x;
  const int x0 = kOwn2Stride * ti;
  const int ys = blockIdx.y * seglen;
  const int ye = ys + seglen < NYc ? ys + seglen : NYc;
  kappa += static_cast<int64_t>(blockIdx.z) * nel * NSUB;
  values += static_cast<int64_t>(blockIdx.z) * nnz;

  const int X = x0 + lane;
  const bool cell_in = X < NXc;
  const bool row_own = X <= NXc && (lane > 0 || ti == 0);
  const int Xc = cell_in ? X : NXc - 1;         // clamped cell column (reads only)
  const int X1 = X + 1 <= NXc ? X + 1 : NXc;    // clamped right corner column
  const int X0 = X <= NXc ? X : NXc;

  const int yfirst = ys > 0 ? ys - 1 : ys;     // a segment above the bottom starts one row lower
  const int yend = ye == NYc ? NYc + 1 : ye;   // the top segment also writes the top line

  // corners (X, Y') and (X + 1, Y') of line Y' (clamped to the lattice)
  auto load_line = [&](int Yl, double(&c)[2][2]) {
    const int64_t r = static_cast<int64_t>(Yl <= NYc ? Yl : NYc) * LX;
#pragma unroll
    for (int d = 0; d < 2; ++d) {
      c[0][d] = coords[2 * (r + X0) + d];
      c[1][d] = coords[2 * (r + X1) + d];
    }
  };
  // element of this lane's cell in row Y' and its coefficient (clamped)
  auto load_elem = [&](int Yl) {
    const int yc = Yl < NYc ? Yl : NYc - 1;
    return elem2d[static_cast<int64_t>(yc / P) * nex + Xc / P];
  };
  auto load_kap = [&](int Yl, int32_t el) {
    const int yc = Yl < NYc ? Yl : NYc - 1;
    return kappa[static_cast<int64_t>(el) * NSUB + (Xc % P) + P * (yc % P)];
  };
  // pipeline: the step of row Y holds the lines Y and Y + 1 and the
  // coefficient of row Y, and has the element of row Y + 1
  double lo[2][2], hi[2][2];
  load_line(yfirst, lo);
  load_line(yfirst + 1, hi);
  int32_t el1 = load_elem(yfirst);
  T kq = load_kap(yfirst, el1);
  el1 = load_elem(yfirst + 1);
  double carry[6];  // (dy, dx) = (-1, -1 .. 1), (0, -1 .. 1) of the row on the next line
#pragma unroll
  for (int o = 0; o < 6; ++o) carry[o] = 0.0;

  // the lines of the strip: rows from xa on, the last one xlast
  const int xa = x0 + (ti == 0 ? 0 : 1);
  const int xlast = x0 + kOwn2Stride < NXc ? x0 + kOwn2Stride : NXc;
  const int64_t pxa = box_prefix(xa, LX);
  const int64_t span_x = box_prefix(xlast + 1, LX) - pxa;
  const int xlo = X > 0, xhi = X < NXc, nx = 1 + xlo + xhi;
  const int64_t before_x = box_prefix(X0, LX) - pxa;

  for (int Y = yfirst; Y < yend; ++Y) {
    const bool cells = cell_in && Y < NYc;
    double hn[2][2];
    load_line(Y + 2, hn);
    const T kn = load_kap(Y + 1, el1);
    const int32_t el2 = load_elem(Y + 2);
    if (cells) {
      const R kap = static_cast<R>(kq);
      // edges in FP64: e_b along x at y = b, f_a along y at x = a
      double e64[2][2], f64[2][2];
#pragma unroll
      for (int d = 0; d < 2; ++d) {
        e64[0][d] = lo[1][d] - lo[0][d];
        e64[1][d] = hi[1][d] - hi[0][d];
        f64[0][d] = hi[0][d] - lo[0][d];
        f64[1][d] = hi[1][d] - lo[1][d];
      }
      // counted once: the last cell of a strip is the first of the next
      const bool own = Y >= ys && lane < kOwn2Stride;
      bool fallback = false;
      if constexpr (!std::is_same<R, double>::value) {
        if (flags & LOR_FP64_FALLBACK) {
          R dmin = R(3.0e38), dmax = R(-3.0e38);
#pragma unroll
          for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int a = 0; a < 2; ++a) {
              const R dd = R(e64[b][0]) * R(f64[a][1]) - R(e64[b][1]) * R(f64[a][0]);
              dmin = dd < dmin ? dd : dmin;
              dmax = dd > dmax ? dd : dmax;
            }
          fallback = !(dmin > R(0)) || dmax > det_thresh * dmin;
        }
      }
      R ent[10];
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
        if (!ok && own && diag) atomicAdd(&diag[1], 1);
      } else {
        double d10[10];
        const bool ok = q1_2d_entries<double>(e64, f64, static_cast<double>(kap), static_cast<double>(beta), d10);
#pragma unroll
        for (int k = 0; k < 10; ++k) ent[k] = static_cast<R>(d10[k]);
        if (own && diag) {
          atomicAdd(&diag[0], 1);
          if (!ok) atomicAdd(&diag[1], 1);
        }
      }
#pragma unroll
      for (int k = 0; k < 10; ++k) sCell[k * 64 + lane] = ent[k];
    }
    __syncthreads();

    // row (X, Y): the carry, then this row's cells at lanes x - a (their
    // corner (a, 0) is this row's point); their corners (a, 1) go to the
    // next carry.  Entry index (dx + 1) + 3 (dy + 1).
    double acc[9];
#pragma unroll
    for (int o = 0; o < 9; ++o) acc[o] = o < 6 ? carry[o] : 0.0;
#pragma unroll
    for (int o = 0; o < 6; ++o) carry[o] = 0.0;
    if (Y < NYc && X <= NXc) {
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const int sx = lane - a;
        if (sx >= 0 && x0 + sx < NXc) {
          const R* cm = sCell + sx;
          const int u0 = a, u1 = a + 2;  // this point as the cell's corner (a, 0) and (a, 1)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int dx = (v & 1) - a, dy = v >> 1;
            acc[(dx + 1) + 3 * (dy + 1)] += static_cast<double>(cm[pair_index4(u0, v) * 64]);
            carry[(dx + 1) + 3 * dy] += static_cast<double>(cm[pair_index4(u1, v) * 64]);
          }
        }
      }
    }
    // the next row's lines, coefficient and element
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int d = 0; d < 2; ++d) {
        lo[c][d] = hi[c][d];
        hi[c][d] = hn[c][d];
      }
    kq = kn;
    el1 = el2;
    if (Y < ys) {  // the row below the segment: carry only
      __syncthreads();
      continue;
    }

    // stage the owned rows of line Y in CSR order: cy y-offsets per row,
    // nx x-offsets per row, (dy, dx) order
    const int ylo = Y > 0, yhi = Y < NYc, cy = 1 + ylo + yhi;
    __syncthreads();  // every lane is done reading the slab (the staging buffer is separate)
    if (row_own) {
      T* row = sStg + before_x * cy + ylo * nx + xlo;
#pragma unroll
      for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
          const bool ok = (dx >= 0 || xlo) && (dx <= 0 || xhi) && (dy >= 0 || ylo) && (dy <= 0 || yhi);
          if (ok) row[dy * nx + dx] = static_cast<T>(acc[(dx + 1) + 3 * (dy + 1)]);
        }
    }
    __syncthreads();
    const int64_t start = box2d_row_start(xa, Y, LX, LY);
    const int span = static_cast<int>(span_x * cy);
    T* dst = values + start;
#pragma unroll
    for (int it = 0; it < kOwn2SpanIters; ++it) {
      const int t = lane + 64 * it;
      if (t < span) dst[t] = sStg[t];
    }
    __syncthreads();  // the staging buffer is rewritten by the next line
  }
}

static int num_cus_2do() {
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
static int launch_2d_owner(const lor_sched* s, int batch, const double* coords, const void* kappa, double beta,
                           void* values, unsigned flags, double thr, int32_t* diag, hipStream_t st) {
  const int nex = s->box[0], ney = s->box[1];
  const int NXc = nex * P, NYc = ney * P;
  const int ntx = static_cast<int>(ceil_div(NXc, kOwn2Stride));
  // segments along y: about 4 waves per SIMD over the chip, at least 8 cell
  // rows each (a segment integrates one extra row to build its carry)
  const int64_t target = int64_t(4) * 4 * num_cus_2do();
  int seglen = static_cast<int>(ceil_div(static_cast<int64_t>(NYc) * ntx * batch, target));
  if (seglen < 8) seglen = 8;
  if (seglen > NYc) seglen = NYc;
  const int nseg = static_cast<int>(ceil_div(NYc, seglen));
  dim3 grid(static_cast<unsigned>(ntx), static_cast<unsigned>(nseg), static_cast<unsigned>(batch));
  k_h1_2d_owner<P, T, R><<<grid, 64, 0, st>>>(nex, ney, seglen, dev_at<int32_t>(s, s->off_elem3d), coords,
                                             static_cast<const T*>(kappa), static_cast<T>(beta), s->nel, s->nnz,
                                             static_cast<T*>(values), flags, static_cast<R>(thr), diag);
  LOR_LAUNCHED("k_h1_2d_owner");
  return LOR_OK;
}

template <typename T, typename R>
int dispatch_2d_owner(int p, const lor_sched* s, int batch, const double* x, const void* k, double beta, void* v,
                      unsigned f, double thr, int32_t* diag, hipStream_t st) {
  if (s->box[0] < 1 || s->box[1] < 1 || static_cast<int64_t>(s->box[0]) * s->box[1] != s->nel)
    LOR_FAIL(LOR_EINVAL, "schedule has no 2D box lattice");
  switch (p) {
    case 1: return launch_2d_owner<1, T, R>(s, batch, x, k, beta, v, f, thr, diag, st);
    case 2: return launch_2d_owner<2, T, R>(s, batch, x, k, beta, v, f, thr, diag, st);
    case 3: return launch_2d_owner<3, T, R>(s, batch, x, k, beta, v, f, thr, diag, st);
    case 4: return launch_2d_owner<4, T, R>(s, batch, x, k, beta, v, f, thr, diag, st);
    case 5: return launch_2d_owner<5, T, R>(s, batch, x, k, beta, v, f, thr, diag, st);
    case 6: return launch_2d_owner<6, T, R>(s, batch, x, k, beta, v, f, thr, diag, st);
    default: LOR_FAIL(LOR_EUNSUPPORTED, "lor_assemble_h1_2d: p = %d not supported", p);
  }
}

template int dispatch_2d_owner<double, double>(int, const lor_sched*, int, const double*, const void*, double, void*,
                                               unsigned, double, int32_t*, hipStream_t);
template int dispatch_2d_owner<float, float>(int, const lor_sched*, int, const double*, const void*, double, void*,
                                             unsigned, double, int32_t*, hipStream_t);

}  // namespace lor
