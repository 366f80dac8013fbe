// Sparsity pattern and assembly schedule of the LOR matrices.
//
// Step S1.2 of the paper builds the processor-local CSR matrix of the LOR
// discretisation in two stages: A1 fills per-macro-element sparse blocks that
// share one local column pattern (computed once for the reference macro
// element), A2 counts the nonzeros of every row without double-counting the
// entries seen by several macro elements, scans the counts into the row
// pointer, then fills the columns.  This file does the integer half of that:
//
//   * reference element: the local stencil (which local dofs a local dof
//     couples to: the 27-point lattice neighbourhood for vertices, the edges
//     (faces) of the shared subelements for Nedelec edges (Raviart-Thomas
//     faces)), computed once on the host and
//     copied into the schedule -- the analogue of the shared column array J_hat;
//   * vertex/edge/face -> (element, local dof) incidence lists (transpose of the
//     element map, counting sort, each list sorted so the result is
//     deterministic);
//   * per row: the sorted union of the local stencils of every incident
//     element gives the columns (deduplicated exactly, so no entry is counted
//     twice whatever the number of elements sharing the row);
//   * exclusive scan of the counts -> row pointer;
//   * element colouring (greedy in element order, run as Jones-Plassmann
//     rounds): elements of one colour share no dof, so the value kernels can
//     add a colour's contributions without atomics and in a fixed order;
//   * per element and local stencil entry, the position of the entry inside its
//     CSR row and whether the element is the entry's first contributor.
#include <algorithm>
#include <climits>
#include <unordered_map>
#include <vector>

#include "lor_common.hpp"

namespace lor {

// ------------------------------------------------------------ device buffer

struct DevBuf {
  void* p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  int alloc(size_t bytes) {
    if (bytes == 0) bytes = 16;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
      p = nullptr;
      set_error("hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
      return LOR_EDEVICE;
    }
    return LOR_OK;
  }
  template <typename T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

// ---------------------------------------------------------- reference element

struct RefElem {
  int nloc = 0, nent = 0;
  std::vector<int32_t> st_ptr, st_col;
  std::vector<uint16_t> ent_row;  // local row of every compact stencil entry
  std::vector<int32_t> reps;    // local dofs whose incidences give element adjacency
  std::vector<uint64_t> recipe64;  // Nedelec: per compact entry, subelement contributions
};

static int nd_local(int p, int ax, int i, int j, int k) {
  const int q = p + 1;
  if (ax == 0) return i + p * (j + q * k);
  if (ax == 1) return p * q * q + i + q * (j + p * k);
  return 2 * p * q * q + i + q * (j + q * k);
}

// The 12 local edges of subelement (i,j,k): x-edges (b,c) -> b + 2c, y-edges
// (a,c) -> 4 + a + 2c, z-edges (a,b) -> 8 + a + 2b.
static void nd_sub_edges(int p, int i, int j, int k, int out[12]) {
  for (int c = 0; c < 2; ++c)
    for (int b = 0; b < 2; ++b) out[b + 2 * c] = nd_local(p, 0, i, j + b, k + c);
  for (int c = 0; c < 2; ++c)
    for (int a = 0; a < 2; ++a) out[4 + a + 2 * c] = nd_local(p, 1, i + a, j, k + c);
  for (int b = 0; b < 2; ++b)
    for (int a = 0; a < 2; ++a) out[8 + a + 2 * b] = nd_local(p, 2, i + a, j + b, k);
}

static RefElem build_ref_h1(int p) {
  RefElem r;
  const int q = p + 1;
  r.nloc = q * q * q;
  r.st_ptr.push_back(0);
  for (int k = 0; k < q; ++k)
    for (int j = 0; j < q; ++j)
      for (int i = 0; i < q; ++i) {
        const int l = i + q * (j + q * k);
        for (int dz = -1; dz <= 1; ++dz)
          for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
              const int a = i + dx, b = j + dy, c = k + dz;
              if (a < 0 || b < 0 || c < 0 || a > p || b > p || c > p) continue;
              r.st_col.push_back(a + q * (b + q * c));
              r.ent_row.push_back(static_cast<uint16_t>(l));
            }
        r.st_ptr.push_back(static_cast<int32_t>(r.st_col.size()));
      }
  r.nent = static_cast<int>(r.st_col.size());
  for (int c = 0; c < 2; ++c)
    for (int b = 0; b < 2; ++b)
      for (int a = 0; a < 2; ++a) r.reps.push_back(a * p + q * (b * p + q * (c * p)));
  return r;
}

static int pair12(int u, int v) {
  if (u > v) std::swap(u, v);
  return 12 * u - (u * (u - 1)) / 2 + (v - u);
}

static RefElem build_ref_nd(int p) {
  RefElem r;
  const int q = p + 1;
  r.nloc = 3 * p * q * q;
  std::vector<std::vector<int>> nbr(r.nloc);
  std::vector<std::vector<int>> subs(r.nloc);  // subelements holding each local edge
  for (int k = 0; k < p; ++k)
    for (int j = 0; j < p; ++j)
      for (int i = 0; i < p; ++i) {
        int ed[12];
        nd_sub_edges(p, i, j, k, ed);
        const int s = i + p * (j + p * k);
        for (int u = 0; u < 12; ++u) {
          subs[ed[u]].push_back(s);
          for (int v = 0; v < 12; ++v) nbr[ed[u]].push_back(ed[v]);
        }
      }
  // recipe: per compact entry (l, l'), the contributions (subelement s, edge
  // pair index) of every subelement holding both edges, in increasing s, as
  // 16-bit codes (s << 7 | pair) packed into 64 bits, 0xffff = none
  r.st_ptr.push_back(0);
  for (int l = 0; l < r.nloc; ++l) {
    auto& v = nbr[l];
    std::sort(v.begin(), v.end());
    v.erase(std::unique(v.begin(), v.end()), v.end());
    std::vector<int>& sl = subs[l];
    std::sort(sl.begin(), sl.end());
    for (int c : v) {
      r.st_col.push_back(c);
      r.ent_row.push_back(static_cast<uint16_t>(l));
      uint64_t rec = ~0ull;
      int m = 0;
      for (int s : sl) {
        const int si = s % p, sj = (s / p) % p, sk = s / (p * p);
        int ed[12];
        nd_sub_edges(p, si, sj, sk, ed);
        int u = -1, w = -1;
        for (int t = 0; t < 12; ++t) {
          if (ed[t] == l) u = t;
          if (ed[t] == c) w = t;
        }
        if (u < 0 || w < 0) continue;
        const uint64_t code = static_cast<uint64_t>((s << 7) | pair12(u, w));
        rec &= ~(0xffffull << (16 * m));
        rec |= code << (16 * m);
        ++m;
      }
      r.recipe64.push_back(rec);
    }
    r.st_ptr.push_back(static_cast<int32_t>(r.st_col.size()));
  }
  r.nent = static_cast<int>(r.st_col.size());
  // both end edges of every coarse edge: elements sharing an edge dof share one
  for (int c = 0; c < 2; ++c)
    for (int b = 0; b < 2; ++b) {
      r.reps.push_back(nd_local(p, 0, 0, b * p, c * p));
      r.reps.push_back(nd_local(p, 0, p - 1, b * p, c * p));
      r.reps.push_back(nd_local(p, 1, b * p, 0, c * p));
      r.reps.push_back(nd_local(p, 1, b * p, p - 1, c * p));
      r.reps.push_back(nd_local(p, 2, b * p, c * p, 0));
      r.reps.push_back(nd_local(p, 2, b * p, c * p, p - 1));
    }
  std::sort(r.reps.begin(), r.reps.end());
  r.reps.erase(std::unique(r.reps.begin(), r.reps.end()), r.reps.end());
  return r;
}

static int rt_local(int p, int ax, int i, int j, int k) {
  const int q = p + 1;
  if (ax == 0) return i + q * (j + p * k);
  if (ax == 1) return p * p * q + i + p * (j + q * k);
  return 2 * p * p * q + i + p * (j + p * k);
}

// The 6 local faces of subelement (i,j,k): x-faces (xi = t) -> t, y-faces
// (eta = t) -> 2 + t, z-faces (zeta = t) -> 4 + t.
static void rt_sub_faces(int p, int i, int j, int k, int out[6]) {
  for (int t = 0; t < 2; ++t) {
    out[t] = rt_local(p, 0, i + t, j, k);
    out[2 + t] = rt_local(p, 1, i, j + t, k);
    out[4 + t] = rt_local(p, 2, i, j, k + t);
  }
}

static int pair6(int u, int v) {
  if (u > v) std::swap(u, v);
  return 6 * u - (u * (u - 1)) / 2 + (v - u);
}

// Raviart-Thomas faces: every face couples to the faces of the (one or two)
// subelements holding it; the recipe lists those subelements' contributions.
static RefElem build_ref_rt(int p) {
  RefElem r;
  const int q = p + 1;
  r.nloc = 3 * p * p * q;
  std::vector<std::vector<int>> nbr(r.nloc);
  std::vector<std::vector<int>> subs(r.nloc);
  for (int k = 0; k < p; ++k)
    for (int j = 0; j < p; ++j)
      for (int i = 0; i < p; ++i) {
        int fc[6];
        rt_sub_faces(p, i, j, k, fc);
        const int s = i + p * (j + p * k);
        for (int u = 0; u < 6; ++u) {
          subs[fc[u]].push_back(s);
          for (int v = 0; v < 6; ++v) nbr[fc[u]].push_back(fc[v]);
        }
      }
  r.st_ptr.push_back(0);
  for (int l = 0; l < r.nloc; ++l) {
    auto& v = nbr[l];
    std::sort(v.begin(), v.end());
    v.erase(std::unique(v.begin(), v.end()), v.end());
    std::vector<int>& sl = subs[l];
    std::sort(sl.begin(), sl.end());
    for (int c : v) {
      r.st_col.push_back(c);
      r.ent_row.push_back(static_cast<uint16_t>(l));
      uint64_t rec = ~0ull;
      int m = 0;
      for (int s : sl) {
        const int si = s % p, sj = (s / p) % p, sk = s / (p * p);
        int fc[6];
        rt_sub_faces(p, si, sj, sk, fc);
        int u = -1, w = -1;
        for (int t = 0; t < 6; ++t) {
          if (fc[t] == l) u = t;
          if (fc[t] == c) w = t;
        }
        if (u < 0 || w < 0) continue;
        const uint64_t code = static_cast<uint64_t>((s << 7) | pair6(u, w));
        rec &= ~(0xffffull << (16 * m));
        rec |= code << (16 * m);
        ++m;
      }
      r.recipe64.push_back(rec);
    }
    r.st_ptr.push_back(static_cast<int32_t>(r.st_col.size()));
  }
  r.nent = static_cast<int>(r.st_col.size());
  // one face on each coarse face: elements sharing a face dof share one of these
  for (int t = 0; t < 2; ++t) {
    r.reps.push_back(rt_local(p, 0, t * p, 0, 0));
    r.reps.push_back(rt_local(p, 1, 0, t * p, 0));
    r.reps.push_back(rt_local(p, 2, 0, 0, t * p));
  }
  std::sort(r.reps.begin(), r.reps.end());
  return r;
}

// 2D H1 (quadrilateral macro elements, bilinear subelements): the 9-point
// lattice neighbourhood, with the recipe of every local entry (the <= 4
// subelements holding both vertices, vertex pair index among the 10 pairs of
// a subelement's corners v = a + 2b).
static RefElem build_ref_h1_2d(int p) {
  RefElem r;
  const int q = p + 1;
  r.nloc = q * q;
  auto pair4 = [](int u, int v) {
    if (u > v) std::swap(u, v);
    return 4 * u - (u * (u - 1)) / 2 + (v - u);
  };
  r.st_ptr.push_back(0);
  for (int j = 0; j < q; ++j)
    for (int i = 0; i < q; ++i) {
      const int l = i + q * j;
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          const int a2 = i + dx, b2 = j + dy;
          if (a2 < 0 || b2 < 0 || a2 > p || b2 > p) continue;
          r.st_col.push_back(a2 + q * b2);
          r.ent_row.push_back(static_cast<uint16_t>(l));
          uint64_t rec = ~0ull;
          int m = 0;
          for (int sj = 0; sj < p; ++sj)
            for (int si = 0; si < p; ++si) {  // increasing subelement index
              const int u = (i - si) + 2 * (j - sj), w = (a2 - si) + 2 * (b2 - sj);
              if (i - si < 0 || i - si > 1 || j - sj < 0 || j - sj > 1) continue;
              if (a2 - si < 0 || a2 - si > 1 || b2 - sj < 0 || b2 - sj > 1) continue;
              const int s = si + p * sj;
              rec &= ~(0xffffull << (16 * m));
              rec |= static_cast<uint64_t>((s << 7) | pair4(u, w)) << (16 * m);
              ++m;
            }
          r.recipe64.push_back(rec);
        }
      r.st_ptr.push_back(static_cast<int32_t>(r.st_col.size()));
    }
  r.nent = static_cast<int>(r.st_col.size());
  for (int b = 0; b < 2; ++b)
    for (int a = 0; a < 2; ++a) r.reps.push_back(a * p + q * (b * p));
  return r;
}

static RefElem build_ref(int space, int p) {
  if (space == LOR_H1) return build_ref_h1(p);
  if (space == LOR_ND) return build_ref_nd(p);
  if (space == LOR_H1_2D) return build_ref_h1_2d(p);
  return build_ref_rt(p);
}

// ------------------------------------------------------------------- scan

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

template <typename TI>
__global__ __launch_bounds__(kScanThreads) void k_scan_tiles(const TI* __restrict__ in, int64_t n,
                                                             int64_t* __restrict__ out,
                                                             int64_t* __restrict__ tile_sums) {
  __shared__ int64_t sh[kScanThreads];
  const int t = threadIdx.x;
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile + t * kScanItems;
  int64_t v[kScanItems];
  int64_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    v[i] = (base + i < n) ? static_cast<int64_t>(in[base + i]) : 0;
    s += v[i];
  }
  sh[t] = s;
  __syncthreads();
  for (int off = 1; off < kScanThreads; off <<= 1) {
    const int64_t x = (t >= off) ? sh[t - off] : 0;
    __syncthreads();
    sh[t] += x;
    __syncthreads();
  }
  int64_t ex = sh[t] - s;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    if (base + i < n) out[base + i] = ex;
    ex += v[i];
  }
  if (t == kScanThreads - 1) tile_sums[blockIdx.x] = sh[t];
}

__global__ void k_scan_add(int64_t* __restrict__ out, int64_t n, const int64_t* __restrict__ tile_off) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) out[i] += tile_off[i / kScanTile];
}

template <typename TI>
__global__ void k_scan_total(const TI* __restrict__ in, int64_t n, int64_t* __restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) out[n] = (n == 0) ? 0 : out[n - 1] + static_cast<int64_t>(in[n - 1]);
}

// Exclusive scan of n values into out[0..n], out[n] = total.
template <typename TI>
static int scan_exclusive(const TI* in, int64_t n, int64_t* out, hipStream_t st) {
  if (n == 0) {
    k_scan_total<TI><<<1, 1, 0, st>>>(in, 0, out);
    LOR_LAUNCHED("k_scan_total");
    return LOR_OK;
  }
  const int64_t ntiles = ceil_div(n, kScanTile);
  DevBuf sums, offs;
  int rc = sums.alloc(sizeof(int64_t) * (ntiles + 1));
  if (rc) return rc;
  rc = offs.alloc(sizeof(int64_t) * (ntiles + 1));
  if (rc) return rc;
  k_scan_tiles<TI><<<ntiles, kScanThreads, 0, st>>>(in, n, out, sums.as<int64_t>());
  LOR_LAUNCHED("k_scan_tiles");
  if (ntiles > 1) {
    rc = scan_exclusive<int64_t>(sums.as<int64_t>(), ntiles, offs.as<int64_t>(), st);
    if (rc) return rc;
    k_scan_add<<<ceil_div(n, 256), 256, 0, st>>>(out, n, offs.as<int64_t>());
    LOR_LAUNCHED("k_scan_add");
  }
  k_scan_total<TI><<<1, 1, 0, st>>>(in, n, out);
  LOR_LAUNCHED("k_scan_total");
  return LOR_OK;
}

// ------------------------------------------------------------ small kernels

__device__ __forceinline__ int32_t dof_id(int32_t v, int is_signed) {
  return (is_signed && v < 0) ? -1 - v : v;
}

__global__ void k_fill_i32(int32_t* __restrict__ a, int64_t n, int32_t v) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

__global__ void k_iota_i32(int32_t* __restrict__ a, int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) a[i] = static_cast<int32_t>(i);
}

__global__ void k_i64_to_i32(const int64_t* __restrict__ a, int64_t n, int32_t* __restrict__ b) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) b[i] = static_cast<int32_t>(a[i]);
}

// Error bits reported by the kernels below.
enum : int32_t {
  kErrMapRange = 1,
  kErrRowTooLong = 2,
  kErrRowCount = 4,
  kErrTooManyColors = 8,
  kErrColorConflict = 16,
  kErrRankMissing = 32,
};

__global__ void k_count_inc(const int32_t* __restrict__ map, int64_t total, int64_t nrows, int is_signed,
                            int32_t* __restrict__ cnt, int32_t* __restrict__ err) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int32_t g = dof_id(map[i], is_signed);
  if (g < 0 || g >= nrows) {
    atomicOr(err, kErrMapRange);
    return;
  }
  atomicAdd(&cnt[g], 1);
}

__global__ void k_fill_inc(const int32_t* __restrict__ map, int64_t total, int64_t nrows, int is_signed,
                           const int32_t* __restrict__ inc_ptr, int32_t* __restrict__ fill,
                           int32_t* __restrict__ inc_list) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int32_t g = dof_id(map[i], is_signed);
  if (g < 0 || g >= nrows) return;
  const int32_t slot = atomicAdd(&fill[g], 1);
  inc_list[inc_ptr[g] + slot] = static_cast<int32_t>(i);
}

// Sort each (short) incidence list so that later passes are order-independent.
__global__ void k_sort_inc(const int32_t* __restrict__ inc_ptr, int32_t* __restrict__ inc_list, int64_t nrows) {
  const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (g >= nrows) return;
  const int32_t a = inc_ptr[g], b = inc_ptr[g + 1];
  for (int32_t i = a + 1; i < b; ++i) {
    const int32_t x = inc_list[i];
    int32_t j = i - 1;
    while (j >= a && inc_list[j] > x) {
      inc_list[j + 1] = inc_list[j];
      --j;
    }
    inc_list[j + 1] = x;
  }
}

// Columns of row g: sorted union of the local stencils of its incidences.
// One lane per row; the per-lane working list lives in LDS (odd stride, so
// lanes working on the same slot hit different banks).
constexpr int kRowThreads = 64;
constexpr int kRowStride = LOR_MAX_ROW_NNZ + 2;

template <bool FILL>
__global__ __launch_bounds__(kRowThreads) void k_row_cols(
    const int32_t* __restrict__ map, int nloc, int is_signed, const int32_t* __restrict__ inc_ptr,
    const int32_t* __restrict__ inc_list, const int32_t* __restrict__ st_ptr,
    const int32_t* __restrict__ st_col, int64_t nrows, int32_t* __restrict__ cnt,
    const int32_t* __restrict__ row_ptr, int32_t* __restrict__ col_idx, int32_t* __restrict__ err) {
  __shared__ int32_t buf[kRowThreads * kRowStride];
  const int64_t g = static_cast<int64_t>(blockIdx.x) * kRowThreads + threadIdx.x;
  if (g >= nrows) return;
  int32_t* b = buf + threadIdx.x * kRowStride;
  int n = 0;
  bool overflow = false;
  for (int32_t ii = inc_ptr[g]; ii < inc_ptr[g + 1] && !overflow; ++ii) {
    const int32_t inc = inc_list[ii];
    const int32_t e = inc / nloc;
    const int32_t l = inc - e * nloc;
    const int32_t* me = map + static_cast<int64_t>(e) * nloc;
    for (int32_t kk = st_ptr[l]; kk < st_ptr[l + 1]; ++kk) {
      const int32_t c = dof_id(me[st_col[kk]], is_signed);
      int pos = n;
      while (pos > 0 && b[pos - 1] > c) --pos;
      if (pos > 0 && b[pos - 1] == c) continue;
      if (n >= LOR_MAX_ROW_NNZ) {
        overflow = true;
        break;
      }
      for (int m = n; m > pos; --m) b[m] = b[m - 1];
      b[pos] = c;
      ++n;
    }
  }
  if (overflow) {
    atomicOr(err, kErrRowTooLong);
    if (!FILL) cnt[g] = 0;
    return;
  }
  if (!FILL) {
    cnt[g] = n;
  } else {
    const int32_t base = row_ptr[g];
    if (row_ptr[g + 1] - base != n) {
      atomicOr(err, kErrRowCount);
      return;
    }
    for (int m = 0; m < n; ++m) col_idx[base + m] = b[m];
  }
}

// One Jones-Plassmann round with priorities = element index: an uncoloured
// element whose lower-index neighbours are all coloured takes the smallest
// colour none of its coloured neighbours uses.  The fixed point equals the
// sequential greedy colouring in element order (deterministic).
__global__ void k_jp_round(const int32_t* __restrict__ map, int nloc, int is_signed,
                           const int32_t* __restrict__ reps, int nreps,
                           const int32_t* __restrict__ inc_ptr, const int32_t* __restrict__ inc_list,
                           int64_t nel, int32_t* color, int32_t* __restrict__ ncolored,
                           int32_t* __restrict__ err) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= nel) return;
  if (__hip_atomic_load(&color[e], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= 0) return;
  uint64_t used = 0;
  const int32_t* me = map + e * nloc;
  for (int r = 0; r < nreps; ++r) {
    const int32_t g = dof_id(me[reps[r]], is_signed);
    for (int32_t ii = inc_ptr[g]; ii < inc_ptr[g + 1]; ++ii) {
      const int32_t e2 = inc_list[ii] / nloc;
      if (e2 == e) continue;
      const int32_t c2 = __hip_atomic_load(&color[e2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (c2 < 0) {
        if (e2 < e) return;
        continue;
      }
      used |= (1ull << c2);
    }
  }
  if (~used == 0ull) {
    atomicOr(err, kErrTooManyColors);
    return;
  }
  const int c = __ffsll(static_cast<long long>(~used)) - 1;
  if (c >= LOR_MAX_COLORS) {
    atomicOr(err, kErrTooManyColors);
    return;
  }
  __hip_atomic_store(&color[e], c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  atomicAdd(ncolored, 1);
}

// Every dof's incident elements must carry pairwise different colours.
__global__ void k_check_colors(const int32_t* __restrict__ inc_ptr, const int32_t* __restrict__ inc_list,
                               int nloc, int64_t nrows, const int32_t* __restrict__ color,
                               int32_t* __restrict__ err) {
  const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (g >= nrows) return;
  const int32_t a = inc_ptr[g], b = inc_ptr[g + 1];
  for (int32_t i = a; i < b; ++i) {
    const int32_t ei = inc_list[i] / nloc;
    for (int32_t j = i + 1; j < b; ++j) {
      const int32_t ej = inc_list[j] / nloc;
      if (ei != ej && color[ei] == color[ej]) {
        atomicOr(err, kErrColorConflict);
        return;
      }
    }
  }
}

__global__ void k_color_flags(const int32_t* __restrict__ color, int64_t nel, int c, int32_t* __restrict__ f) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e < nel) f[e] = (color[e] == c) ? 1 : 0;
}

__global__ void k_color_scatter(const int32_t* __restrict__ color, int64_t nel, int c,
                                const int64_t* __restrict__ pos, int32_t base, int32_t* __restrict__ order) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e < nel && color[e] == c) order[base + pos[e]] = static_cast<int32_t>(e);
}

// Position of every local stencil entry inside its CSR row; lowest colour per nnz.
__global__ void k_rank_pass0(const int32_t* __restrict__ map, int nloc, int is_signed, int nent, int64_t stride,
                             const uint16_t* __restrict__ ent_row, const int32_t* __restrict__ ent_col,
                             const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col_idx,
                             const int32_t* __restrict__ color, int64_t total,
                             int32_t* __restrict__ mincolor, uint8_t* __restrict__ tables,
                             int32_t* __restrict__ err) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int64_t e = idx / nent;
  const int k = static_cast<int>(idx - e * nent);
  const int32_t* me = map + e * nloc;
  const int32_t g = dof_id(me[ent_row[k]], is_signed);
  const int32_t c = dof_id(me[ent_col[k]], is_signed);
  int32_t lo = row_ptr[g], hi = row_ptr[g + 1];
  const int32_t start = lo;
  while (lo < hi) {
    const int32_t mid = (lo + hi) >> 1;
    if (col_idx[mid] < c)
      lo = mid + 1;
    else
      hi = mid;
  }
  uint8_t* tab = tables + e * stride + k;
  if (lo >= row_ptr[g + 1] || col_idx[lo] != c) {
    atomicOr(err, kErrRankMissing);
    *tab = 0;
    return;
  }
  *tab = static_cast<uint8_t>(lo - start);
  atomicMin(&mincolor[lo], color[e]);
}

__global__ void k_rank_pass1(const int32_t* __restrict__ map, int nloc, int is_signed, int nent, int64_t stride,
                             const uint16_t* __restrict__ ent_row, const int32_t* __restrict__ row_ptr,
                             const int32_t* __restrict__ color, int64_t total,
                             const int32_t* __restrict__ mincolor, uint8_t* __restrict__ tables) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int64_t e = idx / nent;
  const int k = static_cast<int>(idx - e * nent);
  const int32_t g = dof_id(map[e * nloc + ent_row[k]], is_signed);
  uint8_t* tab = tables + e * stride + k;
  const uint8_t t = *tab;
  if (mincolor[row_ptr[g] + (t & kRankMask)] == color[e]) *tab = static_cast<uint8_t>(t | kFirstBit);
}

// Table deduplication: elements whose rank tables are byte-identical share one
// class.  64-bit FNV-1a of every element table; the host numbers classes by
// first appearance; equality with the class representative is then verified
// word by word, so a hash collision can only cost the deduplication, never
// correctness.
__global__ void k_table_hash(const uint32_t* __restrict__ tables, int64_t words, int64_t nel,
                             uint64_t* __restrict__ hash) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= nel) return;
  const uint32_t* t = tables + e * words;
  uint64_t h = 1469598103934665603ull;
  for (int64_t w = 0; w < words; ++w) {
    h ^= t[w];
    h *= 1099511628211ull;
  }
  hash[e] = h;
}

__global__ void k_table_verify(const uint32_t* __restrict__ tables, int64_t words, int64_t nel,
                               const int32_t* __restrict__ cls, const int32_t* __restrict__ rep,
                               int32_t* __restrict__ mismatch) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= nel * words) return;
  const int64_t e = idx / words;
  const int64_t w = idx - e * words;
  if (tables[e * words + w] != tables[static_cast<int64_t>(rep[cls[e]]) * words + w]) atomicOr(mismatch, 1);
}

__global__ void k_table_gather(const uint32_t* __restrict__ tables, int64_t words, int64_t nclass,
                               const int32_t* __restrict__ rep, uint32_t* __restrict__ out) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= nclass * words) return;
  const int64_t c = idx / words;
  out[idx] = tables[static_cast<int64_t>(rep[c]) * words + (idx - c * words)];
}

__global__ void k_gather_i32(const int32_t* __restrict__ src, const int32_t* __restrict__ idx, int64_t n,
                             int32_t* __restrict__ dst) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[idx[i]];
}


// ------------------------------------------------ owner-computes schedule (H1)
//
// The owner-computes value kernel works on the global lattice of a box of
// elements: lattice point (X, Y, Z) has vertex id base(Y, Z) + X, and the
// cell (X, Y, Z) belongs to element elem3d(X / p, Y / p, Z / p).  These
// kernels find each element's face neighbours (same lattice orientation),
// and, once the host has laid the elements out as a box, check everything
// the value kernel relies on against the element map and the finished
// pattern; any failure only marks the mesh as not eligible (the colour
// schedule is always built).

enum : int32_t { kOwnAmbiguous = 1, kOwnAsymmetric = 2, kOwnVertex = 4, kOwnRow = 8, kOwnCover = 16 };

// Slot of a face direction in the neighbour table: +x, +y, +z, (+y+z), -x, -y, -z.
__host__ __device__ constexpr int nbr_slot(int ax, int sg) { return sg > 0 ? ax : 4 + ax; }

// One thread per (element, face direction): the element f != e whose lattice
// continues e's lattice across that face (f's layer 0 is e's layer p for a +
// direction, and the other way round for a - direction, point by point).
__global__ void k_owner_nbrs(const int32_t* __restrict__ map, int p, int64_t nel,
                             const int32_t* __restrict__ inc_ptr, const int32_t* __restrict__ inc_list,
                             int32_t* __restrict__ nbr, int32_t* __restrict__ flag) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= nel * 6) return;
  const int64_t e = t / 6;
  const int dir = static_cast<int>(t - e * 6);
  const int ax = dir % 3, sg = dir < 3 ? 1 : -1;
  const int q = p + 1, nloc = q * q * q;
  const int stride[3] = {1, q, q * q};
  const int le = sg > 0 ? p * stride[ax] : 0;  // corner of e on the face
  const int lf = sg > 0 ? 0 : p * stride[ax];  // the same point in f
  const int u1 = stride[(ax + 1) % 3], u2 = stride[(ax + 2) % 3];
  const int32_t* me = map + e * nloc;
  const int32_t v = me[le];
  int32_t found = -1;
  for (int32_t i = inc_ptr[v]; i < inc_ptr[v + 1]; ++i) {
    const int32_t f = inc_list[i] / nloc;
    const int32_t l = inc_list[i] - f * nloc;
    if (f == e || l != lf) continue;
    const int32_t* mf = map + static_cast<int64_t>(f) * nloc;
    bool same = true;
    for (int a = 0; a <= p && same; ++a)
      for (int b = 0; b <= p && same; ++b) same = mf[lf + a * u1 + b * u2] == me[le + a * u1 + b * u2];
    if (!same) continue;
    if (found >= 0) atomicOr(flag, kOwnAmbiguous);
    found = f;
  }
  nbr[e * 8 + nbr_slot(ax, sg)] = found;
}

// Diagonal neighbour +y+z (the +z neighbour of the +y neighbour) and the
// symmetry of the face relation.
__global__ void k_owner_diag(int64_t nel, int32_t* __restrict__ nbr, int32_t* __restrict__ flag) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= nel) return;
  int32_t* n = nbr + e * 8;
  for (int ax = 0; ax < 3; ++ax) {
    const int32_t f = n[nbr_slot(ax, 1)];
    if (f >= 0 && nbr[static_cast<int64_t>(f) * 8 + nbr_slot(ax, -1)] != e) atomicOr(flag, kOwnAsymmetric);
    const int32_t g = n[nbr_slot(ax, -1)];
    if (g >= 0 && nbr[static_cast<int64_t>(g) * 8 + nbr_slot(ax, 1)] != e) atomicOr(flag, kOwnAsymmetric);
  }
  const int32_t fy = n[1];
  n[3] = fy >= 0 ? nbr[static_cast<int64_t>(fy) * 8 + 2] : -1;
  n[7] = -1;
}

// base(Y, Z): the vertex id at lattice point (0, Y, Z), read from the element
// at box position (0, min(Y / p, ny - 1), min(Z / p, nz - 1)).
__global__ void k_owner_base(const int32_t* __restrict__ map, int p, const int32_t* __restrict__ elem3d, int nx,
                             int ny, int nz, int32_t* __restrict__ base) {
  const int ly = ny * p + 1, lz = nz * p + 1;
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= static_cast<int64_t>(ly) * lz) return;
  const int Y = static_cast<int>(t % ly), Z = static_cast<int>(t / ly);
  const int ey = min(Y / p, ny - 1), ez = min(Z / p, nz - 1);
  const int q = p + 1;
  const int32_t e = elem3d[(static_cast<int64_t>(ez) * ny + ey) * nx];
  base[t] = map[static_cast<int64_t>(e) * q * q * q + q * ((Y - p * ey) + q * (Z - p * ez))];
}

// One thread per (box position, local vertex): the vertex id equals
// base(Y, Z) + X at its global lattice point.
__global__ void k_owner_verts(const int32_t* __restrict__ map, int p, const int32_t* __restrict__ elem3d, int nx,
                              int ny, int nz, const int32_t* __restrict__ base, int32_t* __restrict__ flag) {
  const int q = p + 1, nloc = q * q * q;
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t nel = static_cast<int64_t>(nx) * ny * nz;
  if (t >= nel * nloc) return;
  const int64_t pos = t / nloc;
  const int l = static_cast<int>(t - pos * nloc);
  const int ex = static_cast<int>(pos % nx), ey = static_cast<int>((pos / nx) % ny), ez = static_cast<int>(pos / (static_cast<int64_t>(nx) * ny));
  const int X = p * ex + l % q, Y = p * ey + (l / q) % q, Z = p * ez + l / (q * q);
  const int32_t e = elem3d[pos];
  if (map[static_cast<int64_t>(e) * nloc + l] != base[static_cast<int64_t>(Z) * (ny * p + 1) + Y] + X)
    atomicOr(flag, kOwnVertex);
}

// One thread per lattice point: the row of its vertex holds exactly the
// lattice neighbours present, in (dz, dy, dx) order (which must therefore be
// increasing), and every vertex is reached once.
__global__ void k_owner_rows(int p, int nx, int ny, int nz, const int32_t* __restrict__ base, int64_t nrows,
                             const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col_idx,
                             int32_t* __restrict__ hit, int32_t* __restrict__ flag) {
  const int LX = nx * p + 1, LY = ny * p + 1, LZ = nz * p + 1;
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= static_cast<int64_t>(LX) * LY * LZ) return;
  const int X = static_cast<int>(t % LX), Y = static_cast<int>((t / LX) % LY);
  const int Z = static_cast<int>(t / (static_cast<int64_t>(LX) * LY));
  const int64_t v = static_cast<int64_t>(base[static_cast<int64_t>(Z) * LY + Y]) + X;
  if (v < 0 || v >= nrows) {
    atomicOr(flag, kOwnRow);
    return;
  }
  atomicAdd(&hit[v], 1);
  const int xlo = X > 0, xhi = X < LX - 1, ylo = Y > 0, yhi = Y < LY - 1, zlo = Z > 0, zhi = Z < LZ - 1;
  const int32_t rb = row_ptr[v];
  if (row_ptr[v + 1] - rb != (1 + xlo + xhi) * (1 + ylo + yhi) * (1 + zlo + zhi)) {
    atomicOr(flag, kOwnRow);
    return;
  }
  int k = 0;
  for (int dz = -zlo; dz <= zhi; ++dz)
    for (int dy = -ylo; dy <= yhi; ++dy)
      for (int dx = -xlo; dx <= xhi; ++dx, ++k)
        if (col_idx[rb + k] != base[static_cast<int64_t>(Z + dz) * LY + Y + dy] + X + dx) {
          atomicOr(flag, kOwnRow);
          return;
        }
}

__global__ void k_owner_cover(const int32_t* __restrict__ hit, int64_t nrows, int32_t* __restrict__ flag) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < nrows && hit[i] != 1) atomicOr(flag, kOwnCover);
}

// --------------------------------------------------------------- host side

static size_t align256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

template <typename T>
static int upload(const std::vector<T>& v, void* dst, hipStream_t st) {
  if (v.empty()) return LOR_OK;
  LOR_HIP(hipMemcpyAsync(dst, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, st));
  return LOR_OK;
}

static size_t layout(lor_sched* s, const RefElem& r) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  s->off_order = take(sizeof(int32_t) * s->nel);
  s->off_color = take(sizeof(int32_t) * s->nel);
  s->off_class = take(sizeof(int32_t) * s->nel);
  s->tab_stride = (r.nent + 15) / 16 * 16;
  s->off_tables = take(static_cast<size_t>(s->nel) * s->tab_stride);
  s->off_inc_ptr = take(sizeof(int32_t) * (s->nrows + 1));
  s->off_inc_list = take(sizeof(int32_t) * s->nel * r.nloc);
  s->off_st_ptr = take(sizeof(int32_t) * r.st_ptr.size());
  s->off_st_col = take(sizeof(int32_t) * r.st_col.size());
  s->off_ent_row = take(sizeof(uint16_t) * r.ent_row.size());
  s->off_recipe = take(sizeof(uint64_t) * std::max<size_t>(1, r.recipe64.size()));
  s->off_zero = take(256);
  s->off_order_class = take(sizeof(int32_t) * s->nel);
  s->off_nbr = take(sizeof(int32_t) * 8 * s->nel);
  s->off_elem3d = take(sizeof(int32_t) * s->nel);
  // a box has (LY)(LZ) = nrows / LX lattice lines along x, and LX >= p + 1
  s->off_base = take(sizeof(int32_t) * (s->nrows / (s->p + 1) + 1));
  return off;
}

// Owner-computes schedule of an H1 mesh: face neighbours, the box layout of
// the elements, base(Y, Z), and the checks of the value kernel's
// assumptions.  Leaves sched->owner = 0 if the mesh is not eligible; returns
// an error only for device failures.
static int build_owner(lor_sched* s, const int32_t* map, const int32_t* row_ptr, const int32_t* col_idx,
                       hipStream_t st) {
  s->owner = 0;
  s->box[0] = s->box[1] = s->box[2] = 0;
  const int64_t nel = s->nel;
  const int p = s->p;
  if (nel == 0 || s->space != LOR_H1) return LOR_OK;
  int32_t* d_nbr = dev_at<int32_t>(s, s->off_nbr);
  DevBuf flag;
  int rc;
  if ((rc = flag.alloc(sizeof(int32_t)))) return rc;
  LOR_HIP(hipMemsetAsync(flag.p, 0, sizeof(int32_t), st));
  k_owner_nbrs<<<ceil_div(nel * 6, 256), 256, 0, st>>>(map, p, nel, dev_at<int32_t>(s, s->off_inc_ptr),
                                                       dev_at<int32_t>(s, s->off_inc_list), d_nbr, flag.as<int32_t>());
  LOR_LAUNCHED("k_owner_nbrs");
  k_owner_diag<<<ceil_div(nel, 256), 256, 0, st>>>(nel, d_nbr, flag.as<int32_t>());
  LOR_LAUNCHED("k_owner_diag");
  int32_t hflag = 0;
  std::vector<int32_t> nb(static_cast<size_t>(nel) * 8);
  LOR_HIP(hipMemcpyAsync(&hflag, flag.p, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  LOR_HIP(hipMemcpyAsync(nb.data(), d_nbr, sizeof(int32_t) * nb.size(), hipMemcpyDeviceToHost, st));
  LOR_HIP(hipStreamSynchronize(st));
  if (hflag != 0) return LOR_OK;
  // box layout: from the one element without -x, -y, -z neighbours, walk +x,
  // +y and +z; every element must be reached exactly once and its neighbours
  // must be its box neighbours
  auto N = [&](int64_t e, int slot) { return nb[static_cast<size_t>(e) * 8 + slot]; };
  int64_t corner = -1;
  for (int64_t e = 0; e < nel; ++e)
    if (N(e, 4) < 0 && N(e, 5) < 0 && N(e, 6) < 0) {
      if (corner >= 0) return LOR_OK;
      corner = e;
    }
  if (corner < 0) return LOR_OK;
  int64_t dims[3] = {0, 0, 0};
  for (int ax = 0; ax < 3; ++ax)
    for (int64_t e = corner; e >= 0 && dims[ax] <= nel; e = N(e, ax)) ++dims[ax];
  if (dims[0] * dims[1] * dims[2] != nel) return LOR_OK;
  const int64_t nx = dims[0], ny = dims[1], nz = dims[2];
  std::vector<int32_t> e3(static_cast<size_t>(nel), -1);
  std::vector<char> seen(static_cast<size_t>(nel), 0);
  for (int64_t ez = 0; ez < nz; ++ez)
    for (int64_t ey = 0; ey < ny; ++ey) {
      const size_t at = static_cast<size_t>((ez * ny + ey) * nx);
      int64_t e = ez == 0 && ey == 0 ? corner : ey == 0 ? N(e3[at - nx * ny], 2) : N(e3[at - nx], 1);
      for (int64_t ex = 0; ex < nx; ++ex) {
        if (e < 0 || seen[e]) return LOR_OK;
        seen[e] = 1;
        e3[at + ex] = static_cast<int32_t>(e);
        e = N(e, 0);
      }
      if (e >= 0) return LOR_OK;
    }
  for (int64_t ez = 0; ez < nz; ++ez)
    for (int64_t ey = 0; ey < ny; ++ey)
      for (int64_t ex = 0; ex < nx; ++ex) {
        const int64_t e = e3[(ez * ny + ey) * nx + ex];
        const int64_t c[3] = {ex, ey, ez}, n[3] = {nx, ny, nz};
        for (int ax = 0; ax < 3; ++ax) {
          int64_t up = -1, dn = -1;
          int64_t cc[3] = {c[0], c[1], c[2]};
          if (c[ax] + 1 < n[ax]) {
            cc[ax] = c[ax] + 1;
            up = e3[(cc[2] * ny + cc[1]) * nx + cc[0]];
          }
          cc[ax] = c[ax] - 1;
          if (c[ax] > 0) dn = e3[(cc[2] * ny + cc[1]) * nx + cc[0]];
          if (N(e, nbr_slot(ax, 1)) != up || N(e, nbr_slot(ax, -1)) != dn) return LOR_OK;
        }
      }
  if (nx * p + 1 > INT32_MAX || ny * p + 1 > INT32_MAX || nz * p + 1 > INT32_MAX) return LOR_OK;
  const int64_t LX = nx * p + 1, LY = ny * p + 1, LZ = nz * p + 1;
  if (LX * LY * LZ != s->nrows || LY * LZ > s->nrows / (p + 1) + 1) return LOR_OK;
  int32_t* d_e3 = dev_at<int32_t>(s, s->off_elem3d);
  int32_t* d_base = dev_at<int32_t>(s, s->off_base);
  if ((rc = upload(e3, d_e3, st))) return rc;
  k_owner_base<<<ceil_div(LY * LZ, 256), 256, 0, st>>>(map, p, d_e3, static_cast<int>(nx), static_cast<int>(ny),
                                                     static_cast<int>(nz), d_base);
  LOR_LAUNCHED("k_owner_base");
  k_owner_verts<<<ceil_div(nel * nloc_h1(p), 256), 256, 0, st>>>(map, p, d_e3, static_cast<int>(nx),
                                                                 static_cast<int>(ny), static_cast<int>(nz), d_base,
                                                                 flag.as<int32_t>());
  LOR_LAUNCHED("k_owner_verts");
  DevBuf hit;
  if ((rc = hit.alloc(sizeof(int32_t) * s->nrows))) return rc;
  LOR_HIP(hipMemsetAsync(hit.p, 0, sizeof(int32_t) * s->nrows, st));
  k_owner_rows<<<ceil_div(s->nrows, 256), 256, 0, st>>>(p, static_cast<int>(nx), static_cast<int>(ny),
                                                        static_cast<int>(nz), d_base, s->nrows, row_ptr, col_idx,
                                                        hit.as<int32_t>(), flag.as<int32_t>());
  LOR_LAUNCHED("k_owner_rows");
  k_owner_cover<<<ceil_div(s->nrows, 256), 256, 0, st>>>(hit.as<int32_t>(), s->nrows, flag.as<int32_t>());
  LOR_LAUNCHED("k_owner_cover");
  LOR_HIP(hipMemcpyAsync(&hflag, flag.p, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  LOR_HIP(hipStreamSynchronize(st));
  if (hflag != 0) return LOR_OK;
  s->box[0] = static_cast<int32_t>(nx);
  s->box[1] = static_cast<int32_t>(ny);
  s->box[2] = static_cast<int32_t>(nz);
  s->owner = 1;
  return LOR_OK;
}

static int read_err(const int32_t* d_err, hipStream_t st, int32_t* h) {
  LOR_HIP(hipMemcpyAsync(h, d_err, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  LOR_HIP(hipStreamSynchronize(st));
  return LOR_OK;
}

static int report_err(int32_t e) {
  if (e & kErrMapRange) LOR_FAIL(LOR_EINVAL, "element map entry outside [0, nrows)");
  if (e & kErrRowTooLong) LOR_FAIL(LOR_EUNSUPPORTED, "a row has more than %d nonzeros", LOR_MAX_ROW_NNZ);
  if (e & kErrTooManyColors) LOR_FAIL(LOR_EUNSUPPORTED, "element colouring needs more than %d colours", LOR_MAX_COLORS);
  if (e & kErrColorConflict)
    LOR_FAIL(LOR_EINVAL, "elements sharing a dof got the same colour: the element lattices are not conforming");
  if (e & (kErrRowCount | kErrRankMissing))
    LOR_FAIL(LOR_EINVAL, "row_ptr does not match the element map (call phase 1 with the same map)");
  return LOR_OK;
}

// Incidence lists (transpose of the element map) into inc_ptr / inc_list.
static int build_incidence(const int32_t* map, int64_t nel, int nloc, int is_signed, int64_t nrows,
                           int32_t* inc_ptr, int32_t* inc_list, int32_t* d_err, hipStream_t st) {
  const int64_t total = nel * nloc;
  DevBuf cnt, ptr64;
  int rc = cnt.alloc(sizeof(int32_t) * (nrows + 1));
  if (rc) return rc;
  rc = ptr64.alloc(sizeof(int64_t) * (nrows + 1));
  if (rc) return rc;
  LOR_HIP(hipMemsetAsync(cnt.p, 0, sizeof(int32_t) * (nrows + 1), st));
  if (total > 0) {
    k_count_inc<<<ceil_div(total, 256), 256, 0, st>>>(map, total, nrows, is_signed, cnt.as<int32_t>(), d_err);
    LOR_LAUNCHED("k_count_inc");
  }
  rc = scan_exclusive<int32_t>(cnt.as<int32_t>(), nrows, ptr64.as<int64_t>(), st);
  if (rc) return rc;
  k_i64_to_i32<<<ceil_div(nrows + 1, 256), 256, 0, st>>>(ptr64.as<int64_t>(), nrows + 1, inc_ptr);
  LOR_LAUNCHED("k_i64_to_i32");
  LOR_HIP(hipMemsetAsync(cnt.p, 0, sizeof(int32_t) * (nrows + 1), st));
  if (total > 0) {
    k_fill_inc<<<ceil_div(total, 256), 256, 0, st>>>(map, total, nrows, is_signed, inc_ptr,
                                                     cnt.as<int32_t>(), inc_list);
    LOR_LAUNCHED("k_fill_inc");
  }
  k_sort_inc<<<ceil_div(nrows, 256), 256, 0, st>>>(inc_ptr, inc_list, nrows);
  LOR_LAUNCHED("k_sort_inc");
  return LOR_OK;
}

}  // namespace lor

using namespace lor;

extern "C" size_t lor_pattern_workspace(int space, int p, int64_t nel, int64_t nrows) {
  if (space != LOR_H1 && space != LOR_ND && space != LOR_RT && space != LOR_H1_2D) return 0;
  if (p < 1 || p > LOR_MAX_P || nel < 0 || nrows < 1 || nrows >= INT32_MAX) return 0;
  const int nloc = space == LOR_H1      ? nloc_h1(p)
                   : space == LOR_ND    ? nloc_nd(p)
                   : space == LOR_H1_2D ? (p + 1) * (p + 1)
                                        : nloc_rt(p);
  if (nel * static_cast<int64_t>(nloc) >= INT32_MAX) return 0;
  lor_sched s{};
  s.space = space;
  s.p = p;
  s.nel = nel;
  s.nrows = nrows;
  return layout(&s, build_ref(space, p));
}

extern "C" int lor_pattern(int space, int p, int64_t nel, int64_t nrows, const int32_t* elem_map,
                           int32_t* row_ptr, int64_t* nnz, int32_t* col_idx, lor_sched* sched,
                           void* stream) {
  clear_error();
  if (space != LOR_H1 && space != LOR_ND && space != LOR_RT && space != LOR_H1_2D)
    LOR_FAIL(LOR_EINVAL, "space must be LOR_H1, LOR_ND, LOR_RT or LOR_H1_2D");
  if (p < 1 || p > LOR_MAX_P) LOR_FAIL(LOR_EINVAL, "p = %d outside [1, %d]", p, LOR_MAX_P);
  if (nel < 0) LOR_FAIL(LOR_EINVAL, "nel < 0");
  if (nrows < 1) LOR_FAIL(LOR_EINVAL, "nrows < 1");
  if (!row_ptr || !nnz || !sched) LOR_FAIL(LOR_EINVAL, "row_ptr, nnz and sched must not be NULL");
  if (nel > 0 && !elem_map) LOR_FAIL(LOR_EINVAL, "elem_map is NULL");
  const int nloc = space == LOR_H1      ? nloc_h1(p)
                   : space == LOR_ND    ? nloc_nd(p)
                   : space == LOR_H1_2D ? (p + 1) * (p + 1)
                                        : nloc_rt(p);
  if (nel * static_cast<int64_t>(nloc) >= INT32_MAX) LOR_FAIL(LOR_EOVERFLOW, "nel * nloc >= 2^31");
  if (nrows >= INT32_MAX) LOR_FAIL(LOR_EOVERFLOW, "nrows >= 2^31 - 1");
  const int is_signed = space == LOR_ND || space == LOR_RT;
  hipStream_t st = as_stream(stream);
  const RefElem ref = build_ref(space, p);
  const int64_t total = nel * nloc;
  int rc;
  if (col_idx != nullptr) {
    if (!sched->dev) LOR_FAIL(LOR_EINVAL, "sched->dev is NULL (allocate sched->dev_bytes after phase 1)");
    if (sched->space != space || sched->p != p || sched->nel != nel || sched->nrows != nrows ||
        sched->nnz != *nnz)
      LOR_FAIL(LOR_EINVAL, "sched does not come from phase 1 of the same pattern");
    lor_sched probe = *sched;
    if (layout(&probe, ref) != sched->dev_bytes) LOR_FAIL(LOR_EINVAL, "sched->dev_bytes changed since phase 1");
  }

  DevBuf err, st_ptr, st_col;
  if ((rc = err.alloc(sizeof(int32_t)))) return rc;
  LOR_HIP(hipMemsetAsync(err.p, 0, sizeof(int32_t), st));
  int32_t herr = 0;

  if (col_idx == nullptr) {
    // ---------------------------------------------------------------- phase 1
    DevBuf inc_ptr, inc_list, cnt, ptr64;
    if ((rc = inc_ptr.alloc(sizeof(int32_t) * (nrows + 1)))) return rc;
    if ((rc = inc_list.alloc(sizeof(int32_t) * std::max<int64_t>(1, total)))) return rc;
    if ((rc = cnt.alloc(sizeof(int32_t) * nrows))) return rc;
    if ((rc = ptr64.alloc(sizeof(int64_t) * (nrows + 1)))) return rc;
    if ((rc = st_ptr.alloc(sizeof(int32_t) * ref.st_ptr.size()))) return rc;
    if ((rc = st_col.alloc(sizeof(int32_t) * ref.st_col.size()))) return rc;
    if ((rc = upload(ref.st_ptr, st_ptr.p, st))) return rc;
    if ((rc = upload(ref.st_col, st_col.p, st))) return rc;
    if ((rc = build_incidence(elem_map, nel, nloc, is_signed, nrows, inc_ptr.as<int32_t>(),
                              inc_list.as<int32_t>(), err.as<int32_t>(), st)))
      return rc;
    if ((rc = read_err(err.as<int32_t>(), st, &herr))) return rc;
    if ((rc = report_err(herr))) return rc;
    k_row_cols<false><<<ceil_div(nrows, kRowThreads), kRowThreads, 0, st>>>(
        elem_map, nloc, is_signed, inc_ptr.as<int32_t>(), inc_list.as<int32_t>(), st_ptr.as<int32_t>(),
        st_col.as<int32_t>(), nrows, cnt.as<int32_t>(), nullptr, nullptr, err.as<int32_t>());
    LOR_LAUNCHED("k_row_cols<count>");
    if ((rc = scan_exclusive<int32_t>(cnt.as<int32_t>(), nrows, ptr64.as<int64_t>(), st))) return rc;
    int64_t total_nnz = 0;
    LOR_HIP(hipMemcpyAsync(&total_nnz, ptr64.as<int64_t>() + nrows, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    if ((rc = read_err(err.as<int32_t>(), st, &herr))) return rc;
    if ((rc = report_err(herr))) return rc;
    if (total_nnz >= INT32_MAX) LOR_FAIL(LOR_EOVERFLOW, "nnz = %lld >= 2^31", (long long)total_nnz);
    k_i64_to_i32<<<ceil_div(nrows + 1, 256), 256, 0, st>>>(ptr64.as<int64_t>(), nrows + 1, row_ptr);
    LOR_LAUNCHED("k_i64_to_i32");
    LOR_HIP(hipStreamSynchronize(st));
    *nnz = total_nnz;
    sched->space = space;
    sched->p = p;
    sched->nel = nel;
    sched->nrows = nrows;
    sched->nnz = total_nnz;
    sched->nloc = nloc;
    sched->nent = ref.nent;
    sched->ncolors = 0;
    sched->nclass = 0;
    sched->dev = nullptr;
    sched->owner = 0;
    sched->box[0] = sched->box[1] = sched->box[2] = 0;
    sched->dev_bytes = layout(sched, ref);
    return LOR_OK;
  }

  // ------------------------------------------------------------------ phase 2
  const int64_t nnzv = *nnz;
  int32_t* d_order = dev_at<int32_t>(sched, sched->off_order);
  int32_t* d_color = dev_at<int32_t>(sched, sched->off_color);
  int32_t* d_class = dev_at<int32_t>(sched, sched->off_class);
  uint8_t* d_tab = dev_at<uint8_t>(sched, sched->off_tables);
  int32_t* d_inc_ptr = dev_at<int32_t>(sched, sched->off_inc_ptr);
  int32_t* d_inc_list = dev_at<int32_t>(sched, sched->off_inc_list);
  int32_t* d_st_ptr = dev_at<int32_t>(sched, sched->off_st_ptr);
  int32_t* d_st_col = dev_at<int32_t>(sched, sched->off_st_col);
  uint16_t* d_ent_row = dev_at<uint16_t>(sched, sched->off_ent_row);
  uint64_t* d_recipe = dev_at<uint64_t>(sched, sched->off_recipe);
  DevBuf reps;
  if ((rc = reps.alloc(sizeof(int32_t) * ref.reps.size()))) return rc;
  if ((rc = upload(ref.st_ptr, d_st_ptr, st))) return rc;
  if ((rc = upload(ref.st_col, d_st_col, st))) return rc;
  if ((rc = upload(ref.ent_row, d_ent_row, st))) return rc;
  if ((rc = upload(ref.recipe64, d_recipe, st))) return rc;
  if ((rc = upload(ref.reps, reps.p, st))) return rc;
  LOR_HIP(hipMemsetAsync(dev_at<uint8_t>(sched, sched->off_zero), 0, 256, st));

  if ((rc = build_incidence(elem_map, nel, nloc, is_signed, nrows, d_inc_ptr, d_inc_list, err.as<int32_t>(), st)))
    return rc;
  k_row_cols<true><<<ceil_div(nrows, kRowThreads), kRowThreads, 0, st>>>(
      elem_map, nloc, is_signed, d_inc_ptr, d_inc_list, d_st_ptr, d_st_col, nrows, nullptr, row_ptr, col_idx,
      err.as<int32_t>());
  LOR_LAUNCHED("k_row_cols<fill>");
  if ((rc = read_err(err.as<int32_t>(), st, &herr))) return rc;
  if ((rc = report_err(herr))) return rc;

  // colouring
  DevBuf ncol;
  if ((rc = ncol.alloc(sizeof(int32_t)))) return rc;
  LOR_HIP(hipMemsetAsync(ncol.p, 0, sizeof(int32_t), st));
  if (nel > 0) {
    k_fill_i32<<<ceil_div(nel, 256), 256, 0, st>>>(d_color, nel, -1);
    LOR_LAUNCHED("k_fill_i32");
  }
  int32_t colored = 0;
  for (int64_t round = 0; colored < nel; ++round) {
    if (round > nel) LOR_FAIL(LOR_EDEVICE, "element colouring did not converge");
    k_jp_round<<<ceil_div(nel, 256), 256, 0, st>>>(elem_map, nloc, is_signed, reps.as<int32_t>(),
                                                   static_cast<int>(ref.reps.size()), d_inc_ptr, d_inc_list,
                                                   nel, d_color, ncol.as<int32_t>(), err.as<int32_t>());
    LOR_LAUNCHED("k_jp_round");
    LOR_HIP(hipMemcpyAsync(&colored, ncol.p, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    if ((rc = read_err(err.as<int32_t>(), st, &herr))) return rc;
    if ((rc = report_err(herr))) return rc;
  }
  k_check_colors<<<ceil_div(nrows, 256), 256, 0, st>>>(d_inc_ptr, d_inc_list, nloc, nrows, d_color,
                                                       err.as<int32_t>());
  LOR_LAUNCHED("k_check_colors");
  if ((rc = read_err(err.as<int32_t>(), st, &herr))) return rc;
  if ((rc = report_err(herr))) return rc;

  // element order by colour (stable)
  {
    DevBuf flags, pos;
    if ((rc = flags.alloc(sizeof(int32_t) * std::max<int64_t>(1, nel)))) return rc;
    if ((rc = pos.alloc(sizeof(int64_t) * (nel + 1)))) return rc;
    int32_t base = 0;
    int nc = 0;
    sched->color_ptr[0] = 0;
    for (int c = 0; c < LOR_MAX_COLORS && base < nel; ++c) {
      k_color_flags<<<ceil_div(nel, 256), 256, 0, st>>>(d_color, nel, c, flags.as<int32_t>());
      LOR_LAUNCHED("k_color_flags");
      if ((rc = scan_exclusive<int32_t>(flags.as<int32_t>(), nel, pos.as<int64_t>(), st))) return rc;
      k_color_scatter<<<ceil_div(nel, 256), 256, 0, st>>>(d_color, nel, c, pos.as<int64_t>(), base, d_order);
      LOR_LAUNCHED("k_color_scatter");
      int64_t cnt = 0;
      LOR_HIP(hipMemcpyAsync(&cnt, pos.as<int64_t>() + nel, sizeof(int64_t), hipMemcpyDeviceToHost, st));
      LOR_HIP(hipStreamSynchronize(st));
      base += static_cast<int32_t>(cnt);
      sched->color_ptr[c + 1] = base;
      nc = c + 1;
    }
    if (base != nel) LOR_FAIL(LOR_EDEVICE, "colour order incomplete");
    sched->ncolors = nc;
    for (int c = nc + 1; c <= LOR_MAX_COLORS; ++c) sched->color_ptr[c] = base;
  }

  // rank tables
  {
    DevBuf mincol;
    if ((rc = mincol.alloc(sizeof(int32_t) * std::max<int64_t>(1, nnzv)))) return rc;
    const int64_t tot = nel * ref.nent;
    k_fill_i32<<<ceil_div(std::max<int64_t>(1, nnzv), 256), 256, 0, st>>>(mincol.as<int32_t>(), nnzv, INT32_MAX);
    LOR_LAUNCHED("k_fill_i32");
    if (tot > 0) {
      LOR_HIP(hipMemsetAsync(d_tab, 0, static_cast<size_t>(nel) * sched->tab_stride, st));
      k_rank_pass0<<<ceil_div(tot, 256), 256, 0, st>>>(elem_map, nloc, is_signed, ref.nent, sched->tab_stride,
                                                        d_ent_row, d_st_col,
                                                        row_ptr, col_idx, d_color, tot, mincol.as<int32_t>(), d_tab,
                                                        err.as<int32_t>());
      LOR_LAUNCHED("k_rank_pass0");
      k_rank_pass1<<<ceil_div(tot, 256), 256, 0, st>>>(elem_map, nloc, is_signed, ref.nent, sched->tab_stride,
                                                        d_ent_row, row_ptr,
                                                        d_color, tot, mincol.as<int32_t>(), d_tab);
      LOR_LAUNCHED("k_rank_pass1");
    }
    if ((rc = read_err(err.as<int32_t>(), st, &herr))) return rc;
    if ((rc = report_err(herr))) return rc;
  }
  // element classes (identical rank tables share one stored table)
  sched->nclass = nel;
  if (nel > 0) {
    const int64_t words = sched->tab_stride / 4;
    uint32_t* tabw = dev_at<uint32_t>(sched, sched->off_tables);
    DevBuf hash;
    if ((rc = hash.alloc(sizeof(uint64_t) * nel))) return rc;
    k_table_hash<<<ceil_div(nel, 256), 256, 0, st>>>(tabw, words, nel, hash.as<uint64_t>());
    LOR_LAUNCHED("k_table_hash");
    std::vector<uint64_t> h(static_cast<size_t>(nel));
    LOR_HIP(hipMemcpyAsync(h.data(), hash.p, sizeof(uint64_t) * nel, hipMemcpyDeviceToHost, st));
    LOR_HIP(hipStreamSynchronize(st));
    std::unordered_map<uint64_t, int32_t> first;
    std::vector<int32_t> cls(static_cast<size_t>(nel)), rep;
    for (int64_t e = 0; e < nel; ++e) {
      auto it = first.find(h[e]);
      if (it == first.end()) {
        it = first.emplace(h[e], static_cast<int32_t>(rep.size())).first;
        rep.push_back(static_cast<int32_t>(e));
      }
      cls[e] = it->second;
    }
    const int64_t ncls = static_cast<int64_t>(rep.size());
    DevBuf drep, mism;
    if ((rc = drep.alloc(sizeof(int32_t) * ncls))) return rc;
    if ((rc = mism.alloc(sizeof(int32_t)))) return rc;
    if ((rc = upload(cls, d_class, st))) return rc;
    if ((rc = upload(rep, drep.p, st))) return rc;
    LOR_HIP(hipMemsetAsync(mism.p, 0, sizeof(int32_t), st));
    k_table_verify<<<ceil_div(nel * words, 256), 256, 0, st>>>(tabw, words, nel, d_class, drep.as<int32_t>(),
                                                              mism.as<int32_t>());
    LOR_LAUNCHED("k_table_verify");
    int32_t hm = 0;
    if ((rc = read_err(mism.as<int32_t>(), st, &hm))) return rc;
    if (hm == 0 && ncls < nel) {
      DevBuf tmp;
      if ((rc = tmp.alloc(static_cast<size_t>(ncls) * sched->tab_stride))) return rc;
      k_table_gather<<<ceil_div(ncls * words, 256), 256, 0, st>>>(tabw, words, ncls, drep.as<int32_t>(),
                                                                  tmp.as<uint32_t>());
      LOR_LAUNCHED("k_table_gather");
      LOR_HIP(hipMemcpyAsync(tabw, tmp.p, static_cast<size_t>(ncls) * sched->tab_stride, hipMemcpyDeviceToDevice,
                             st));
      LOR_HIP(hipStreamSynchronize(st));
      sched->nclass = ncls;
    } else {
      // a hash collision (or nothing to share): every element keeps its own table
      k_iota_i32<<<ceil_div(nel, 256), 256, 0, st>>>(d_class, nel);
      LOR_LAUNCHED("k_iota_i32");
    }
    k_gather_i32<<<ceil_div(nel, 256), 256, 0, st>>>(d_class, d_order, nel,
                                                    dev_at<int32_t>(sched, sched->off_order_class));
    LOR_LAUNCHED("k_gather_i32");
  }
  sched->max_row_nnz = 0;
  LOR_HIP(hipStreamSynchronize(st));
  return build_owner(sched, elem_map, row_ptr, col_idx, st);
}
