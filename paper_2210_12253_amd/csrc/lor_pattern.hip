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

static size_t align256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

// Bump allocator over one device allocation that holds the temporaries of one
// call, so that no call allocates (and, through hipFree, synchronises) per
// step.  Slices are handed out in order; release() returns everything taken
// after a mark.  All work runs on one stream, so a released slice can be
// handed out again at once.
struct Arena {
  DevBuf buf;
  size_t cap = 0, used = 0;
  int alloc(size_t bytes) {
    cap = bytes;
    used = 0;
    return buf.alloc(bytes);
  }
  template <typename T>
  T* take(size_t count) {
    const size_t end = used + align256(sizeof(T) * std::max<size_t>(count, 1));
    if (end > cap) return nullptr;
    T* r = reinterpret_cast<T*>(static_cast<char*>(buf.p) + used);
    used = end;
    return r;
  }
  void release(size_t mark) { used = mark; }
};

// Releases, on scope exit, everything taken from the arena in the scope.
struct ArenaScope {
  Arena& a;
  size_t mark;
  explicit ArenaScope(Arena& arena) : a(arena), mark(arena.used) {}
  ~ArenaScope() { a.release(mark); }
};

// Bytes an Arena::take of count T's consumes.
template <typename T>
static size_t arena_bytes(size_t count) {
  return align256(sizeof(T) * std::max<size_t>(count, 1));
}

#define LOR_TAKE(PTR, ARENA, T, N)                                             \
  do {                                                                         \
    (PTR) = (ARENA).template take<T>(N);                                       \
    if (!(PTR)) LOR_FAIL(LOR_EDEVICE, "internal error: scratch arena too small"); \
  } while (0)

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

// Scratch bytes of scan_exclusive over n values.
static size_t scan_ws_bytes(int64_t n) {
  if (n == 0) return 0;
  const int64_t nt = ceil_div(n, kScanTile);
  return 2 * arena_bytes<int64_t>(nt + 1) + (nt > 1 ? scan_ws_bytes(nt) : 0);
}

// Exclusive scan of n values into out[0..n], out[n] = total; tile sums in
// scan_ws_bytes(n) bytes of the arena.
template <typename TI>
static int scan_exclusive(const TI* in, int64_t n, int64_t* out, Arena& a, hipStream_t st) {
  if (n == 0) {
    k_scan_total<TI><<<1, 1, 0, st>>>(in, 0, out);
    LOR_LAUNCHED("k_scan_total");
    return LOR_OK;
  }
  const int64_t ntiles = ceil_div(n, kScanTile);
  ArenaScope scope(a);
  int64_t *sums, *offs;
  LOR_TAKE(sums, a, int64_t, ntiles + 1);
  LOR_TAKE(offs, a, int64_t, ntiles + 1);
  k_scan_tiles<TI><<<ntiles, kScanThreads, 0, st>>>(in, n, out, sums);
  LOR_LAUNCHED("k_scan_tiles");
  if (ntiles > 1) {
    const int rc = scan_exclusive<int64_t>(sums, ntiles, offs, a, st);
    if (rc) return rc;
    k_scan_add<<<ceil_div(n, 256), 256, 0, st>>>(out, n, offs);
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
// lanes working on the same slot hit different banks) and holds CAP columns.
// The short form (kRowCapShort: every row of the structured meshes and of the
// irregular test meshes fits) lets several waves share a SIMD; a row that
// does not fit goes to the list `ovf` and is done again by the full form
// (LOR_MAX_ROW_NNZ columns, one wave per SIMD).  `rows` (optional) lists the
// rows to do, else rows 0 .. nlist - 1.  The fill form skips, into `ovf`, the
// rows that phase 1 counted longer than CAP.
constexpr int kRowThreads = 64;
constexpr int kRowCapShort = 40;

template <bool FILL, int CAP>
__global__ __launch_bounds__(kRowThreads) void k_row_cols(
    const int32_t* __restrict__ map, int nloc, int is_signed, const int32_t* __restrict__ inc_ptr,
    const int32_t* __restrict__ inc_list, const int32_t* __restrict__ st_ptr,
    const int32_t* __restrict__ st_col, const int32_t* __restrict__ rows, int64_t nlist,
    int32_t* __restrict__ cnt, const int32_t* __restrict__ row_ptr, int32_t* __restrict__ col_idx,
    int32_t* __restrict__ ovf, int32_t* __restrict__ novf, int32_t* __restrict__ err) {
  constexpr bool FULL = CAP >= LOR_MAX_ROW_NNZ;
  constexpr int STRIDE = CAP % 2 == 0 ? CAP + 1 : CAP + 2;
  __shared__ int32_t buf[kRowThreads * STRIDE];
  const int64_t t = static_cast<int64_t>(blockIdx.x) * kRowThreads + threadIdx.x;
  if (t >= nlist) return;
  const int64_t g = rows ? rows[t] : t;
  if (FILL && !FULL && row_ptr[g + 1] - row_ptr[g] > CAP) {
    ovf[atomicAdd(novf, 1)] = static_cast<int32_t>(g);
    return;
  }
  int32_t* b = buf + threadIdx.x * STRIDE;
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
      if (n >= CAP) {
        overflow = true;
        break;
      }
      for (int m = n; m > pos; --m) b[m] = b[m - 1];
      b[pos] = c;
      ++n;
    }
  }
  if (overflow) {
    if (!FILL) cnt[g] = 0;
    if (FULL)
      atomicOr(err, kErrRowTooLong);
    else
      ovf[atomicAdd(novf, 1)] = static_cast<int32_t>(g);
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
                           int32_t* __restrict__ maxcolor, int32_t* __restrict__ err) {
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
  atomicMax(maxcolor, c);
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

// Stable sort of the elements by colour, one wave per 64 consecutive
// elements: k_color_hist counts each colour in the wave (cnt is colour-major,
// [nc][nblk]); after an exclusive scan of cnt into off, element e of colour c
// goes to off[c][wave] + (lanes below it with colour c).  Elements whose
// colour is outside [0, nc) are left out (the caller checks the total).
__global__ __launch_bounds__(64) void k_color_hist(const int32_t* __restrict__ color, int64_t nel, int nc,
                                                   int64_t nblk, int32_t* __restrict__ cnt) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * 64 + threadIdx.x;
  const int32_t c = e < nel ? color[e] : -1;
  for (int cc = 0; cc < nc; ++cc) {
    const uint64_t m = __ballot(c == cc);
    if (threadIdx.x == 0) cnt[cc * nblk + blockIdx.x] = __popcll(m);
  }
}

__global__ __launch_bounds__(64) void k_color_place(const int32_t* __restrict__ color, int64_t nel, int nc,
                                                    int64_t nblk, const int64_t* __restrict__ off,
                                                    int32_t* __restrict__ order) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * 64 + threadIdx.x;
  const int32_t c = e < nel ? color[e] : -1;
  const uint64_t below = (1ull << threadIdx.x) - 1ull;
  int64_t at = -1;
  for (int cc = 0; cc < nc; ++cc) {
    const uint64_t m = __ballot(c == cc);
    if (c == cc) at = off[cc * nblk + blockIdx.x] + __popcll(m & below);
  }
  if (at >= 0) order[at] = static_cast<int32_t>(e);
}

// Colour pointer: colour c starts at off[c][0]; off[nc * nblk] is the total.
__global__ void k_color_ptr(const int64_t* __restrict__ off, int nc, int64_t nblk, int32_t* __restrict__ cptr) {
  const int c = threadIdx.x;
  if (c <= nc) cptr[c] = static_cast<int32_t>(off[c * nblk]);
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


// ------------------------------------------------------------ box lattice (H1)
//
// An H1 mesh of degree p is a box lattice when its elements tile a box of
// nx x ny x nz elements with every element's local axes along the box axes,
// and the vertex at point (X, Y, Z) of the global lattice of
// (LX, LY, LZ) = (nx p + 1, ny p + 1, nz p + 1) points has the lexicographic
// id X + LX (Y + LY Z) -- the structured meshes of the paper's benchmarks,
// with the elements in any order.  On such a mesh everything the general path
// searches for has a closed form:
//   * two lattice points share a subcell of some element exactly when they
//     differ by at most one along every axis, so the row of (X, Y, Z) holds
//     the in-box points of its 3 x 3 x 3 neighbourhood, and their ids increase
//     in (dz, dy, dx) order.  Along one axis a point has 1 + [X > 0] +
//     [X < LX - 1] neighbours, so row lengths are products of per-axis counts
//     and the row pointer is a sum of products of their prefix sums;
//   * colouring elements by the parities of their box position is proper
//     (elements sharing a vertex differ by at most one along every axis) and
//     is what the greedy colouring produces for elements in box order;
//   * the position of an entry in its row depends only on which neighbours
//     its row point has, and its first contributor only on the colours of the
//     elements holding both points; for an element both follow from whether it
//     touches each of the six box faces and from its parities, so elements
//     agreeing in those share one rank table.
// The owner-computes value kernel relies on exactly this layout.

// Distinct class keys of k_box_color_key (9 bits): a box lattice needs at
// most this many rank tables.
constexpr int kBoxKeys = 512;

struct BoxLattice {
  int64_t LX = 0, LY = 0, LZ = 0;
  int nx = 0, ny = 0, nz = 0;
};

// Element 0's vertices at local (0,0,0), (1,0,0), (0,1,0), (0,0,1): the lattice
// strides, if the mesh is a box lattice.
__global__ void k_box_probe(const int32_t* __restrict__ map, int p, int32_t* __restrict__ out) {
  const int q = p + 1;
  const int i = threadIdx.x;
  if (i < 4) out[i] = map[i == 0 ? 0 : i == 1 ? 1 : i == 2 ? q : q * q];
}

// One thread per (element, local vertex): every vertex id must be the
// lexicographic id of its lattice point, the element's corner a lattice point
// of the element grid; the element claims its box position (pos3d starts at
// -1), and a position claimed twice marks the mesh as no box lattice.  With
// nel = nx ny nz elements placed at distinct positions, every position is
// taken.
template <int P>
__global__ void k_box_place(const int32_t* __restrict__ map, int32_t nel, int32_t LX, int32_t LY, int32_t LZ,
                            int nx, int ny, int32_t* __restrict__ elem3d, int32_t* __restrict__ flag) {
  constexpr int Q = P + 1, NLOC = Q * Q * Q;
  const int32_t t = static_cast<int32_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= nel * NLOC) return;  // nel * NLOC < 2^31
  const int32_t e = t / NLOC;
  const int l = t - e * NLOC;
  const int32_t v0 = map[e * NLOC];
  const int lx = l % Q, ly = (l / Q) % Q, lz = l / (Q * Q);
  bool bad = map[t] != v0 + lx + LX * (ly + LY * lz);
  if (l == 0) {
    const int32_t X0 = v0 % LX, Y0 = (v0 / LX) % LY, Z0 = v0 / (LX * LY);
    bad = bad || v0 < 0 || Z0 >= LZ || X0 % P != 0 || Y0 % P != 0 || Z0 % P != 0 || X0 + P >= LX ||
          Y0 + P >= LY || Z0 + P >= LZ;
    if (!bad) {
      const int64_t pos = (static_cast<int64_t>(Z0 / P) * ny + Y0 / P) * nx + X0 / P;
      bad = atomicCAS(&elem3d[pos], -1, e) != -1;
    }
  }
  // one atomic per wave at most (a mesh that is no box lattice fails almost
  // everywhere)
  const uint64_t m = __ballot(bad);
  if (m != 0 && (threadIdx.x & 63) == static_cast<unsigned>(__ffsll(static_cast<long long>(m)) - 1))
    atomicOr(flag, 1);
}

// Row pointer of the lattice pattern, entries [0, nrows].
__global__ void k_box_row_ptr(int64_t LX, int64_t LY, int64_t LZ, int32_t* __restrict__ row_ptr) {
  const int64_t n = LX * LY * LZ;
  const int64_t v = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (v > n) return;
  const int64_t SX = 3 * LX - 2, SY = 3 * LY - 2, SZ = 3 * LZ - 2;
  if (v == n) {
    row_ptr[v] = static_cast<int32_t>(SX * SY * SZ);
    return;
  }
  row_ptr[v] = static_cast<int32_t>(box_row_start(v % LX, (v / LX) % LY, v / (LX * LY), LX, LY, LZ));
}

// Columns of one lattice line (Y, Z) per workgroup: the line's rows are
// consecutive, and so are their entries; consecutive threads write
// consecutive entries.  With C = cy cz neighbour lines, row 0 holds entries
// [0, 2C), interior row X >= 1 holds [(3X - 1) C, (3X + 2) C), the last row
// the final 2C; inside a row, entries run in (dz, dy, dx) order.  The line's
// (cy, cz) are template arguments, so the divisions are by constants.  The
// caller's row pointer is checked against the lattice's.
constexpr int kBoxColThreads = 256;

template <int CY, int CZ>
__device__ __forceinline__ void box_line_cols(int32_t LX, int32_t LY, int32_t Y, int32_t Z, int64_t start,
                                              int32_t* __restrict__ col_idx) {
  constexpr int C = CY * CZ;
  const int ylo = Y > 0, zlo = Z > 0;
  // id of lattice point (0, Y - ylo + iy, Z - zlo + iz) = b0 + iz LX LY + iy LX
  const int32_t b0 = ((Z - zlo) * LY + (Y - ylo)) * LX;
  const int32_t lxy = LX * LY;
  const int32_t total = (3 * LX - 2) * C, last = (3 * LX - 4) * C;
  for (int32_t o = threadIdx.x; o < total; o += kBoxColThreads) {
    int32_t X, izy, col;
    if (o < 2 * C) {  // row 0: dx in {0, 1}
      X = 0;
      izy = o >> 1;
      col = o & 1;
    } else if (o >= last) {  // row LX - 1: dx in {-1, 0}
      const int32_t u = o - last;
      X = LX - 1;
      izy = u >> 1;
      col = X - 1 + (u & 1);
    } else {  // interior row: dx in {-1, 0, 1}
      const int32_t w = o - 2 * C;
      const int32_t r = w / (3 * C);
      const int32_t u = w - r * (3 * C);
      X = r + 1;
      izy = u / 3;
      col = X - 1 + (u - 3 * izy);
    }
    const int32_t iz = izy / CY, iy = izy - iz * CY;
    col_idx[start + o] = b0 + iz * lxy + iy * LX + col;
  }
}

__global__ __launch_bounds__(kBoxColThreads) void k_box_cols(int32_t LX, int32_t LY, int32_t LZ,
                                                             const int32_t* __restrict__ row_ptr,
                                                             int32_t* __restrict__ col_idx,
                                                             int32_t* __restrict__ err) {
  const int32_t line = blockIdx.x;
  const int32_t Y = line % LY, Z = line / LY;
  const int cy = box_count(Y, LY), cz = box_count(Z, LZ), cyz = cy * cz;
  const int64_t SX = 3 * static_cast<int64_t>(LX) - 2, SY = 3 * static_cast<int64_t>(LY) - 2;
  const int64_t start = box_prefix(Z, LZ) * SY * SX + cz * box_prefix(Y, LY) * SX;
  const int64_t v0 = static_cast<int64_t>(line) * LX;
  bool bad = false;
  for (int32_t X = threadIdx.x; X <= LX; X += kBoxColThreads)
    bad = bad || row_ptr[v0 + X] != start + cyz * box_prefix(X, LX);
  if (bad) atomicOr(err, kErrRowCount);
  // cy, cz in {2, 3}: every axis has at least two lattice points
  switch (cy * 4 + cz) {
#define LOR_BOX_LINE(A, B)                             \
  case A * 4 + B:                                      \
    box_line_cols<A, B>(LX, LY, Y, Z, start, col_idx); \
    break;
    LOR_BOX_LINE(2, 2)
    LOR_BOX_LINE(2, 3)
    LOR_BOX_LINE(3, 2)
    LOR_BOX_LINE(3, 3)
#undef LOR_BOX_LINE
    default:
      break;
  }
}

// Per box position: the element's colour (parities, over the axes with more
// than one element) and its table class key (per axis: touches the low face,
// touches the high face, parity).
__global__ void k_box_color_key(const int32_t* __restrict__ elem3d, int nx, int ny, int nz, int wx, int wy, int wz,
                                int32_t* __restrict__ color, int32_t* __restrict__ key) {
  const int64_t pos = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (pos >= static_cast<int64_t>(nx) * ny * nz) return;
  const int ex = static_cast<int>(pos % nx), ey = static_cast<int>((pos / nx) % ny);
  const int ez = static_cast<int>(pos / (static_cast<int64_t>(nx) * ny));
  const int32_t e = elem3d[pos];
  color[e] = (ex & 1) * wx + (ey & 1) * wy + (ez & 1) * wz;
  auto axis = [](int c, int n) { return (c == 0 ? 1 : 0) | (c == n - 1 ? 2 : 0) | ((c & 1) << 2); };
  key[e] = axis(ex, nx) | (axis(ey, ny) << 3) | (axis(ez, nz) << 6);
}

// Rank table of class c from its representative element rep[c]: position of
// every stencil entry in its row, and the first-contributor bit (the
// element's colour is the lowest among the elements holding both points of
// the entry; on a box lattice every element holding both has the entry).
// Padding bytes of the table are zeroed.
__global__ void k_box_rank(const int32_t* __restrict__ map, int nloc, int nent, int64_t stride,
                           const uint16_t* __restrict__ ent_row, const int32_t* __restrict__ ent_col,
                           const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col_idx,
                           const int32_t* __restrict__ color, const int32_t* __restrict__ inc_ptr,
                           const int32_t* __restrict__ inc_list, const int32_t* __restrict__ rep, int64_t ncls,
                           uint8_t* __restrict__ tables, int32_t* __restrict__ err) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= ncls * stride) return;
  const int64_t c = idx / stride;
  const int k = static_cast<int>(idx - c * stride);
  uint8_t* tab = tables + idx;
  if (k >= nent) {
    *tab = 0;
    return;
  }
  const int32_t e = rep[c];
  const int32_t* me = map + static_cast<int64_t>(e) * nloc;
  const int32_t g = me[ent_row[k]], col = me[ent_col[k]];
  int32_t lo = row_ptr[g], hi = row_ptr[g + 1];
  const int32_t start = lo;
  while (lo < hi) {
    const int32_t mid = (lo + hi) >> 1;
    if (col_idx[mid] < col)
      lo = mid + 1;
    else
      hi = mid;
  }
  if (lo >= row_ptr[g + 1] || col_idx[lo] != col) {
    atomicOr(err, kErrRankMissing);
    *tab = 0;
    return;
  }
  int32_t lowest = INT32_MAX;
  for (int32_t i = inc_ptr[g]; i < inc_ptr[g + 1]; ++i) {
    const int32_t f = inc_list[i] / nloc;
    for (int32_t j = inc_ptr[col]; j < inc_ptr[col + 1]; ++j)
      if (inc_list[j] / nloc == f) {
        lowest = min(lowest, color[f]);
        break;
      }
  }
  *tab = static_cast<uint8_t>((lo - start) | (lowest == color[e] ? kFirstBit : 0));
}

// base(Y, Z) = id of lattice point (0, Y, Z), read by the owner-computes kernel.
__global__ void k_box_base(int64_t LX, int64_t nlines, int32_t* __restrict__ base) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t < nlines) base[t] = static_cast<int32_t>(t * LX);
}

// 2D box lattices (quadrilateral H1 meshes): the same, one dimension down.
// The vertex at lattice point (X, Y) of the LX x LY points has id X + LX Y;
// the row of (X, Y) holds the in-box points of its 3 x 3 neighbourhood in
// (dy, dx) order, so row starts are box_prefix(Y) (3 LX - 2) + box_count(Y)
// box_prefix(X).  Element 0's vertices at local (0, 0), (1, 0), (0, 1) give
// the strides.
__global__ void k_box2d_probe(const int32_t* __restrict__ map, int p, int32_t* __restrict__ out) {
  const int i = threadIdx.x;
  if (i < 3) out[i] = map[i == 0 ? 0 : i == 1 ? 1 : p + 1];
}

template <int P>
__global__ void k_box2d_place(const int32_t* __restrict__ map, int32_t nel, int32_t LX, int32_t LY, int nx,
                              int32_t* __restrict__ elem2d, int32_t* __restrict__ flag) {
  constexpr int Q = P + 1, NLOC = Q * Q;
  const int32_t t = static_cast<int32_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= nel * NLOC) return;  // nel * NLOC < 2^31
  const int32_t e = t / NLOC;
  const int l = t - e * NLOC;
  const int32_t v0 = map[e * NLOC];
  bool bad = map[t] != v0 + (l % Q) + LX * (l / Q);
  if (l == 0) {
    const int32_t X0 = v0 % LX, Y0 = v0 / LX;
    bad = bad || v0 < 0 || Y0 >= LY || X0 % P != 0 || Y0 % P != 0 || X0 + P >= LX || Y0 + P >= LY;
    if (!bad) bad = atomicCAS(&elem2d[static_cast<int64_t>(Y0 / P) * nx + X0 / P], -1, e) != -1;
  }
  const uint64_t m = __ballot(bad);
  if (m != 0 && (threadIdx.x & 63) == static_cast<unsigned>(__ffsll(static_cast<long long>(m)) - 1))
    atomicOr(flag, 1);
}

// Face lattices (H(div) meshes): with (MX, MY, MZ) cells, the x-face at
// lattice x = X of cell row (Y, Z) has id X + (MX + 1)(Y + MY Z), y-faces
// OY + X + MX (Y + (MY + 1) Z) with OY = (MX + 1) MY MZ, z-faces
// OZ + X + MX (Y + MY Z) with OZ = OY + MX (MY + 1) MZ.  Element 0's local
// x-faces (0,0,0) and (1,0,0), y-faces (0,0,0) and (0,1,0), z-faces (0,0,0)
// and (0,0,1) give the strides 1, MX and MX MY (signs dropped; these faces
// exist at every p, also p = 1, where an element has one cell); one thread
// per (element, local face) checks every id against the element's box
// position, which its local x-face (0,0,0) gives.
__device__ __forceinline__ int32_t face_id(int32_t v) { return v < 0 ? -1 - v : v; }

__global__ void k_facebox_probe(const int32_t* __restrict__ map, int p, int32_t* __restrict__ out) {
  const int q = p + 1, nx = p * p * q, i = threadIdx.x;
  const int at[6] = {0, 1, nx, nx + p, 2 * nx, 2 * nx + p * p};
  if (i < 6) out[i] = face_id(map[at[i]]);
}

template <int P>
__global__ void k_facebox_place(const int32_t* __restrict__ map, int32_t nel, int32_t MX, int32_t MY, int32_t MZ,
                                int nx, int ny, int32_t* __restrict__ elem3d, int32_t* __restrict__ flag) {
  constexpr int Q = P + 1, NF = 3 * P * P * Q, NX = P * P * Q;
  const int32_t t = static_cast<int32_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= nel * NF) return;  // nel * NF < 2^31
  const int32_t e = t / NF;
  const int l = t - e * NF;
  const int64_t f0 = face_id(map[static_cast<int64_t>(e) * NF]);
  const int64_t X0 = f0 % (MX + 1), Y0 = (f0 / (MX + 1)) % MY, Z0 = f0 / ((MX + 1) * static_cast<int64_t>(MY));
  const int64_t OY = (MX + 1) * static_cast<int64_t>(MY) * MZ, OZ = OY + MX * static_cast<int64_t>(MY + 1) * MZ;
  int64_t want;
  if (l < NX) {
    const int i = l % Q, j = (l / Q) % P, k = l / (Q * P);
    want = (X0 + i) + (MX + 1) * ((Y0 + j) + MY * (Z0 + k));
  } else if (l < 2 * NX) {
    const int r = l - NX, i = r % P, j = (r / P) % Q, k = r / (P * Q);
    want = OY + (X0 + i) + MX * ((Y0 + j) + (MY + 1) * (Z0 + k));
  } else {
    const int r = l - 2 * NX, i = r % P, j = (r / P) % P, k = r / (P * P);
    want = OZ + (X0 + i) + MX * ((Y0 + j) + MY * (Z0 + k));
  }
  bool bad = face_id(map[t]) != want;
  if (l == 0) {
    bad = bad || Z0 >= MZ || X0 % P != 0 || Y0 % P != 0 || Z0 % P != 0 || X0 + P > MX || Y0 + P > MY ||
          Z0 + P > MZ;
    if (!bad) bad = atomicCAS(&elem3d[((Z0 / P) * ny + Y0 / P) * nx + X0 / P], -1, e) != -1;
  }
  const uint64_t m = __ballot(bad);
  if (m != 0 && (threadIdx.x & 63) == static_cast<unsigned>(__ffsll(static_cast<long long>(m)) - 1))
    atomicOr(flag, 1);
}

// The caller's row pointer against the face lattice's closed form: rows of
// x-faces, then y-faces, then z-faces; 6 entries on the box boundary, 11
// inside.
__device__ __forceinline__ int64_t fl_prefix(int64_t X, int64_t M) {
  return X <= 0 ? 0 : X <= M ? 6 + 11 * (X - 1) : 12 + 11 * (M - 1);
}
__global__ void k_facebox_rows(const int32_t* __restrict__ row_ptr, int64_t MX, int64_t MY, int64_t MZ,
                               int32_t* __restrict__ flag) {
  const int64_t OY = (MX + 1) * MY * MZ, OZ = OY + MX * (MY + 1) * MZ, n = OZ + MX * MY * (MZ + 1);
  const int64_t f = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (f > n) return;
  const int64_t nx = MY * MZ * fl_prefix(MX + 1, MX), ny = MZ * MX * fl_prefix(MY + 1, MY);
  int64_t want;
  if (f == n) {
    want = nx + ny + MX * MY * fl_prefix(MZ + 1, MZ);
  } else if (f < OY) {
    const int64_t X = f % (MX + 1), YZ = f / (MX + 1);
    want = YZ * fl_prefix(MX + 1, MX) + fl_prefix(X, MX);
  } else if (f < OZ) {
    const int64_t r = f - OY, X = r % MX, Y = (r / MX) % (MY + 1), Z = r / (MX * (MY + 1));
    want = nx + Z * MX * fl_prefix(MY + 1, MY) + MX * fl_prefix(Y, MY) + X * ((Y == 0 || Y == MY) ? 6 : 11);
  } else {
    const int64_t r = f - OZ, XY = r % (MX * MY), Z = r / (MX * MY);
    want = nx + ny + MX * MY * fl_prefix(Z, MZ) + XY * ((Z == 0 || Z == MZ) ? 6 : 11);
  }
  if (row_ptr[f] != want) atomicOr(flag, 1);
}

// Edge lattices (H(curl) meshes): with (MX, MY, MZ) cells, the x-edge from
// lattice point (X, Y, Z) has id X + MX (Y + (MY + 1) Z), y-edges
// OY + X + (MX + 1)(Y + MY Z) with OY = MX (MY + 1)(MZ + 1), z-edges
// OZ + X + (MX + 1)(Y + (MY + 1) Z) with OZ = OY + (MX + 1) MY (MZ + 1).
// Element 0's local x-edges (0,0,0), (0,1,0) and y-edges (0,0,0), (1,0,0),
// (0,0,1) give the strides 1, MX and (MX + 1) MY (they exist at every p).
__global__ void k_edgebox_probe(const int32_t* __restrict__ map, int p, int32_t* __restrict__ out) {
  const int q = p + 1, ny = p * q * q, i = threadIdx.x;
  const int at[5] = {0, p, ny, ny + 1, ny + q * p};
  if (i < 5) out[i] = face_id(map[at[i]]);
}

template <int P>
__global__ void k_edgebox_place(const int32_t* __restrict__ map, int32_t nel, int32_t MX, int32_t MY, int32_t MZ,
                                int nx, int ny, int32_t* __restrict__ elem3d, int32_t* __restrict__ flag) {
  constexpr int Q = P + 1, NE = 3 * P * Q * Q, NX = P * Q * Q;
  const int32_t t = static_cast<int32_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= nel * NE) return;  // nel * NE < 2^31
  const int32_t e = t / NE;
  const int l = t - e * NE;
  const int64_t f0 = face_id(map[static_cast<int64_t>(e) * NE]);
  const int64_t X0 = f0 % MX, Y0 = (f0 / MX) % (MY + 1), Z0 = f0 / (MX * static_cast<int64_t>(MY + 1));
  const int64_t OY = MX * static_cast<int64_t>(MY + 1) * (MZ + 1), OZ = OY + (MX + 1) * static_cast<int64_t>(MY) * (MZ + 1);
  int64_t want;
  if (l < NX) {
    const int i = l % P, j = (l / P) % Q, k = l / (P * Q);
    want = (X0 + i) + MX * ((Y0 + j) + (MY + 1) * (Z0 + k));
  } else if (l < 2 * NX) {
    const int r = l - NX, i = r % Q, j = (r / Q) % P, k = r / (Q * P);
    want = OY + (X0 + i) + (MX + 1) * ((Y0 + j) + MY * (Z0 + k));
  } else {
    const int r = l - 2 * NX, i = r % Q, j = (r / Q) % Q, k = r / (Q * Q);
    want = OZ + (X0 + i) + (MX + 1) * ((Y0 + j) + (MY + 1) * (Z0 + k));
  }
  bool bad = face_id(map[t]) != want;
  if (l == 0) {
    bad = bad || Z0 > MZ || X0 % P != 0 || Y0 % P != 0 || Z0 % P != 0 || X0 + P > MX || Y0 + P > MY ||
          Z0 + P > MZ;
    if (!bad) bad = atomicCAS(&elem3d[((Z0 / P) * ny + Y0 / P) * nx + X0 / P], -1, e) != -1;
  }
  const uint64_t m = __ballot(bad);
  if (m != 0 && (threadIdx.x & 63) == static_cast<unsigned>(__ffsll(static_cast<long long>(m)) - 1))
    atomicOr(flag, 1);
}

// The caller's CSR pattern against the edge lattice's closed form: the row
// of an edge along m holds the edges of the <= 4 cells around it, sorted:
// x-edges, y-edges, z-edges, each group in (z, y, x) order over per-axis
// ranges (along m: the edge's cell for its own group, the 2 end nodes for
// the others; along another axis d: the cells d - 1, d for the group along
// d, the nodes d - 1 .. d + 1 for the others, as far as they exist).
__global__ void k_edgebox_rows(const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col_idx, int64_t MX,
                               int64_t MY, int64_t MZ, int32_t* __restrict__ flag) {
  const int64_t L[3] = {MX, MY, MZ};
  const int64_t OY = MX * (MY + 1) * (MZ + 1), OZ = OY + (MX + 1) * MY * (MZ + 1);
  const int64_t n = OZ + (MX + 1) * (MY + 1) * MZ;
  const int64_t f = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (f >= n) return;
  int m;
  int64_t c[3];
  if (f < OY) {
    m = 0;
    c[0] = f % MX;
    c[1] = (f / MX) % (MY + 1);
    c[2] = f / (MX * (MY + 1));
  } else if (f < OZ) {
    const int64_t r = f - OY;
    m = 1;
    c[0] = r % (MX + 1);
    c[1] = (r / (MX + 1)) % MY;
    c[2] = r / ((MX + 1) * MY);
  } else {
    const int64_t r = f - OZ;
    m = 2;
    c[0] = r % (MX + 1);
    c[1] = (r / (MX + 1)) % (MY + 1);
    c[2] = r / ((MX + 1) * (MY + 1));
  }
  int64_t start = row_ptr[f], pos = 0;
  bool bad = false;
  for (int g = 0; g < 3; ++g) {
    int64_t lo[3], cnt[3];
    for (int d = 0; d < 3; ++d) {
      if (d == m) {
        lo[d] = c[d];
        cnt[d] = g == m ? 1 : 2;
      } else {
        lo[d] = c[d] - (c[d] > 0);
        cnt[d] = (g == d ? 0 : 1) + (c[d] > 0) + (c[d] < L[d]);
      }
    }
    for (int64_t iz = 0; iz < cnt[2]; ++iz)
      for (int64_t iy = 0; iy < cnt[1]; ++iy)
        for (int64_t ix = 0; ix < cnt[0]; ++ix) {
          const int64_t x = lo[0] + ix, y = lo[1] + iy, z = lo[2] + iz;
          const int64_t want = g == 0   ? x + MX * (y + (MY + 1) * z)
                               : g == 1 ? OY + x + (MX + 1) * (y + MY * z)
                                        : OZ + x + (MX + 1) * (y + (MY + 1) * z);
          if (start + pos >= row_ptr[f + 1] || col_idx[start + pos] != want) bad = true;
          ++pos;
        }
  }
  if (start + pos != row_ptr[f + 1]) bad = true;
  if (bad) atomicOr(flag, 1);
}

// The caller's row pointer against the 2D lattice's closed form.
__global__ void k_box2d_rows(const int32_t* __restrict__ row_ptr, int64_t LX, int64_t LY, int32_t* __restrict__ flag) {
  const int64_t n = LX * LY;
  const int64_t v = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (v > n) return;
  const int64_t want = v == n ? (3 * LX - 2) * (3 * LY - 2)
                              : box_prefix(v / LX, LY) * (3 * LX - 2) + box_count(v / LX, LY) * box_prefix(v % LX, LX);
  if (row_ptr[v] != want) atomicOr(flag, 1);
}

// --------------------------------------------------------------- host side

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
  // one rank table per element at most; a box lattice (found in phase 1) has
  // at most kBoxKeys distinct ones
  const int64_t ntab = (s->owner && s->space == LOR_H1) ? std::min<int64_t>(s->nel, kBoxKeys) : s->nel;
  s->off_tables = take(static_cast<size_t>(ntab) * s->tab_stride);
  s->off_inc_ptr = take(sizeof(int32_t) * (s->nrows + 1));
  s->off_inc_list = take(sizeof(int32_t) * s->nel * r.nloc);
  s->off_st_ptr = take(sizeof(int32_t) * r.st_ptr.size());
  s->off_st_col = take(sizeof(int32_t) * r.st_col.size());
  s->off_ent_row = take(sizeof(uint16_t) * r.ent_row.size());
  s->off_recipe = take(sizeof(uint64_t) * std::max<size_t>(1, r.recipe64.size()));
  s->off_zero = take(256);
  s->off_order_class = take(sizeof(int32_t) * s->nel);
  s->off_elem3d = take(sizeof(int32_t) * s->nel);
  // a box has (LY)(LZ) = nrows / LX lattice lines along x, and LX >= p + 1
  s->off_base = take(sizeof(int32_t) * (s->nrows / (s->p + 1) + 1));
  return off;
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

// Scratch bytes of build_incidence.
static size_t incidence_ws_bytes(int64_t nrows) {
  return arena_bytes<int32_t>(nrows + 1) + arena_bytes<int64_t>(nrows + 1) + scan_ws_bytes(nrows);
}

// Incidence lists (transpose of the element map) into inc_ptr / inc_list.
static int build_incidence(const int32_t* map, int64_t nel, int nloc, int is_signed, int64_t nrows,
                           int32_t* inc_ptr, int32_t* inc_list, int32_t* d_err, Arena& a, hipStream_t st) {
  const int64_t total = nel * nloc;
  ArenaScope scope(a);
  int32_t* cnt;
  int64_t* ptr64;
  LOR_TAKE(cnt, a, int32_t, nrows + 1);
  LOR_TAKE(ptr64, a, int64_t, nrows + 1);
  LOR_HIP(hipMemsetAsync(cnt, 0, sizeof(int32_t) * (nrows + 1), st));
  if (total > 0) {
    k_count_inc<<<ceil_div(total, 256), 256, 0, st>>>(map, total, nrows, is_signed, cnt, d_err);
    LOR_LAUNCHED("k_count_inc");
  }
  int rc = scan_exclusive<int32_t>(cnt, nrows, ptr64, a, st);
  if (rc) return rc;
  k_i64_to_i32<<<ceil_div(nrows + 1, 256), 256, 0, st>>>(ptr64, nrows + 1, inc_ptr);
  LOR_LAUNCHED("k_i64_to_i32");
  LOR_HIP(hipMemsetAsync(cnt, 0, sizeof(int32_t) * (nrows + 1), st));
  if (total > 0) {
    k_fill_inc<<<ceil_div(total, 256), 256, 0, st>>>(map, total, nrows, is_signed, inc_ptr, cnt, inc_list);
    LOR_LAUNCHED("k_fill_inc");
  }
  k_sort_inc<<<ceil_div(nrows, 256), 256, 0, st>>>(inc_ptr, inc_list, nrows);
  LOR_LAUNCHED("k_sort_inc");
  return LOR_OK;
}

// Both passes of k_row_cols over all rows: the short form, then the full
// form over the rows that did not fit (one host read of their number).
// Scratch: ovf_ws_bytes(nrows).
static size_t ovf_ws_bytes(int64_t nrows) { return arena_bytes<int32_t>(nrows) + arena_bytes<int32_t>(1); }

template <bool FILL>
static int row_cols(const int32_t* map, int nloc, int is_signed, const int32_t* inc_ptr, const int32_t* inc_list,
                    const int32_t* st_ptr, const int32_t* st_col, int64_t nrows, int32_t* cnt, const int32_t* row_ptr,
                    int32_t* col_idx, int32_t* d_err, Arena& a, hipStream_t st) {
  if (nrows == 0) return LOR_OK;
  ArenaScope scope(a);
  int32_t *ovf, *novf;
  LOR_TAKE(ovf, a, int32_t, nrows);
  LOR_TAKE(novf, a, int32_t, 1);
  LOR_HIP(hipMemsetAsync(novf, 0, sizeof(int32_t), st));
  k_row_cols<FILL, kRowCapShort><<<ceil_div(nrows, kRowThreads), kRowThreads, 0, st>>>(
      map, nloc, is_signed, inc_ptr, inc_list, st_ptr, st_col, nullptr, nrows, cnt, row_ptr, col_idx, ovf, novf,
      d_err);
  LOR_LAUNCHED("k_row_cols<short>");
  int32_t h = 0;
  if (int rc = read_err(novf, st, &h)) return rc;
  if (h > 0) {
    k_row_cols<FILL, LOR_MAX_ROW_NNZ><<<ceil_div(h, kRowThreads), kRowThreads, 0, st>>>(
        map, nloc, is_signed, inc_ptr, inc_list, st_ptr, st_col, ovf, h, cnt, row_ptr, col_idx, nullptr, nullptr,
        d_err);
    LOR_LAUNCHED("k_row_cols<full>");
  }
  return LOR_OK;
}

// Box-lattice detection of an H1 mesh (see the box lattice kernels): the
// lattice strides from element 0, then every element checked and placed in
// elem3d (nel int32, device).  *found is false when the mesh is no box
// lattice; an error is returned only for device failures.
static int find_box(const int32_t* map, int p, int64_t nel, int64_t nrows, int32_t* elem3d, Arena& a,
                    hipStream_t st, BoxLattice* box, bool* found) {
  *found = false;
  if (nel == 0) return LOR_OK;
  ArenaScope scope(a);
  int32_t* probe;
  LOR_TAKE(probe, a, int32_t, 5);
  int rc;
  k_box_probe<<<1, 64, 0, st>>>(map, p, probe);
  LOR_LAUNCHED("k_box_probe");
  int32_t h[4];
  LOR_HIP(hipMemcpyAsync(h, probe, sizeof(h), hipMemcpyDeviceToHost, st));
  LOR_HIP(hipStreamSynchronize(st));
  const int64_t q = p + 1;
  const int64_t LX = static_cast<int64_t>(h[2]) - h[0], LXY = static_cast<int64_t>(h[3]) - h[0];
  if (static_cast<int64_t>(h[1]) - h[0] != 1 || LX < q || LXY < LX * q || LXY % LX != 0 || nrows % LXY != 0)
    return LOR_OK;
  const int64_t LY = LXY / LX, LZ = nrows / LXY;
  if (LZ < q || (LX - 1) % p != 0 || (LY - 1) % p != 0 || (LZ - 1) % p != 0) return LOR_OK;
  const int64_t nx = (LX - 1) / p, ny = (LY - 1) / p, nz = (LZ - 1) / p;
  if (nx * ny * nz != nel) return LOR_OK;
  int32_t* flag = probe + 4;
  LOR_HIP(hipMemsetAsync(flag, 0, sizeof(int32_t), st));
  k_fill_i32<<<ceil_div(nel, 256), 256, 0, st>>>(elem3d, nel, -1);
  LOR_LAUNCHED("k_fill_i32");
  const int64_t threads = nel * q * q * q;
  const int32_t lx = static_cast<int32_t>(LX), ly = static_cast<int32_t>(LY), lz = static_cast<int32_t>(LZ);
  const int32_t ne = static_cast<int32_t>(nel);
  const int inx = static_cast<int>(nx), iny = static_cast<int>(ny);
  switch (p) {
#define LOR_BOX_PLACE(PP)                                                                              \
  case PP:                                                                                             \
    k_box_place<PP><<<ceil_div(threads, 256), 256, 0, st>>>(map, ne, lx, ly, lz, inx, iny, elem3d, flag); \
    break;
    LOR_BOX_PLACE(1)
    LOR_BOX_PLACE(2)
    LOR_BOX_PLACE(3)
    LOR_BOX_PLACE(4)
    LOR_BOX_PLACE(5)
    LOR_BOX_PLACE(6)
#undef LOR_BOX_PLACE
    default:
      LOR_FAIL(LOR_EINVAL, "p = %d outside [1, %d]", p, LOR_MAX_P);
  }
  LOR_LAUNCHED("k_box_place");
  int32_t hflag = 0;
  if ((rc = read_err(flag, st, &hflag))) return rc;
  if (hflag != 0) return LOR_OK;
  box->LX = LX;
  box->LY = LY;
  box->LZ = LZ;
  box->nx = static_cast<int>(nx);
  box->ny = static_cast<int>(ny);
  box->nz = static_cast<int>(nz);
  *found = true;
  return LOR_OK;
}

// 2D box-lattice detection of a quadrilateral H1 mesh, after its general
// schedule: every element checked and placed in elem2d (nel int32, device),
// and row_ptr checked against the lattice's closed form.  *found is false
// when the mesh is no 2D box lattice.
static int find_box_2d(const int32_t* map, int p, int64_t nel, int64_t nrows, const int32_t* row_ptr,
                       int32_t* elem2d, Arena& a, hipStream_t st, BoxLattice* box, bool* found) {
  *found = false;
  if (nel == 0) return LOR_OK;
  ArenaScope scope(a);
  int32_t* probe;
  LOR_TAKE(probe, a, int32_t, 5);
  int rc;
  k_box2d_probe<<<1, 64, 0, st>>>(map, p, probe);
  LOR_LAUNCHED("k_box2d_probe");
  int32_t h[3];
  LOR_HIP(hipMemcpyAsync(h, probe, sizeof(h), hipMemcpyDeviceToHost, st));
  LOR_HIP(hipStreamSynchronize(st));
  const int64_t LX = static_cast<int64_t>(h[2]) - h[0];
  if (static_cast<int64_t>(h[1]) - h[0] != 1 || LX < p + 1 || nrows % LX != 0) return LOR_OK;
  const int64_t LY = nrows / LX;
  if (LY < p + 1 || (LX - 1) % p != 0 || (LY - 1) % p != 0) return LOR_OK;
  const int64_t nx = (LX - 1) / p, ny = (LY - 1) / p;
  if (nx * ny != nel) return LOR_OK;
  int32_t* flag = probe + 4;
  LOR_HIP(hipMemsetAsync(flag, 0, sizeof(int32_t), st));
  k_fill_i32<<<ceil_div(nel, 256), 256, 0, st>>>(elem2d, nel, -1);
  LOR_LAUNCHED("k_fill_i32");
  const int64_t q = p + 1, threads = nel * q * q;
  const int32_t lx = static_cast<int32_t>(LX), ly = static_cast<int32_t>(LY), ne = static_cast<int32_t>(nel);
  const int inx = static_cast<int>(nx);
  switch (p) {
#define LOR_BOX2D_PLACE(PP)                                                                                  \
  case PP:                                                                                                   \
    k_box2d_place<PP><<<ceil_div(threads, 256), 256, 0, st>>>(map, ne, lx, ly, inx, elem2d, flag);           \
    break;
    LOR_BOX2D_PLACE(1)
    LOR_BOX2D_PLACE(2)
    LOR_BOX2D_PLACE(3)
    LOR_BOX2D_PLACE(4)
    LOR_BOX2D_PLACE(5)
    LOR_BOX2D_PLACE(6)
#undef LOR_BOX2D_PLACE
    default:
      LOR_FAIL(LOR_EINVAL, "p = %d outside [1, %d]", p, LOR_MAX_P);
  }
  LOR_LAUNCHED("k_box2d_place");
  k_box2d_rows<<<ceil_div(nrows + 1, 256), 256, 0, st>>>(row_ptr, LX, LY, flag);
  LOR_LAUNCHED("k_box2d_rows");
  int32_t hflag = 0;
  if ((rc = read_err(flag, st, &hflag))) return rc;
  if (hflag != 0) return LOR_OK;
  box->LX = LX;
  box->LY = LY;
  box->LZ = 1;
  box->nx = static_cast<int>(nx);
  box->ny = static_cast<int>(ny);
  box->nz = 1;
  *found = true;
  return LOR_OK;
}

// Face-lattice detection of an H(div) mesh, after its general schedule:
// every element checked and placed in elem3d, row_ptr checked against the
// closed form.  *found is false when the face map is no face lattice.
static int find_face_box(const int32_t* map, int p, int64_t nel, int64_t nrows, const int32_t* row_ptr,
                         int32_t* elem3d, Arena& a, hipStream_t st, BoxLattice* box, bool* found) {
  *found = false;
  if (nel == 0) return LOR_OK;
  ArenaScope scope(a);
  int32_t* probe;
  LOR_TAKE(probe, a, int32_t, 7);
  int rc;
  k_facebox_probe<<<1, 64, 0, st>>>(map, p, probe);
  LOR_LAUNCHED("k_facebox_probe");
  int32_t h[6];
  LOR_HIP(hipMemcpyAsync(h, probe, sizeof(h), hipMemcpyDeviceToHost, st));
  LOR_HIP(hipStreamSynchronize(st));
  const int64_t MX = static_cast<int64_t>(h[3]) - h[2];
  if (static_cast<int64_t>(h[1]) - h[0] != 1 || MX < p || MX % p != 0) return LOR_OK;
  const int64_t dz = static_cast<int64_t>(h[5]) - h[4];
  if (dz <= 0 || dz % MX != 0) return LOR_OK;
  const int64_t MY = dz / MX;
  // nrows = (MX + 1) MY MZ + MX (MY + 1) MZ + MX MY (MZ + 1)
  const int64_t per_z = (MX + 1) * MY + MX * (MY + 1) + MX * MY;
  if (MY < p || MY % p != 0 || nrows < MX * MY || (nrows - MX * MY) % per_z != 0) return LOR_OK;
  const int64_t MZ = (nrows - MX * MY) / per_z;
  if (MZ < p || MZ % p != 0) return LOR_OK;
  const int64_t nx = MX / p, ny = MY / p, nz = MZ / p;
  if (nx * ny * nz != nel) return LOR_OK;
  int32_t* flag = probe + 6;
  LOR_HIP(hipMemsetAsync(flag, 0, sizeof(int32_t), st));
  k_fill_i32<<<ceil_div(nel, 256), 256, 0, st>>>(elem3d, nel, -1);
  LOR_LAUNCHED("k_fill_i32");
  const int64_t threads = nel * 3 * p * p * (p + 1);
  const int32_t mx = static_cast<int32_t>(MX), my = static_cast<int32_t>(MY), mz = static_cast<int32_t>(MZ);
  const int32_t ne = static_cast<int32_t>(nel);
  const int inx = static_cast<int>(nx), iny = static_cast<int>(ny);
  switch (p) {
#define LOR_FACEBOX_PLACE(PP)                                                                                    \
  case PP:                                                                                                       \
    k_facebox_place<PP><<<ceil_div(threads, 256), 256, 0, st>>>(map, ne, mx, my, mz, inx, iny, elem3d, flag);    \
    break;
    LOR_FACEBOX_PLACE(1)
    LOR_FACEBOX_PLACE(2)
    LOR_FACEBOX_PLACE(3)
    LOR_FACEBOX_PLACE(4)
    LOR_FACEBOX_PLACE(5)
    LOR_FACEBOX_PLACE(6)
#undef LOR_FACEBOX_PLACE
    default:
      LOR_FAIL(LOR_EINVAL, "p = %d outside [1, %d]", p, LOR_MAX_P);
  }
  LOR_LAUNCHED("k_facebox_place");
  k_facebox_rows<<<ceil_div(nrows + 1, 256), 256, 0, st>>>(row_ptr, MX, MY, MZ, flag);
  LOR_LAUNCHED("k_facebox_rows");
  int32_t hflag = 0;
  if ((rc = read_err(flag, st, &hflag))) return rc;
  if (hflag != 0) return LOR_OK;
  box->LX = MX;
  box->LY = MY;
  box->LZ = MZ;
  box->nx = static_cast<int>(nx);
  box->ny = static_cast<int>(ny);
  box->nz = static_cast<int>(nz);
  *found = true;
  return LOR_OK;
}

// Edge-lattice detection of an H(curl) mesh, after its general schedule:
// every element checked and placed in elem3d, the CSR pattern checked
// against the closed form.  *found is false when the edge map is no edge
// lattice.
static int find_edge_box(const int32_t* map, int p, int64_t nel, int64_t nrows, const int32_t* row_ptr,
                         const int32_t* col_idx, int32_t* elem3d, Arena& a, hipStream_t st, BoxLattice* box,
                         bool* found) {
  *found = false;
  if (nel == 0) return LOR_OK;
  ArenaScope scope(a);
  int32_t* probe;
  LOR_TAKE(probe, a, int32_t, 7);
  int rc;
  k_edgebox_probe<<<1, 64, 0, st>>>(map, p, probe);
  LOR_LAUNCHED("k_edgebox_probe");
  int32_t h[5];
  LOR_HIP(hipMemcpyAsync(h, probe, sizeof(h), hipMemcpyDeviceToHost, st));
  LOR_HIP(hipStreamSynchronize(st));
  const int64_t MX = static_cast<int64_t>(h[1]) - h[0];
  if (static_cast<int64_t>(h[3]) - h[2] != 1 || MX < p || MX % p != 0) return LOR_OK;
  const int64_t dz = static_cast<int64_t>(h[4]) - h[2];
  if (dz <= 0 || dz % (MX + 1) != 0) return LOR_OK;
  const int64_t MY = dz / (MX + 1);
  // nrows = MX (MY + 1)(MZ + 1) + (MX + 1) MY (MZ + 1) + (MX + 1)(MY + 1) MZ
  const int64_t base = MX * (MY + 1) + (MX + 1) * MY, per_z = base + (MX + 1) * (MY + 1);
  if (MY < p || MY % p != 0 || nrows < base || (nrows - base) % per_z != 0) return LOR_OK;
  const int64_t MZ = (nrows - base) / per_z;
  if (MZ < p || MZ % p != 0) return LOR_OK;
  const int64_t nx = MX / p, ny = MY / p, nz = MZ / p;
  if (nx * ny * nz != nel) return LOR_OK;
  int32_t* flag = probe + 6;
  LOR_HIP(hipMemsetAsync(flag, 0, sizeof(int32_t), st));
  k_fill_i32<<<ceil_div(nel, 256), 256, 0, st>>>(elem3d, nel, -1);
  LOR_LAUNCHED("k_fill_i32");
  const int64_t threads = nel * 3 * p * (p + 1) * (p + 1);
  const int32_t mx = static_cast<int32_t>(MX), my = static_cast<int32_t>(MY), mz = static_cast<int32_t>(MZ);
  const int32_t ne = static_cast<int32_t>(nel);
  const int inx = static_cast<int>(nx), iny = static_cast<int>(ny);
  switch (p) {
#define LOR_EDGEBOX_PLACE(PP)                                                                                    \
  case PP:                                                                                                       \
    k_edgebox_place<PP><<<ceil_div(threads, 256), 256, 0, st>>>(map, ne, mx, my, mz, inx, iny, elem3d, flag);    \
    break;
    LOR_EDGEBOX_PLACE(1)
    LOR_EDGEBOX_PLACE(2)
    LOR_EDGEBOX_PLACE(3)
    LOR_EDGEBOX_PLACE(4)
    LOR_EDGEBOX_PLACE(5)
    LOR_EDGEBOX_PLACE(6)
#undef LOR_EDGEBOX_PLACE
    default:
      LOR_FAIL(LOR_EINVAL, "p = %d outside [1, %d]", p, LOR_MAX_P);
  }
  LOR_LAUNCHED("k_edgebox_place");
  k_edgebox_rows<<<ceil_div(nrows, 256), 256, 0, st>>>(row_ptr, col_idx, MX, MY, MZ, flag);
  LOR_LAUNCHED("k_edgebox_rows");
  int32_t hflag = 0;
  if ((rc = read_err(flag, st, &hflag))) return rc;
  if (hflag != 0) return LOR_OK;
  box->LX = MX;
  box->LY = MY;
  box->LZ = MZ;
  box->nx = static_cast<int>(nx);
  box->ny = static_cast<int>(ny);
  box->nz = static_cast<int>(nz);
  *found = true;
  return LOR_OK;
}

static int order_by_color(lor_sched* s, int64_t nel, int nc, Arena& a, hipStream_t st);

static int64_t box_nnz(const BoxLattice& b) { return (3 * b.LX - 2) * (3 * b.LY - 2) * (3 * b.LZ - 2); }

// Phase 2 on a box lattice: columns, colours, one rank table per class, the
// owner-computes fields.  elem3d (in the schedule) is filled by find_box.
static int box_schedule(lor_sched* s, const RefElem& ref, const BoxLattice& b, const int32_t* map,
                        const int32_t* row_ptr, int32_t* col_idx, int32_t* d_err, Arena& a, hipStream_t st) {
  const int64_t nel = s->nel;
  int rc;
  int32_t herr = 0;
  k_box_cols<<<b.LY * b.LZ, kBoxColThreads, 0, st>>>(static_cast<int32_t>(b.LX), static_cast<int32_t>(b.LY),
                                                     static_cast<int32_t>(b.LZ), row_ptr, col_idx, d_err);
  LOR_LAUNCHED("k_box_cols");
  // colours from the parities of the axes with more than one element
  int w = 1;
  const int wx = b.nx > 1 ? w : 0;
  w <<= b.nx > 1;
  const int wy = b.ny > 1 ? w : 0;
  w <<= b.ny > 1;
  const int wz = b.nz > 1 ? w : 0;
  w <<= b.nz > 1;  // number of colours
  int32_t* d_color = dev_at<int32_t>(s, s->off_color);
  int32_t* d_class = dev_at<int32_t>(s, s->off_class);
  const int32_t* d_e3 = dev_at<int32_t>(s, s->off_elem3d);
  k_box_color_key<<<ceil_div(nel, 256), 256, 0, st>>>(d_e3, b.nx, b.ny, b.nz, wx, wy, wz, d_color, d_class);
  LOR_LAUNCHED("k_box_color_key");
  if ((rc = order_by_color(s, nel, w, a, st))) return rc;
  // classes numbered by first appearance in element order, the first element
  // of a class its representative
  std::vector<int32_t> key(static_cast<size_t>(nel)), rep;
  LOR_HIP(hipMemcpyAsync(key.data(), d_class, sizeof(int32_t) * nel, hipMemcpyDeviceToHost, st));
  LOR_HIP(hipStreamSynchronize(st));
  std::vector<int32_t> cls_of_key(kBoxKeys, -1);
  for (int64_t e = 0; e < nel; ++e) {
    int32_t& c = cls_of_key[key[e]];
    if (c < 0) {
      c = static_cast<int32_t>(rep.size());
      rep.push_back(static_cast<int32_t>(e));
    }
    key[e] = c;
  }
  const int64_t ncls = static_cast<int64_t>(rep.size());
  ArenaScope scope(a);
  int32_t* drep;
  LOR_TAKE(drep, a, int32_t, kBoxKeys);
  if ((rc = upload(key, d_class, st))) return rc;
  if ((rc = upload(rep, drep, st))) return rc;
  k_box_rank<<<ceil_div(ncls * s->tab_stride, 256), 256, 0, st>>>(
      map, s->nloc, ref.nent, s->tab_stride, dev_at<uint16_t>(s, s->off_ent_row), dev_at<int32_t>(s, s->off_st_col),
      row_ptr, col_idx, d_color, dev_at<int32_t>(s, s->off_inc_ptr), dev_at<int32_t>(s, s->off_inc_list),
      drep, ncls, dev_at<uint8_t>(s, s->off_tables), d_err);
  LOR_LAUNCHED("k_box_rank");
  k_gather_i32<<<ceil_div(nel, 256), 256, 0, st>>>(d_class, dev_at<int32_t>(s, s->off_order), nel,
                                                  dev_at<int32_t>(s, s->off_order_class));
  LOR_LAUNCHED("k_gather_i32");
  const int64_t nlines = b.LY * b.LZ;
  k_box_base<<<ceil_div(nlines, 256), 256, 0, st>>>(b.LX, nlines, dev_at<int32_t>(s, s->off_base));
  LOR_LAUNCHED("k_box_base");
  if ((rc = read_err(d_err, st, &herr))) return rc;
  if ((rc = report_err(herr))) return rc;
  s->nclass = ncls;
  s->box[0] = b.nx;
  s->box[1] = b.ny;
  s->box[2] = b.nz;
  s->owner = 1;
  return LOR_OK;
}

// Scratch bytes of order_by_color.
static size_t order_ws_bytes(int64_t nel) {
  const int64_t n = LOR_MAX_COLORS * ceil_div(nel, 64);
  return arena_bytes<int32_t>(n) + arena_bytes<int64_t>(n + 1) + arena_bytes<int32_t>(LOR_MAX_COLORS + 1) +
         scan_ws_bytes(n);
}

// Element order by colour (stable: within a colour, by element index) and the
// colour pointer, for colours 0 .. nc - 1 (every element's colour below nc).
static int order_by_color(lor_sched* s, int64_t nel, int nc, Arena& a, hipStream_t st) {
  for (int c = 0; c <= LOR_MAX_COLORS; ++c) s->color_ptr[c] = 0;
  s->ncolors = 0;
  if (nel == 0) return LOR_OK;
  if (nc < 1 || nc > LOR_MAX_COLORS) LOR_FAIL(LOR_EUNSUPPORTED, "%d colours (at most %d)", nc, LOR_MAX_COLORS);
  const int32_t* d_color = dev_at<int32_t>(s, s->off_color);
  int32_t* d_order = dev_at<int32_t>(s, s->off_order);
  const int64_t nblk = ceil_div(nel, 64), n = nc * nblk;
  ArenaScope scope(a);
  int32_t *cnt, *cptr;
  int64_t* off;
  LOR_TAKE(cnt, a, int32_t, n);
  LOR_TAKE(off, a, int64_t, n + 1);
  LOR_TAKE(cptr, a, int32_t, LOR_MAX_COLORS + 1);
  k_color_hist<<<nblk, 64, 0, st>>>(d_color, nel, nc, nblk, cnt);
  LOR_LAUNCHED("k_color_hist");
  int rc;
  if ((rc = scan_exclusive<int32_t>(cnt, n, off, a, st))) return rc;
  k_color_place<<<nblk, 64, 0, st>>>(d_color, nel, nc, nblk, off, d_order);
  LOR_LAUNCHED("k_color_place");
  k_color_ptr<<<1, 128, 0, st>>>(off, nc, nblk, cptr);
  LOR_LAUNCHED("k_color_ptr");
  int32_t h[LOR_MAX_COLORS + 1];
  LOR_HIP(hipMemcpyAsync(h, cptr, sizeof(int32_t) * (nc + 1), hipMemcpyDeviceToHost, st));
  LOR_HIP(hipStreamSynchronize(st));
  if (h[nc] != nel) LOR_FAIL(LOR_EDEVICE, "colour order incomplete");
  for (int c = 0; c <= nc; ++c) s->color_ptr[c] = h[c];
  for (int c = nc + 1; c <= LOR_MAX_COLORS; ++c) s->color_ptr[c] = h[nc];
  s->ncolors = nc;
  return LOR_OK;
}

// Jones-Plassmann rounds launched between two reads of the colouring
// progress (rounds after the last element is coloured return at once).
constexpr int kJpRoundsPerCheck = 16;

// Phase 2 on any mesh: columns from the incidence lists, greedy colouring,
// rank tables of every element, then one stored table per distinct table.
static int general_schedule(lor_sched* s, const RefElem& ref, int is_signed, const int32_t* map,
                            const int32_t* row_ptr, int32_t* col_idx, int32_t* d_err, Arena& a, hipStream_t st) {
  const int64_t nel = s->nel, nrows = s->nrows, nnzv = s->nnz;
  const int nloc = s->nloc;
  int32_t* d_color = dev_at<int32_t>(s, s->off_color);
  int32_t* d_class = dev_at<int32_t>(s, s->off_class);
  uint8_t* d_tab = dev_at<uint8_t>(s, s->off_tables);
  const int32_t* d_inc_ptr = dev_at<int32_t>(s, s->off_inc_ptr);
  const int32_t* d_inc_list = dev_at<int32_t>(s, s->off_inc_list);
  int rc;
  int32_t herr = 0;
  int ncolors = 0;
  if ((rc = row_cols<true>(map, nloc, is_signed, d_inc_ptr, d_inc_list, dev_at<int32_t>(s, s->off_st_ptr),
                           dev_at<int32_t>(s, s->off_st_col), nrows, nullptr, row_ptr, col_idx, d_err, a, st)))
    return rc;
  if ((rc = read_err(d_err, st, &herr))) return rc;
  if ((rc = report_err(herr))) return rc;

  // colouring
  int32_t *reps, *ncol;
  {
    ArenaScope scope(a);
    LOR_TAKE(reps, a, int32_t, ref.reps.size());
    LOR_TAKE(ncol, a, int32_t, 2);  // coloured elements, highest colour
    if ((rc = upload(ref.reps, reps, st))) return rc;
    k_fill_i32<<<1, 64, 0, st>>>(ncol, 2, 0);
    LOR_LAUNCHED("k_fill_i32");
    if (nel > 0) {
      k_fill_i32<<<ceil_div(nel, 256), 256, 0, st>>>(d_color, nel, -1);
      LOR_LAUNCHED("k_fill_i32");
    }
    int32_t colored[2] = {0, 0};
    for (int64_t round = 0; colored[0] < nel; round += kJpRoundsPerCheck) {
      if (round > nel) LOR_FAIL(LOR_EDEVICE, "element colouring did not converge");
      for (int r = 0; r < kJpRoundsPerCheck; ++r) {
        k_jp_round<<<ceil_div(nel, 256), 256, 0, st>>>(map, nloc, is_signed, reps, static_cast<int>(ref.reps.size()),
                                                       d_inc_ptr, d_inc_list, nel, d_color, ncol, ncol + 1, d_err);
        LOR_LAUNCHED("k_jp_round");
      }
      LOR_HIP(hipMemcpyAsync(colored, ncol, sizeof(colored), hipMemcpyDeviceToHost, st));
      if ((rc = read_err(d_err, st, &herr))) return rc;
      if ((rc = report_err(herr))) return rc;
    }
    ncolors = nel > 0 ? colored[1] + 1 : 0;
  }
  k_check_colors<<<ceil_div(nrows, 256), 256, 0, st>>>(d_inc_ptr, d_inc_list, nloc, nrows, d_color, d_err);
  LOR_LAUNCHED("k_check_colors");
  if ((rc = read_err(d_err, st, &herr))) return rc;
  if ((rc = report_err(herr))) return rc;
  if ((rc = order_by_color(s, nel, ncolors, a, st))) return rc;

  // rank tables
  {
    DevBuf mincol;
    if ((rc = mincol.alloc(sizeof(int32_t) * std::max<int64_t>(1, nnzv)))) return rc;
    const int64_t tot = nel * ref.nent;
    k_fill_i32<<<ceil_div(std::max<int64_t>(1, nnzv), 256), 256, 0, st>>>(mincol.as<int32_t>(), nnzv, INT32_MAX);
    LOR_LAUNCHED("k_fill_i32");
    if (tot > 0) {
      LOR_HIP(hipMemsetAsync(d_tab, 0, static_cast<size_t>(nel) * s->tab_stride, st));
      k_rank_pass0<<<ceil_div(tot, 256), 256, 0, st>>>(map, nloc, is_signed, ref.nent, s->tab_stride,
                                                        dev_at<uint16_t>(s, s->off_ent_row),
                                                        dev_at<int32_t>(s, s->off_st_col), row_ptr, col_idx,
                                                        d_color, tot, mincol.as<int32_t>(), d_tab, d_err);
      LOR_LAUNCHED("k_rank_pass0");
      k_rank_pass1<<<ceil_div(tot, 256), 256, 0, st>>>(map, nloc, is_signed, ref.nent, s->tab_stride,
                                                        dev_at<uint16_t>(s, s->off_ent_row), row_ptr, d_color, tot,
                                                        mincol.as<int32_t>(), d_tab);
      LOR_LAUNCHED("k_rank_pass1");
    }
    if ((rc = read_err(d_err, st, &herr))) return rc;
    if ((rc = report_err(herr))) return rc;
  }
  // element classes (identical rank tables share one stored table)
  s->nclass = nel;
  if (nel > 0) {
    const int64_t words = s->tab_stride / 4;
    uint32_t* tabw = dev_at<uint32_t>(s, s->off_tables);
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
      if ((rc = tmp.alloc(static_cast<size_t>(ncls) * s->tab_stride))) return rc;
      k_table_gather<<<ceil_div(ncls * words, 256), 256, 0, st>>>(tabw, words, ncls, drep.as<int32_t>(),
                                                                  tmp.as<uint32_t>());
      LOR_LAUNCHED("k_table_gather");
      LOR_HIP(hipMemcpyAsync(tabw, tmp.p, static_cast<size_t>(ncls) * s->tab_stride, hipMemcpyDeviceToDevice, st));
      LOR_HIP(hipStreamSynchronize(st));
      s->nclass = ncls;
    } else {
      // a hash collision (or nothing to share): every element keeps its own table
      k_iota_i32<<<ceil_div(nel, 256), 256, 0, st>>>(d_class, nel);
      LOR_LAUNCHED("k_iota_i32");
    }
    k_gather_i32<<<ceil_div(nel, 256), 256, 0, st>>>(d_class, dev_at<int32_t>(s, s->off_order), nel,
                                                    dev_at<int32_t>(s, s->off_order_class));
    LOR_LAUNCHED("k_gather_i32");
  }
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
  int rc;
  if (col_idx != nullptr) {
    if (!sched->dev) LOR_FAIL(LOR_EINVAL, "sched->dev is NULL (allocate sched->dev_bytes after phase 1)");
    if (sched->space != space || sched->p != p || sched->nel != nel || sched->nrows != nrows ||
        sched->nnz != *nnz)
      LOR_FAIL(LOR_EINVAL, "sched does not come from phase 1 of the same pattern");
    lor_sched probe = *sched;
    if (layout(&probe, ref) != sched->dev_bytes) LOR_FAIL(LOR_EINVAL, "sched->dev_bytes changed since phase 1");
  }

  // temporaries of this call, in one allocation
  const size_t box_ws = arena_bytes<int32_t>(1) + arena_bytes<int32_t>(8) + arena_bytes<int32_t>(nel);
  Arena a;
  int32_t* d_err;
  int32_t herr = 0;
  BoxLattice box;
  bool is_box = false;

  if (col_idx == nullptr) {
    // ---------------------------------------------------------------- phase 1
    if ((rc = a.alloc(box_ws))) return rc;
    LOR_TAKE(d_err, a, int32_t, 1);
    LOR_HIP(hipMemsetAsync(d_err, 0, sizeof(int32_t), st));
    int64_t total_nnz = 0;
    if (space == LOR_H1) {
      ArenaScope scope(a);
      int32_t* e3;
      LOR_TAKE(e3, a, int32_t, nel);
      if ((rc = find_box(elem_map, p, nel, nrows, e3, a, st, &box, &is_box))) return rc;
    }
    if (is_box) {
      total_nnz = box_nnz(box);
      if (total_nnz >= INT32_MAX) LOR_FAIL(LOR_EOVERFLOW, "nnz = %lld >= 2^31", (long long)total_nnz);
      k_box_row_ptr<<<ceil_div(nrows + 1, 256), 256, 0, st>>>(box.LX, box.LY, box.LZ, row_ptr);
      LOR_LAUNCHED("k_box_row_ptr");
    } else {
      Arena g;
      if ((rc = g.alloc(arena_bytes<int32_t>(nrows + 1) + arena_bytes<int32_t>(nel * nloc) +
                        arena_bytes<int32_t>(nrows) + arena_bytes<int64_t>(nrows + 1) +
                        arena_bytes<int32_t>(ref.st_ptr.size()) + arena_bytes<int32_t>(ref.st_col.size()) +
                        std::max({incidence_ws_bytes(nrows), scan_ws_bytes(nrows), ovf_ws_bytes(nrows)}))))
        return rc;
      int32_t *inc_ptr, *inc_list, *cnt, *st_ptr, *st_col;
      int64_t* ptr64;
      LOR_TAKE(inc_ptr, g, int32_t, nrows + 1);
      LOR_TAKE(inc_list, g, int32_t, nel * nloc);
      LOR_TAKE(cnt, g, int32_t, nrows);
      LOR_TAKE(ptr64, g, int64_t, nrows + 1);
      LOR_TAKE(st_ptr, g, int32_t, ref.st_ptr.size());
      LOR_TAKE(st_col, g, int32_t, ref.st_col.size());
      if ((rc = upload(ref.st_ptr, st_ptr, st))) return rc;
      if ((rc = upload(ref.st_col, st_col, st))) return rc;
      if ((rc = build_incidence(elem_map, nel, nloc, is_signed, nrows, inc_ptr, inc_list, d_err, g, st))) return rc;
      if ((rc = read_err(d_err, st, &herr))) return rc;
      if ((rc = report_err(herr))) return rc;
      if ((rc = row_cols<false>(elem_map, nloc, is_signed, inc_ptr, inc_list, st_ptr, st_col, nrows, cnt, nullptr,
                                nullptr, d_err, g, st)))
        return rc;
      if ((rc = scan_exclusive<int32_t>(cnt, nrows, ptr64, g, st))) return rc;
      LOR_HIP(hipMemcpyAsync(&total_nnz, ptr64 + nrows, sizeof(int64_t), hipMemcpyDeviceToHost, st));
      if ((rc = read_err(d_err, st, &herr))) return rc;
      if ((rc = report_err(herr))) return rc;
      if (total_nnz >= INT32_MAX) LOR_FAIL(LOR_EOVERFLOW, "nnz = %lld >= 2^31", (long long)total_nnz);
      k_i64_to_i32<<<ceil_div(nrows + 1, 256), 256, 0, st>>>(ptr64, nrows + 1, row_ptr);
      LOR_LAUNCHED("k_i64_to_i32");
      LOR_HIP(hipStreamSynchronize(st));
    }
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
    sched->owner = is_box ? 1 : 0;
    sched->box[0] = is_box ? box.nx : 0;
    sched->box[1] = is_box ? box.ny : 0;
    sched->box[2] = is_box ? box.nz : 0;
    sched->dev_bytes = layout(sched, ref);
    return LOR_OK;
  }

  // ------------------------------------------------------------------ phase 2
  if ((rc = a.alloc(box_ws + incidence_ws_bytes(nrows) + order_ws_bytes(nel) + ovf_ws_bytes(nrows) +
                    arena_bytes<int32_t>(std::max<size_t>(ref.reps.size(), kBoxKeys)) + arena_bytes<int32_t>(2))))
    return rc;
  LOR_TAKE(d_err, a, int32_t, 1);
  LOR_HIP(hipMemsetAsync(d_err, 0, sizeof(int32_t), st));
  if ((rc = upload(ref.st_ptr, dev_at<int32_t>(sched, sched->off_st_ptr), st))) return rc;
  if ((rc = upload(ref.st_col, dev_at<int32_t>(sched, sched->off_st_col), st))) return rc;
  if ((rc = upload(ref.ent_row, dev_at<uint16_t>(sched, sched->off_ent_row), st))) return rc;
  if ((rc = upload(ref.recipe64, dev_at<uint64_t>(sched, sched->off_recipe), st))) return rc;
  LOR_HIP(hipMemsetAsync(dev_at<uint8_t>(sched, sched->off_zero), 0, 256, st));
  if ((rc = build_incidence(elem_map, nel, nloc, is_signed, nrows, dev_at<int32_t>(sched, sched->off_inc_ptr),
                            dev_at<int32_t>(sched, sched->off_inc_list), d_err, a, st)))
    return rc;
  const bool box1 = sched->owner == 1 && space == LOR_H1;  // (a 2D box lattice is found in phase 2)
  sched->owner = 0;
  sched->box[0] = sched->box[1] = sched->box[2] = 0;
  sched->max_row_nnz = 0;
  if (space == LOR_H1 &&
      (rc = find_box(elem_map, p, nel, nrows, dev_at<int32_t>(sched, sched->off_elem3d), a, st, &box, &is_box)))
    return rc;
  if (is_box != box1) LOR_FAIL(LOR_EINVAL, "elem_map is not the one phase 1 saw");
  if (is_box)
    rc = box_schedule(sched, ref, box, elem_map, row_ptr, col_idx, d_err, a, st);
  else
    rc = general_schedule(sched, ref, is_signed, elem_map, row_ptr, col_idx, d_err, a, st);
  if (rc) return rc;
  // a quadrilateral mesh keeps its general schedule (the coloured kernel) and
  // gains the owner-computes one if it is a 2D box lattice; an H(div) mesh
  // if its face map is a face lattice
  if (space == LOR_ND) {
    if ((rc = find_edge_box(elem_map, p, nel, nrows, row_ptr, col_idx, dev_at<int32_t>(sched, sched->off_elem3d), a,
                            st, &box, &is_box)))
      return rc;
    if (is_box) {
      sched->box[0] = box.nx;
      sched->box[1] = box.ny;
      sched->box[2] = box.nz;
      sched->owner = 1;
    }
  }
  if (space == LOR_RT) {
    if ((rc = find_face_box(elem_map, p, nel, nrows, row_ptr, dev_at<int32_t>(sched, sched->off_elem3d), a, st, &box,
                            &is_box)))
      return rc;
    if (is_box) {
      sched->box[0] = box.nx;
      sched->box[1] = box.ny;
      sched->box[2] = box.nz;
      sched->owner = 1;
    }
  }
  if (space == LOR_H1_2D) {
    if ((rc = find_box_2d(elem_map, p, nel, nrows, row_ptr, dev_at<int32_t>(sched, sched->off_elem3d), a, st, &box,
                          &is_box)))
      return rc;
    if (is_box) {
      sched->box[0] = box.nx;
      sched->box[1] = box.ny;
      sched->box[2] = 1;
      sched->owner = 1;
    }
  }
  LOR_HIP(hipStreamSynchronize(st));
  return LOR_OK;
}
