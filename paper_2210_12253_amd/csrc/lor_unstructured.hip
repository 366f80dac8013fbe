// The comparator of Section 4's assembly results: a generic, fully
// unstructured assembly that ignores the macro-element structure.  The LOR
// mesh is first made explicit (every subelement becomes an element with its
// own 8 vertex ids: lor_refine_map), then one group of 8 lanes per element
// (one lane per element dof) builds the element's dense 8x8 matrix and adds
// its row straight into the global CSR matrix: binary search for each column
// position, hardware FP64 atomic add.  The summation order therefore varies
// from run to run (results agree to rounding, not bitwise).
#include <algorithm>

#include "lor_common.hpp"
#include "lor_h1_math.hpp"

namespace lor {

constexpr int kUnsThreads = 256;
constexpr int kUnsElems = kUnsThreads / 8;  // elements per workgroup

// sub_map[(e p^3 + s) * 8 + v] = vertex (i+a, j+b, k+c) of element e, with
// s = i + p(j + p k) and v = a + 2b + 4c.
__global__ __launch_bounds__(kUnsThreads) void k_refine_map(int p, int64_t nel, const int32_t* __restrict__ elem_dofs,
                                                            int32_t* __restrict__ sub_map) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int nsub = p * p * p, q = p + 1;
  if (t >= nel * nsub * 8) return;
  const int v = static_cast<int>(t & 7);
  const int64_t es = t >> 3;
  const int64_t e = es / nsub;
  const int s = static_cast<int>(es - e * nsub);
  const int i = s % p, j = (s / p) % p, k = s / (p * p);
  const int a = v & 1, b = (v >> 1) & 1, c = v >> 2;
  sub_map[t] = elem_dofs[e * q * q * q + (i + a) + q * ((j + b) + q * (k + c))];
}

__global__ __launch_bounds__(kUnsThreads) void k_zero_f64(double* __restrict__ v, int64_t n) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) v[i] = 0.0;
}

__global__ __launch_bounds__(kUnsThreads) void k_unstructured_h1(
    int64_t nsub, int64_t ndofs, const int32_t* __restrict__ sub_map, const double* __restrict__ coords,
    const double* __restrict__ kappa, double beta, const int32_t* __restrict__ row_ptr,
    const int32_t* __restrict__ col_idx, int64_t nnz, double* __restrict__ values, int32_t* __restrict__ diag) {
  __shared__ double sX[kUnsElems][8][3];
  __shared__ int32_t sG[kUnsElems][8];
  __shared__ H1Factors<double> sF[kUnsElems];
  const int le = threadIdx.x >> 3, i = threadIdx.x & 7;
  const int64_t e = static_cast<int64_t>(blockIdx.x) * kUnsElems + le;
  const bool live = e < nsub;
  if (live) {
    const int32_t g = sub_map[e * 8 + i];
    const bool ok = g >= 0 && g < ndofs;
    sG[le][i] = ok ? g : -1;
#pragma unroll
    for (int d = 0; d < 3; ++d) sX[le][i][d] = ok ? coords[3 * static_cast<int64_t>(g) + d] : 0.0;
  }
  __syncthreads();
  bool valid = live;
#pragma unroll
  for (int v = 0; v < 8; ++v) valid = valid && sG[le][v] >= 0;
  if (live && !valid && i == 0 && diag) atomicAdd(&diag[0], 1);  // vertex id outside [0, ndofs): skipped
  if (valid && i == 0) {  // the element's factor tables, shared with its 8 lanes
    double X[8][3];
#pragma unroll
    for (int v = 0; v < 8; ++v)
#pragma unroll
      for (int d = 0; d < 3; ++d) X[v][d] = sX[le][v][d];
    double ex[2][2][3], ey[2][2][3], ez[2][2][3];
    h1_edges<double>(X, ex, ey, ez);
    H1Factors<double> F;
    const bool ok = h1_factors<double>(ex, ey, ez, kappa[e], beta, F);
    sF[le] = F;
    if (!ok && diag) atomicAdd(&diag[1], 1);
  }
  __syncthreads();
  if (!valid) return;
  const int32_t gi = sG[le][i];
  const int64_t rb = min(max(static_cast<int64_t>(row_ptr[gi]), int64_t(0)), nnz);
  const int64_t re = min(max(static_cast<int64_t>(row_ptr[gi + 1]), rb), nnz);
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const double a = h1_entry<double>(sF[le], i, j);
    const int32_t gj = sG[le][j];
    int64_t lo = rb, hi = re;  // first position in row gi with column >= gj
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (col_idx[mid] < gj)
        lo = mid + 1;
      else
        hi = mid;
    }
    if (lo < re && col_idx[lo] == gj)
      unsafeAtomicAdd(values + lo, a);
    else if (diag)
      atomicAdd(&diag[0], 1);
  }
}

}  // namespace lor

using namespace lor;

extern "C" int lor_refine_map(int p, int64_t nel, const int32_t* elem_dofs, int32_t* sub_map, void* stream) {
  clear_error();
  if (p < 1 || p > LOR_MAX_P) LOR_FAIL(LOR_EINVAL, "p = %d outside [1, %d]", p, LOR_MAX_P);
  if (nel < 0) LOR_FAIL(LOR_EINVAL, "nel < 0");
  const int64_t total = nel * p * p * p * 8;
  if (total >= (int64_t(1) << 31)) LOR_FAIL(LOR_EOVERFLOW, "nel * p^3 * 8 >= 2^31");
  if (nel == 0) return LOR_OK;
  if (!elem_dofs || !sub_map) LOR_FAIL(LOR_EINVAL, "elem_dofs or sub_map is NULL");
  k_refine_map<<<static_cast<unsigned>(ceil_div(total, kUnsThreads)), kUnsThreads, 0, as_stream(stream)>>>(
      p, nel, elem_dofs, sub_map);
  LOR_LAUNCHED("k_refine_map");
  return LOR_OK;
}

extern "C" int lor_assemble_h1_unstructured(int64_t nsub, int64_t ndofs, int64_t nnz, const int32_t* sub_map,
                                            const double* coords, const double* kappa, double beta,
                                            const int32_t* row_ptr, const int32_t* col_idx, double* values,
                                            int32_t* diag, void* stream) {
  clear_error();
  if (nsub < 0 || ndofs < 1 || nnz < 0) LOR_FAIL(LOR_EINVAL, "nsub < 0, ndofs < 1 or nnz < 0");
  if (nsub * 8 >= (int64_t(1) << 31) || nnz >= (int64_t(1) << 31)) LOR_FAIL(LOR_EOVERFLOW, "nsub * 8 or nnz >= 2^31");
  if (nnz > 0 && (!row_ptr || !col_idx || !values)) LOR_FAIL(LOR_EINVAL, "row_ptr, col_idx or values is NULL");
  if (nsub > 0 && (!sub_map || !coords || !kappa)) LOR_FAIL(LOR_EINVAL, "sub_map, coords or kappa is NULL");
  hipStream_t st = as_stream(stream);
  if (nnz > 0) {
    const int64_t blocks = std::min<int64_t>(ceil_div(nnz, kUnsThreads), 8192);
    k_zero_f64<<<static_cast<unsigned>(blocks), kUnsThreads, 0, st>>>(values, nnz);
    LOR_LAUNCHED("k_zero_f64");
  }
  if (nsub == 0 || nnz == 0) return LOR_OK;
  k_unstructured_h1<<<static_cast<unsigned>(ceil_div(nsub, kUnsElems)), kUnsThreads, 0, st>>>(
      nsub, ndofs, sub_map, coords, kappa, beta, row_ptr, col_idx, nnz, values, diag);
  LOR_LAUNCHED("k_unstructured_h1");
  return LOR_OK;
}
