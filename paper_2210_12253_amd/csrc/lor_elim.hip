// Elimination of essential boundary conditions from the assembled CSR matrix
// (Section 3, Step S1.2, step A4), on one device.
//
// The essential set is first written as a byte marker over the degrees of
// freedom (the paper's marker array).  Then a group of 16 lanes per essential
// dof i walks row i (LOR rows have at most 33 entries): every entry becomes 0 except the diagonal (1, kept, or 0), and
// for every column c != i that is not itself essential, the transposed entry
// (c, i) is located by binary search in row c (columns are sorted) and set to
// 0.  The LOR pattern is structurally symmetric, so column i is reached
// through row i and the elimination is threaded over the essential dofs only,
// as the paper does for the rows and columns of the diagonal block.  Entries
// of a row that is itself essential are left to that row's own lane group, so
// every entry is written by one group (two only if the essential list repeats
// a dof, and then with the same value): the result is deterministic.
#include <algorithm>

#include "lor_common.hpp"

namespace lor {

constexpr int kElimThreads = 256;
constexpr int kElimGroup = 16;  // lanes per essential row

__global__ __launch_bounds__(kElimThreads) void k_elim_clear(uint8_t* __restrict__ marker, int64_t n) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) marker[i] = 0;
}

__global__ __launch_bounds__(kElimThreads) void k_elim_mark(const int32_t* __restrict__ ess, int64_t ness,
                                                            int64_t nrows, uint8_t* __restrict__ marker,
                                                            int32_t* __restrict__ diag) {
  const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= ness) return;
  const int32_t i = ess[k];
  if (i < 0 || i >= nrows) {
    if (diag) atomicAdd(&diag[0], 1);
    return;
  }
  marker[i] = 1;
}

template <typename T>
__global__ __launch_bounds__(kElimThreads) void k_elim_rows(
    const int32_t* __restrict__ ess, int64_t ness, int64_t nrows, int64_t nnz, int batch,
    const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col_idx, const uint8_t* __restrict__ marker,
    T* __restrict__ values, int policy, int32_t* __restrict__ diag) {
  const int64_t k = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) / kElimGroup;
  const int lane = static_cast<int>(threadIdx.x) % kElimGroup;
  if (k >= ness) return;
  const int32_t i = ess[k];
  if (i < 0 || i >= nrows) return;  // counted by k_elim_mark
  // clamp the row bounds to [0, nnz] so that a malformed row pointer cannot
  // send a lane outside the arrays
  const int64_t beg = min(max(static_cast<int64_t>(row_ptr[i]), int64_t(0)), nnz);
  const int64_t end = min(max(static_cast<int64_t>(row_ptr[i + 1]), beg), nnz);
  const T dval = policy == LOR_DIAG_ONE ? T(1) : T(0);
  for (int64_t pos = beg + lane; pos < end; pos += kElimGroup) {
    const int32_t c = col_idx[pos];
    if (c == i) {
      if (policy != LOR_DIAG_KEEP)
        for (int b = 0; b < batch; ++b) values[b * nnz + pos] = dval;
      continue;
    }
    for (int b = 0; b < batch; ++b) values[b * nnz + pos] = T(0);
    if (c < 0 || c >= nrows) {
      if (diag) atomicAdd(&diag[1], 1);
      continue;
    }
    if (marker[c]) continue;  // row c is essential: its own lane group clears (c, i)
    const int64_t cb = min(max(static_cast<int64_t>(row_ptr[c]), int64_t(0)), nnz);
    const int64_t ce = min(max(static_cast<int64_t>(row_ptr[c + 1]), cb), nnz);
    int64_t lo = cb, hi = ce;  // first position in row c with column >= i
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (col_idx[mid] < i)
        lo = mid + 1;
      else
        hi = mid;
    }
    if (lo < ce && col_idx[lo] == i) {
      for (int b = 0; b < batch; ++b) values[b * nnz + lo] = T(0);
    } else if (diag) {
      atomicAdd(&diag[1], 1);  // (c, i) absent: the pattern is not structurally symmetric
    }
  }
}

}  // namespace lor

using namespace lor;

extern "C" int lor_eliminate_bc(int64_t nrows, int64_t nnz, int batch, const int32_t* row_ptr,
                                const int32_t* col_idx, void* values, int dtype, int64_t ness,
                                const int32_t* ess_dofs, uint8_t* marker, int diag_policy, int32_t* diag,
                                void* stream) {
  clear_error();
  if (nrows < 0 || nnz < 0 || ness < 0) LOR_FAIL(LOR_EINVAL, "nrows, nnz and ness must be >= 0");
  if (nrows >= (int64_t(1) << 31) || nnz >= (int64_t(1) << 31))
    LOR_FAIL(LOR_EOVERFLOW, "nrows or nnz does not fit int32 indices");
  if (ness >= (int64_t(1) << 31)) LOR_FAIL(LOR_EOVERFLOW, "ness >= 2^31");
  if (batch < 1 || batch > 65535) LOR_FAIL(LOR_EINVAL, "batch outside [1, 65535]");
  if (dtype != LOR_F64 && dtype != LOR_F32) LOR_FAIL(LOR_EINVAL, "dtype must be LOR_F64 or LOR_F32");
  if (diag_policy != LOR_DIAG_ONE && diag_policy != LOR_DIAG_KEEP && diag_policy != LOR_DIAG_ZERO)
    LOR_FAIL(LOR_EINVAL, "diag_policy must be LOR_DIAG_ONE, LOR_DIAG_KEEP or LOR_DIAG_ZERO");
  if (nrows > 0 && (!row_ptr || !marker)) LOR_FAIL(LOR_EINVAL, "row_ptr or marker is NULL");
  if (ness > 0 && !ess_dofs) LOR_FAIL(LOR_EINVAL, "ess_dofs is NULL");
  if (ness > 0 && nnz > 0 && (!col_idx || !values)) LOR_FAIL(LOR_EINVAL, "col_idx or values is NULL");
  if (nrows == 0) return LOR_OK;
  hipStream_t st = as_stream(stream);
  {
    const int64_t blocks = std::min<int64_t>(ceil_div(nrows, kElimThreads), 4096);
    k_elim_clear<<<static_cast<unsigned>(blocks), kElimThreads, 0, st>>>(marker, nrows);
    LOR_LAUNCHED("k_elim_clear");
  }
  if (ness == 0) return LOR_OK;
  k_elim_mark<<<static_cast<unsigned>(ceil_div(ness, kElimThreads)), kElimThreads, 0, st>>>(ess_dofs, ness, nrows,
                                                                                            marker, diag);
  LOR_LAUNCHED("k_elim_mark");
  if (nnz == 0) return LOR_OK;
  const unsigned blocks = static_cast<unsigned>(ceil_div(ness * kElimGroup, kElimThreads));
  if (dtype == LOR_F64)
    k_elim_rows<double><<<blocks, kElimThreads, 0, st>>>(ess_dofs, ness, nrows, nnz, batch, row_ptr, col_idx, marker,
                                                         static_cast<double*>(values), diag_policy, diag);
  else
    k_elim_rows<float><<<blocks, kElimThreads, 0, st>>>(ess_dofs, ness, nrows, nnz, batch, row_ptr, col_idx, marker,
                                                        static_cast<float*>(values), diag_policy, diag);
  LOR_LAUNCHED("k_elim_rows");
  return LOR_OK;
}
