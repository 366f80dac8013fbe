// Shared host/device helpers of the LOR assembly library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>
#include <type_traits>

#include "../../include/lor.h"

namespace lor {

// ----------------------------------------------------------------- errors

// Thread-local message of the last failing call (lor_last_error).
void set_error(const char* fmt, ...);
void clear_error();

struct Status {
  int code = LOR_OK;
  bool ok() const { return code == LOR_OK; }
};

#define LOR_FAIL(CODE, ...)        \
  do {                             \
    ::lor::set_error(__VA_ARGS__); \
    return (CODE);                 \
  } while (0)

#define LOR_HIP(CALL)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (CALL);                                                            \
    if (e_ != hipSuccess) {                                                            \
      ::lor::set_error("%s failed: %s (%s:%d)", #CALL, hipGetErrorString(e_), __FILE__, \
                       __LINE__);                                                      \
      return LOR_EDEVICE;                                                              \
    }                                                                                  \
  } while (0)

// Launch-error check right after a <<<>>> launch.
#define LOR_LAUNCHED(NAME)                                                             \
  do {                                                                                 \
    hipError_t e_ = hipGetLastError();                                                 \
    if (e_ != hipSuccess) {                                                            \
      ::lor::set_error("launch of %s failed: %s", NAME, hipGetErrorString(e_));         \
      return LOR_EDEVICE;                                                              \
    }                                                                                  \
  } while (0)

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ------------------------------------------------------ reference element

// Local dof counts per element.
inline int nloc_h1(int p) { return (p + 1) * (p + 1) * (p + 1); }
inline int nloc_nd(int p) { return 3 * p * (p + 1) * (p + 1); }
inline int nloc_rt(int p) { return 3 * p * p * (p + 1); }

// Per-element table entry: bits 0..6 = position of the entry inside its CSR
// row, bit 7 = this element is the first (lowest colour) contributor.
constexpr uint8_t kFirstBit = 0x80u;
constexpr uint8_t kRankMask = 0x7fu;

// Workgroup barrier for LDS traffic only.  __syncthreads() is also a
// workgroup-scope memory fence, which makes every wave wait for all of its
// outstanding global loads and stores first; the assembly kernels keep global
// prefetches and stores in flight across phases, so they synchronise LDS with
// this barrier instead (wait for the wave's LDS operations, then s_barrier).
__device__ __forceinline__ void lds_barrier() {
  __asm__ volatile("" ::: "memory");
  // s_waitcnt lgkmcnt(0) with vmcnt and expcnt left at their maxima
  __builtin_amdgcn_s_waitcnt(0xC07F);
  __builtin_amdgcn_s_barrier();
  __asm__ volatile("" ::: "memory");
}

// Box lattices (H1 meshes whose vertex at lattice point (X, Y, Z) has id
// X + LX (Y + LY Z)): the row of a point holds its in-box 3 x 3 x 3
// neighbours in (dz, dy, dx) order.  box_count: neighbours of a point along
// one axis of L >= 2 points; box_prefix: their sum over the points before X
// (X in [0, L]); box_row_start: the CSR row start of point (X, Y, Z).
__host__ __device__ __forceinline__ int box_count(int64_t X, int64_t L) { return 1 + (X > 0) + (X < L - 1); }
__host__ __device__ __forceinline__ int64_t box_prefix(int64_t X, int64_t L) {
  return X == 0 ? 0 : 3 * X - 1 - (X == L ? 1 : 0);
}
__host__ __device__ __forceinline__ int64_t box_row_start(int64_t X, int64_t Y, int64_t Z, int64_t LX, int64_t LY,
                                                          int64_t LZ) {
  const int64_t SX = 3 * LX - 2, SY = 3 * LY - 2;
  const int64_t cz = box_count(Z, LZ), cyz = box_count(Y, LY) * cz;
  return box_prefix(Z, LZ) * SY * SX + cz * box_prefix(Y, LY) * SX + cyz * box_prefix(X, LX);
}

template <typename T>
inline T* dev_at(const lor_sched* s, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(s->dev) + off);
}

}  // namespace lor
