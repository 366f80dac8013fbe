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

template <typename T>
inline T* dev_at(const lor_sched* s, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(s->dev) + off);
}

}  // namespace lor
