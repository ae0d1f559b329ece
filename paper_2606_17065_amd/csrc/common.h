// Internal helpers shared by the HIP translation units of libmoe.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/moe.h"

typedef __bf16 bf16_t;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

#define MOE_MAX_E 1024
#define MOE_MAX_K 16

// Route workspace state words (int32), shared by the route kernels.
enum {
  ST_DONE = 0,        // price loop finished
  ST_CONVERGED = 1,
  ST_ITERS = 2,
  ST_OVERFLOW = 3,
  ST_STATUS = 4,
  ST_ROUNDS = 5,
  ST_SIGMA = 6,       // float bits
  ST_EPS = 7,         // float bits
  ST_NEED_REPAIR = 8,
  ST_REPAIRED = 9,
  ST_LEN = 16
};

__device__ __forceinline__ uint32_t f32_key(float x) {
  uint32_t u = __float_as_uint(x);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ float key_f32(uint32_t k) {
  uint32_t u = (k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k;
  return __uint_as_float(u);
}

__device__ __forceinline__ float bf2f(bf16_t x) { return (float)x; }
__device__ __forceinline__ bf16_t f2bf(float x) { return (bf16_t)x; }

template <typename T> struct ActIO;
template <> struct ActIO<float> {
  __device__ static __forceinline__ float ld(const float* p, size_t i) { return p[i]; }
  __device__ static __forceinline__ void st(float* p, size_t i, float v) { p[i] = v; }
};
template <> struct ActIO<bf16_t> {
  __device__ static __forceinline__ float ld(const bf16_t* p, size_t i) { return (float)p[i]; }
  __device__ static __forceinline__ void st(bf16_t* p, size_t i, float v) { p[i] = (bf16_t)v; }
};

static inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Bump allocator over the caller's workspace.
struct WsCarve {
  char* base;
  size_t off;
  template <typename T> T* take(size_t count) {
    off = align_up(off, 256);
    T* p = reinterpret_cast<T*>(base ? base + off : nullptr);
    off += count * sizeof(T);
    return p;
  }
};

#define MOE_LAUNCH_CHECK()                                 \
  do {                                                     \
    if (hipGetLastError() != hipSuccess) return MOE_EHIP;  \
  } while (0)
