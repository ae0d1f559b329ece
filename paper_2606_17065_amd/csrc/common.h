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
  ST_SKIP_WEIGHTS = 10,  // the final routing is already in place (judged routing kept)
  ST_ITERS_PREV = 11,    // updates of the finished runs (epsilon-scaled restarts)
  ST_STAGE_STOP = 12,    // no further epsilon-scaled restart runs
  ST_EPS0 = 13,          // float bits: the first run's increment
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

// OCP FP8 e4m3 code of an FP32 value: round to nearest, ties to the even
// mantissa, saturate to +-448 (no infinities; the sign of zero is kept).
// Subnormals (|v| < 2^-6) have the quantum 2^-9; normals 2^(e-3).
__device__ __forceinline__ uint32_t fp8_encode(float v) {
  const uint32_t u = __float_as_uint(v);
  const uint32_t sign = (u >> 24) & 0x80u;
  const float a = __uint_as_float(u & 0x7FFFFFFFu);
  uint32_t code;
  if (!(a < 448.0f)) {
    code = 0x7Eu;  // 448 and everything that rounds or saturates to it
  } else if (a < 0.015625f) {
    code = (uint32_t)rintf(a * 512.0f);  // 0..8; 8 is the code of 2^-6
  } else {
    const int e = (int)((__float_as_uint(a) >> 23) & 0xFFu) - 127;  // -6..8
    const float p = __uint_as_float((uint32_t)(130 - e) << 23);     // 2^(3-e)
    uint32_t m = (uint32_t)rintf(a * p);                              // 8..16
    int ee = e;
    if (m == 16u) {
      m = 8u;
      ee += 1;
    }
    code = ((uint32_t)(ee + 7) << 3) | (m - 8u);
    code = code > 0x7Eu ? 0x7Eu : code;
  }
  return code | sign;
}

// Four fp8_encode codes packed in a word (value i in byte i) by gfx950's
// conversion instruction, which rounds exactly as fp8_encode for every FP32
// value of magnitude at most 464 (measured over all of them on the
// MI355X); larger magnitudes, infinities and NaN get fp8_encode's
// saturation to +-448 with the sign kept.
__device__ __forceinline__ uint32_t fp8_encode4(float a, float b, float c, float d) {
  int w = __builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false);
  w = __builtin_amdgcn_cvt_pk_fp8_f32(c, d, w, true);
  uint32_t r = (uint32_t)w;
  const float v[4] = {a, b, c, d};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const uint32_t sat = ((__float_as_uint(v[i]) >> 24) & 0x80u) | 0x7Eu;
    r = fabsf(v[i]) <= 464.0f ? r : ((r & ~(0xFFu << (8 * i))) | (sat << (8 * i)));
  }
  return r;
}

typedef uint8_t fp8_t;
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

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
