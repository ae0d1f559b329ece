// Token permute (histogram + prefix scan + stable scatter + row gather) and
// the weighted combine, for gfx950.
//
// Slots are ordered by expert, then by token.  A token block of 256 owns a
// contiguous run of every expert's slots: its base is the expert's offset
// plus the counts of all earlier blocks, and a token's rank inside its
// block comes from per-wavefront 64-bit occupancy masks.
#include <mutex>

#include "common.h"
#include "internal.h"

namespace {

// Indices arriving from the caller are clamped so that malformed routing
// tables give unspecified values, never an out-of-bounds access.
__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

constexpr int TB = 256;  // tokens per block of the count / scatter kernels

__global__ __launch_bounds__(TB) void dispatch_count(const int32_t* __restrict__ idx, int T,
                                                     int E, int k, int32_t* __restrict__ cnt) {
  __shared__ int hist[MOE_MAX_E];
  const int tid = threadIdx.x;
  for (int e = tid; e < E; e += TB) hist[e] = 0;
  __syncthreads();
  const int t = blockIdx.x * TB + tid;
  if (t < T)
    for (int j = 0; j < k; ++j) atomicAdd(&hist[clampi(idx[(size_t)t * k + j], 0, E - 1)], 1);
  __syncthreads();
  for (int e = tid; e < E; e += TB) cnt[(size_t)blockIdx.x * E + e] = hist[e];
}

// One block of 1024 threads.  Thread (e, p) owns expert e and the p-th of
// P = 1024 / E contiguous runs of token blocks: it sums its run, the runs of
// an expert are scanned in order, the expert totals are scanned into
// offsets, and each thread finally rewrites its run's counts as absolute
// bases (offset of e + counts of all earlier blocks).
__global__ __launch_bounds__(1024) void dispatch_scan(int32_t* __restrict__ cnt_base, int nb,
                                                      int E, int32_t* __restrict__ offsets) {
  __shared__ int runsum[1024];
  __shared__ int tot[2][MOE_MAX_E];
  const int tid = threadIdx.x;
  const int P = 1024 / E;
  const int e = tid % E, p = tid / E;
  const bool own = p < P;
  const int chunk = (nb + P - 1) / P;
  const int b0 = own ? min(nb, p * chunk) : nb, b1 = own ? min(nb, b0 + chunk) : nb;
  int run = 0;
  for (int b = b0; b < b1; b += 8) {
    int c[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) c[i] = b + i < b1 ? cnt_base[(size_t)(b + i) * E + e] : 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) run += c[i];
  }
  runsum[tid] = run;
  __syncthreads();
  int before = 0, total = 0;
  if (own)
    for (int q = 0; q < P; ++q) {
      const int v = runsum[q * E + e];
      if (q < p) before += v;
      total += v;
    }
  if (own && p == 0) tot[0][e] = total;
  __syncthreads();
  // inclusive scan of the expert totals (Hillis-Steele over E <= 1024)
  int cur = 0;
  for (int off = 1; off < E; off <<= 1) {
    if (tid < E) tot[cur ^ 1][tid] = tot[cur][tid] + (tid >= off ? tot[cur][tid - off] : 0);
    cur ^= 1;
    __syncthreads();
  }
  if (own) {
    const int incl = tot[cur][e];
    const int off_e = incl - total;
    if (p == 0) offsets[e] = off_e;
    if (p == 0 && e == E - 1) offsets[E] = incl;
    int acc = off_e + before;
    for (int b = b0; b < b1; ++b) {
      const int c = cnt_base[(size_t)b * E + e];
      cnt_base[(size_t)b * E + e] = acc;
      acc += c;
    }
  }
}

__global__ __launch_bounds__(TB) void dispatch_scatter(const int32_t* __restrict__ idx, int T,
                                                       int E, int k,
                                                       const int32_t* __restrict__ base,
                                                       int32_t* __restrict__ row_map,
                                                       int32_t* __restrict__ inv_map) {
  __shared__ unsigned long long occ[TB / 64][MOE_MAX_E];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int i = tid; i < (TB / 64) * E; i += TB) occ[i / E][i % E] = 0ull;
  __syncthreads();
  const int t = blockIdx.x * TB + tid;
  if (t < T)
    for (int j = 0; j < k; ++j)
      atomicOr(&occ[wv][clampi(idx[(size_t)t * k + j], 0, E - 1)], 1ull << lane);
  __syncthreads();
  if (t < T) {
    const unsigned long long lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    for (int j = 0; j < k; ++j) {
      const int e = clampi(idx[(size_t)t * k + j], 0, E - 1);
      int rank = __popcll(occ[wv][e] & lt);
      for (int w = 0; w < wv; ++w) rank += __popcll(occ[w][e]);
      const int slot = base[(size_t)blockIdx.x * E + e] + rank;
      row_map[slot] = t;
      inv_map[(size_t)t * k + j] = slot;
    }
  }
}

// One wavefront per token: read the row once (16-byte vectors), write it to
// each of the token's k slots.
__global__ __launch_bounds__(256) void dispatch_gather(const u32x4* __restrict__ X, int T,
                                                       int row_vec, int k,
                                                       const int32_t* __restrict__ inv_map,
                                                       u32x4* __restrict__ Xp) {
  const int lane = threadIdx.x & 63;
  const int t = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (t >= T) return;
  int slots[MOE_MAX_K];
#pragma unroll
  for (int j = 0; j < MOE_MAX_K; ++j)
    slots[j] = j < k ? clampi(inv_map[(size_t)t * k + j], 0, T * k - 1) : 0;
  for (int c = lane; c < row_vec; c += 64) {
    const u32x4 v = X[(size_t)t * row_vec + c];
#pragma unroll
    for (int j = 0; j < MOE_MAX_K; ++j)
      if (j < k) Xp[(size_t)slots[j] * row_vec + c] = v;
  }
}

// FP8 variant of the gather: each token row is quantised once per 1 x 128
// block (amax over the block, inv = 448 / amax, codes of x * inv, scale =
// amax / 448; an all-zero block has scale 1 and zero codes) and the codes
// and scales are written to all k slots of the token.  One wavefront per
// token; 16 lanes of 8 elements cover one block.
template <typename TA>
__global__ __launch_bounds__(256) void dispatch_gather_fp8(const TA* __restrict__ X, int T, int d,
                                                           int k,
                                                           const int32_t* __restrict__ inv_map,
                                                           fp8_t* __restrict__ Xq,
                                                           float* __restrict__ Xs) {
  const int lane = threadIdx.x & 63;
  const int t = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (t >= T) return;
  int slots[MOE_MAX_K];
#pragma unroll
  for (int j = 0; j < MOE_MAX_K; ++j)
    slots[j] = j < k ? clampi(inv_map[(size_t)t * k + j], 0, T * k - 1) : 0;
  const int nblk = d / 128;
  for (int c0 = 0; c0 < d; c0 += 512) {
    const int col = c0 + lane * 8;
    const bool act = col < d;
    float v[8];
    if (act) {
      const TA* src = X + (size_t)t * d + col;
#pragma unroll
      for (int i = 0; i < 8; ++i) v[i] = ActIO<TA>::ld(src, i);
    } else {
#pragma unroll
      for (int i = 0; i < 8; ++i) v[i] = 0.0f;
    }
    float am = 0.0f;
#pragma unroll
    for (int i = 0; i < 8; ++i) am = fmaxf(am, fabsf(v[i]));
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) am = fmaxf(am, __shfl_xor(am, o, 64));
    const bool nz = am > 0.0f;
    const float inv = nz ? 448.0f / am : 1.0f;
    const float scale = nz ? am / 448.0f : 1.0f;
    u32x2 q;
    q[0] = q[1] = 0u;
    if (nz) {
      q[0] = fp8_encode4(v[0] * inv, v[1] * inv, v[2] * inv, v[3] * inv);
      q[1] = fp8_encode4(v[4] * inv, v[5] * inv, v[6] * inv, v[7] * inv);
    }
    if (act) {
#pragma unroll
      for (int j = 0; j < MOE_MAX_K; ++j) {
        if (j < k) {
          *(u32x2*)(Xq + (size_t)slots[j] * d + col) = q;
          if ((lane & 15) == 0) Xs[(size_t)slots[j] * nblk + col / 128] = scale;
        }
      }
    }
  }
}

// out[t] = sum_j w[t,j] * Y[inv_map[t,j]], FP32 in j order; one wavefront
// per token, 8 elements per lane per step.  KT > 0: k == KT known at
// compile time, so the k row loads carry no branches and are all in flight
// together (with a run-time k each sits behind its own guard and waits for
// the previous one); KT == 0: any k.
template <typename TA, int KT>
__global__ __launch_bounds__(256) void combine_kernel(const TA* __restrict__ Y, int T, int d,
                                                      int k_rt, const int32_t* __restrict__ inv_map,
                                                      const float* __restrict__ w,
                                                      TA* __restrict__ out) {
  const int k = KT > 0 ? KT : k_rt;
  const int lane = threadIdx.x & 63;
  const int t = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (t >= T) return;
  int slots[MOE_MAX_K];
  float ws[MOE_MAX_K];
#pragma unroll
  for (int j = 0; j < MOE_MAX_K; ++j) {
    slots[j] = j < k ? clampi(inv_map[(size_t)t * k + j], 0, T * k - 1) : 0;
    ws[j] = j < k ? w[(size_t)t * k + j] : 0.0f;
  }
  for (int c0 = lane * 8; c0 < d; c0 += 64 * 8) {
    float acc[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) acc[i] = 0.0f;
#pragma unroll
    for (int j = 0; j < MOE_MAX_K; ++j) {
      if (j < k) {
        const TA* yr = Y + (size_t)slots[j] * d + c0;
#pragma unroll
        for (int i = 0; i < 8; ++i) acc[i] = acc[i] + ws[j] * ActIO<TA>::ld(yr, i);
      }
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) ActIO<TA>::st(out, (size_t)t * d + c0 + i, acc[i]);
  }
}

struct DispWs {
  int32_t* cnt;
};

DispWs carve_dispatch(const moe_cfg& c, void* base, size_t* total) {
  WsCarve wc{(char*)base, 0};
  DispWs r;
  const size_t nb = ((size_t)c.T + TB - 1) / TB;
  r.cnt = wc.take<int32_t>((nb > 0 ? nb : 1) * (size_t)c.E);
  if (total) *total = align_up(wc.off, 256);
  return r;
}

}  // namespace

size_t dispatch_ws_bytes(const moe_cfg& c) {
  size_t total = 0;
  carve_dispatch(c, nullptr, &total);
  return total;
}

extern "C" moe_status moe_dispatch(const moe_cfg* cfg, const void* X, const int32_t* topk_idx,
                                   int32_t* offsets, int32_t* row_map, int32_t* inv_map,
                                   void* X_perm, float* X_perm_scale, void* ws, size_t ws_bytes,
                                   void* stream) {
  moe_status stc = check_cfg_shape(cfg);
  if (stc != MOE_OK) return stc;
  const moe_cfg& c = *cfg;
  const bool fp8 = c.w == MOE_FP8E4M3;
  if (!offsets) return MOE_EINVAL;
  if (c.T > 0 && (!topk_idx || !row_map || !inv_map)) return MOE_EINVAL;
  if (c.T > 0 && X_perm && !X) return MOE_EINVAL;
  if (fp8 && X_perm && c.d % 128 != 0) return MOE_EUNSUPPORTED;
  if (fp8 && c.T > 0 && X_perm && !X_perm_scale) return MOE_EINVAL;
  if (!aligned(X_perm_scale, 4)) return MOE_EINVAL;
  if (!aligned(X, 16) || !aligned(X_perm, 16) || !aligned(topk_idx, 4) || !aligned(offsets, 4) ||
      !aligned(row_map, 4) || !aligned(inv_map, 4))
    return MOE_EINVAL;
  if (ws_bytes < dispatch_ws_bytes(c) || !ws) return MOE_EWORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  DispWs w = carve_dispatch(c, ws, nullptr);
  const int nb = (c.T + TB - 1) / TB;
  PROF_BEGIN("dispatch", st);
  if (c.T > 0) {
    hipLaunchKernelGGL(dispatch_count, dim3(nb), dim3(TB), 0, st, topk_idx, c.T, c.E, c.k, w.cnt);
  }
  hipLaunchKernelGGL(dispatch_scan, dim3(1), dim3(1024), 0, st, w.cnt, nb, c.E, offsets);
  if (c.T > 0) {
    hipLaunchKernelGGL(dispatch_scatter, dim3(nb), dim3(TB), 0, st, topk_idx, c.T, c.E, c.k, w.cnt,
                       row_map, inv_map);
    if (!fp8) {
      // X_perm NULL: maps only (the first expert product gathers X itself)
      if (X_perm) {
        const int row_vec = c.d * act_bytes(c.act) / 16;
        hipLaunchKernelGGL(dispatch_gather, dim3((c.T + 3) / 4), dim3(256), 0, st,
                           (const u32x4*)X, c.T, row_vec, c.k, inv_map, (u32x4*)X_perm);
      }
    } else if (!X_perm) {
      // maps only (moe_expert_ffn_gather_fp8 reads the per-token codes)
    } else if (c.act == MOE_BF16) {
      hipLaunchKernelGGL(HIP_KERNEL_NAME(dispatch_gather_fp8<bf16_t>), dim3((c.T + 3) / 4),
                         dim3(256), 0, st, (const bf16_t*)X, c.T, c.d, c.k, inv_map,
                         (fp8_t*)X_perm, X_perm_scale);
    } else {
      hipLaunchKernelGGL(HIP_KERNEL_NAME(dispatch_gather_fp8<float>), dim3((c.T + 3) / 4),
                         dim3(256), 0, st, (const float*)X, c.T, c.d, c.k, inv_map,
                         (fp8_t*)X_perm, X_perm_scale);
    }
  }
  PROF_END("dispatch", st);
  MOE_LAUNCH_CHECK();
  return MOE_OK;
}

// ---------------------------------------------- dispatch without allocation
// moe_dispatch_noalloc: the per-block expert counts live in a fixed device
// array instead of a caller workspace.  In host code the array's name is only
// a host-side stand-in, so the device address is looked up once per device
// (with that device current) and every launch takes that address.
namespace {

constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(4) << 20;  // 1 Mi counts
constexpr int NOALLOC_MAX_DEVICES = 64;

static __device__ __align__(256) int32_t scratch[NOALLOC_SCRATCH_BYTES / sizeof(int32_t)];

std::mutex g_scratch_mu;
int32_t* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

// Device address of ``scratch`` on the current device (looked up on the
// first call per device, kept for the life of the process).
moe_status noalloc_scratch(int32_t** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= NOALLOC_MAX_DEVICES) return MOE_EHIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return MOE_EHIP;
    g_scratch_ptr[dev] = (int32_t*)p;
  }
  *out = g_scratch_ptr[dev];
  return MOE_OK;
}

}  // namespace

extern "C" moe_status moe_dispatch_noalloc(const moe_cfg* cfg, const void* X,
                                           const int32_t* topk_idx, int32_t* offsets,
                                           int32_t* row_map, int32_t* inv_map, void* X_perm,
                                           float* X_perm_scale, void* stream) {
  moe_status stc = check_cfg_shape(cfg);
  if (stc != MOE_OK) return stc;
  const size_t need = dispatch_ws_bytes(*cfg);
  if (need > NOALLOC_SCRATCH_BYTES) return MOE_EUNSUPPORTED;
  hipStream_t st = (hipStream_t)stream;
  // the stream must belong to the current device, whose copy of the array
  // is the one looked up
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess) return MOE_EHIP;
  if (st) {
    hipDevice_t sdev = -1;
    if (hipStreamGetDevice(st, &sdev) != hipSuccess) return MOE_EHIP;
    if ((int)sdev != cur) return MOE_EINVAL;
  }
  int32_t* ptr = nullptr;
  stc = noalloc_scratch(&ptr);
  if (stc != MOE_OK) return stc;
  // dispatch_count writes every count the scan reads, so nothing is cleared
  return moe_dispatch(cfg, X, topk_idx, offsets, row_map, inv_map, X_perm, X_perm_scale, ptr,
                      NOALLOC_SCRATCH_BYTES, stream);
}

extern "C" moe_status moe_combine(const moe_cfg* cfg, const void* Y, const int32_t* inv_map,
                                  const float* topk_w, void* out, void* stream) {
  moe_status stc = check_cfg_shape(cfg);
  if (stc != MOE_OK) return stc;
  const moe_cfg& c = *cfg;
  if (c.T == 0) return MOE_OK;
  if (!Y || !inv_map || !topk_w || !out) return MOE_EINVAL;
  if (!aligned(Y, 16) || !aligned(out, 16) || !aligned(inv_map, 4) || !aligned(topk_w, 4))
    return MOE_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  dim3 g((c.T + 3) / 4);
  PROF_BEGIN("combine", st);
  if (c.act == MOE_F32) {
    if (c.k == 8)
      hipLaunchKernelGGL(HIP_KERNEL_NAME(combine_kernel<float, 8>), g, dim3(256), 0, st,
                         (const float*)Y, c.T, c.d, c.k, inv_map, topk_w, (float*)out);
    else
      hipLaunchKernelGGL(HIP_KERNEL_NAME(combine_kernel<float, 0>), g, dim3(256), 0, st,
                         (const float*)Y, c.T, c.d, c.k, inv_map, topk_w, (float*)out);
  } else {
    if (c.k == 8)
      hipLaunchKernelGGL(HIP_KERNEL_NAME(combine_kernel<bf16_t, 8>), g, dim3(256), 0, st,
                         (const bf16_t*)Y, c.T, c.d, c.k, inv_map, topk_w, (bf16_t*)out);
    else
      hipLaunchKernelGGL(HIP_KERNEL_NAME(combine_kernel<bf16_t, 0>), g, dim3(256), 0, st,
                         (const bf16_t*)Y, c.T, c.d, c.k, inv_map, topk_w, (bf16_t*)out);
  }
  PROF_END("combine", st);
  MOE_LAUNCH_CHECK();
  return MOE_OK;
}
