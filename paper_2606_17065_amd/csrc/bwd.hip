// Backward of the layer with the routing held fixed, for gfx950 (the
// expert-GEMM part lives in gemm.hip).  No floating-point atomics: every
// reduction has one owner thread and a fixed order, so repeated calls are
// bit-identical.
//
//   combine:   dY[slot(t,j)] = w_tj * dOut_t,  dw_tj = <dOut_t, Y[slot(t,j)]>
//   dispatch:  dX_t = sum_j dX_perm[slot(t,j)]            (j order)
//   gate:      ds_tj = w_tj (dw_tj - sum_i w_ti dw_ti)     (softmax over the
//              chosen experts; no gradient into prices or the selection)
//   router:    dX_t += sum_j ds_tj W_r[e_j];  dW_r[e] = sum over the slots of
//              e (token order) of ds * X_t;  db_r[e] = sum of the same ds.
#include "common.h"
#include "internal.h"

namespace {

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Eight consecutive values as FP32 (16-byte aligned loads), and stored.
__device__ __forceinline__ void ld8(const float* p, float (&v)[8]) {
  const f32x4 a = *(const f32x4*)p, b = *(const f32x4*)(p + 4);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    v[i] = a[i];
    v[4 + i] = b[i];
  }
}
__device__ __forceinline__ void ld8(const bf16_t* p, float (&v)[8]) {
  const bf16x8 a = *(const bf16x8*)p;
#pragma unroll
  for (int i = 0; i < 8; ++i) v[i] = (float)a[i];
}
__device__ __forceinline__ void st8(float* p, const float (&v)[8]) {
  *(f32x4*)p = (f32x4){v[0], v[1], v[2], v[3]};
  *(f32x4*)(p + 4) = (f32x4){v[4], v[5], v[6], v[7]};
}
__device__ __forceinline__ void st8(bf16_t* p, const float (&v)[8]) {
  bf16x8 a;
#pragma unroll
  for (int i = 0; i < 8; ++i) a[i] = (bf16_t)v[i];
  *(bf16x8*)p = a;
}

// One wavefront per token: dw by a fixed-order dot product (lane partials in
// ascending column order, then a fixed butterfly), dY rows scaled by w.
// KT > 0: k == KT known at compile time (the k slot rows are loaded with no
// branch between them, all in flight together); KT == 0: any k.  The same
// operations in the same order either way.
template <typename TA, int KT>
__global__ __launch_bounds__(256) void combine_bwd_kernel(const TA* __restrict__ dOut,
                                                          const TA* __restrict__ Y, int T, int d,
                                                          int k_rt,
                                                          const int32_t* __restrict__ inv_map,
                                                          const float* __restrict__ w,
                                                          TA* __restrict__ dY,
                                                          float* __restrict__ dw) {
  const int k = KT > 0 ? KT : k_rt;
  // one wavefront per token, 8 consecutive elements per lane and step: the
  // dOut segment is read once for all k slots; each slot's dot product
  // runs over the elements in the same order as a slot-by-slot loop
  const int lane = threadIdx.x & 63;
  const int t = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (t >= T) return;
  const int N = T * k;
  int slots[MOE_MAX_K];
  float ws_[MOE_MAX_K], part[MOE_MAX_K];
#pragma unroll
  for (int j = 0; j < MOE_MAX_K; ++j) {
    slots[j] = j < k ? clampi(inv_map[(size_t)t * k + j], 0, N - 1) : 0;
    ws_[j] = j < k ? w[(size_t)t * k + j] : 0.0f;
    part[j] = 0.0f;
  }
  for (int c0 = lane * 8; c0 < d; c0 += 64 * 8) {
    float g[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) g[i] = ActIO<TA>::ld(dOut, (size_t)t * d + c0 + i);
    if (KT > 0) {
      // all k segments requested before the first dY store
      float yv[KT > 0 ? KT : 1][8];
#pragma unroll
      for (int j = 0; j < KT; ++j) ld8(Y + (size_t)slots[j] * d + c0, yv[j]);
#pragma unroll
      for (int j = 0; j < KT; ++j) {
        TA* dyr = dY + (size_t)slots[j] * d + c0;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          part[j] = __builtin_fmaf(g[i], yv[j][i], part[j]);
          ActIO<TA>::st(dyr, i, ws_[j] * g[i]);
        }
      }
      continue;
    }
#pragma unroll
    for (int j = 0; j < MOE_MAX_K; ++j) {
      if (j < k) {
        const TA* yr = Y + (size_t)slots[j] * d + c0;
        TA* dyr = dY + (size_t)slots[j] * d + c0;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          part[j] = __builtin_fmaf(g[i], ActIO<TA>::ld(yr, i), part[j]);
          ActIO<TA>::st(dyr, i, ws_[j] * g[i]);
        }
      }
    }
  }
#pragma unroll
  for (int j = 0; j < MOE_MAX_K; ++j) {
    if (j < k) {
      float p = part[j];
      for (int off = 32; off >= 1; off >>= 1) p += __shfl_xor(p, off, 64);
      if (lane == 0) dw[(size_t)t * k + j] = p;
    }
  }
}

// dX_t = sum_j dX_perm[slot(t,j)] (+ sum_j ds_tj W_r[e_j] when ROUTER) in
// FP32.  With ROUTER the second sum is the router backward into the tokens;
// ds is formed here from w and dw (and written to ds_out).  Without ROUTER
// idx, w, dw, Wr and ds_out are not touched (they may be null).  One
// wavefront per token.  KT as in combine_bwd_kernel.
template <typename TA, bool ROUTER, typename TO, int KT>
__global__ __launch_bounds__(256) void dispatch_bwd_kernel(
    const TA* __restrict__ dXp, int T, int d, int k_rt, int E,
    const int32_t* __restrict__ inv_map, const int32_t* __restrict__ idx,
    const float* __restrict__ w, const float* __restrict__ dw, const float* __restrict__ Wr,
    TO* __restrict__ dX, float* __restrict__ ds_out) {
  const int k = KT > 0 ? KT : k_rt;
  const int lane = threadIdx.x & 63;
  const int t = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (t >= T) return;
  const int N = T * k;
  int slots[MOE_MAX_K], ex[MOE_MAX_K];
  float ds[MOE_MAX_K];
#pragma unroll
  for (int j = 0; j < MOE_MAX_K; ++j) {
    slots[j] = j < k ? clampi(inv_map[(size_t)t * k + j], 0, N - 1) : 0;
    ex[j] = 0;
    ds[j] = 0.0f;
  }
  if (ROUTER) {
    float sw = 0.0f;
#pragma unroll
    for (int j = 0; j < MOE_MAX_K; ++j)
      if (j < k) sw = sw + w[(size_t)t * k + j] * dw[(size_t)t * k + j];
#pragma unroll
    for (int j = 0; j < MOE_MAX_K; ++j) {
      if (j < k) {
        ex[j] = clampi(idx[(size_t)t * k + j], 0, E - 1);
        ds[j] = w[(size_t)t * k + j] * (dw[(size_t)t * k + j] - sw);
      }
    }
    if (lane < k) {
#pragma unroll
      for (int j = 0; j < MOE_MAX_K; ++j)
        if (j == lane) ds_out[(size_t)t * k + j] = ds[j];
    }
  }
  // eight columns per lane and step (d % 8 == 0; 16-byte loads and stores)
  for (int c0 = lane * 8; c0 < d; c0 += 64 * 8) {
    float acc[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) acc[i] = 0.0f;
    if (KT > 0) {
      // every slot segment (and router row) requested before the sums
      float v[KT > 0 ? KT : 1][8], r[ROUTER && KT > 0 ? KT : 1][8];
#pragma unroll
      for (int j = 0; j < KT; ++j) ld8(dXp + (size_t)slots[j] * d + c0, v[j]);
      if (ROUTER) {
#pragma unroll
        for (int j = 0; j < KT; ++j) ld8(Wr + (size_t)ex[j] * d + c0, r[j]);
      }
      // keep the scheduler from sinking the loads back between the sums
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int j = 0; j < KT; ++j)
#pragma unroll
        for (int i = 0; i < 8; ++i) acc[i] = acc[i] + v[j][i];
      if (ROUTER) {
#pragma unroll
        for (int j = 0; j < KT; ++j)
#pragma unroll
          for (int i = 0; i < 8; ++i) acc[i] = __builtin_fmaf(ds[j], r[j][i], acc[i]);
      }
      st8(dX + (size_t)t * d + c0, acc);
      continue;
    }
#pragma unroll
    for (int j = 0; j < MOE_MAX_K; ++j) {
      if (j < k) {
        float v[8];
        ld8(dXp + (size_t)slots[j] * d + c0, v);
#pragma unroll
        for (int i = 0; i < 8; ++i) acc[i] = acc[i] + v[i];
      }
    }
    if (ROUTER) {
#pragma unroll
      for (int j = 0; j < MOE_MAX_K; ++j) {
        if (j < k) {
          float v[8];
          ld8(Wr + (size_t)ex[j] * d + c0, v);
#pragma unroll
          for (int i = 0; i < 8; ++i) acc[i] = __builtin_fmaf(ds[j], v[i], acc[i]);
        }
      }
    }
    st8(dX + (size_t)t * d + c0, acc);
  }
}

// dW_r[e, c] = sum over the slots r of expert e of ds(slot) * X[row_map[r], c]
// and db_r[e] = sum of ds(slot), in two passes.  Pass 1: block (expert, 256
// columns, q) sums the chunks q, q + nq, q + 2 nq, ... of RW_CH slots of
// the expert (slot order inside a chunk, chunks in increasing order); the
// chunk's ds values and token rows are staged in LDS once, so the X loads
// of a chunk are independent.  Pass 2 adds the nq partial sums of each
// (expert, column) in q order.  Both orders are fixed: the result is
// deterministic.
constexpr int RW_CH = 64;

int rw_nq(const moe_cfg& c) {
  // at most 32 partial sums per (expert, column), and at most 64 MB of them
  const size_t per = (size_t)c.E * (size_t)c.d * sizeof(float);
  const size_t cap = ((size_t)64 << 20) / (per > 0 ? per : 1);
  return (int)(cap < 1 ? 1 : (cap > 32 ? 32 : cap));
}

template <typename TA>
__global__ __launch_bounds__(256) void router_wgrad_partial(
    const TA* __restrict__ X, int T, int d, int k, int E, const int32_t* __restrict__ row_map,
    const int32_t* __restrict__ offsets, const int32_t* __restrict__ slot_src,
    const float* __restrict__ ds_tk, int nq, float* __restrict__ part, float* __restrict__ partb) {
  __shared__ float sg[RW_CH];
  __shared__ int st[RW_CH];
  const int e = blockIdx.x, q = blockIdx.z, tid = threadIdx.x;
  const int c = blockIdx.y * 256 + tid;
  const int N = T * k;
  const int r0 = clampi(offsets[e], 0, N), r1 = clampi(offsets[e + 1], r0, N);
  float acc = 0.0f, accb = 0.0f;
  for (int lo = r0 + q * RW_CH; lo < r1; lo += nq * RW_CH) {  // uniform over the block
    const int n = min(RW_CH, r1 - lo);
    __syncthreads();  // the previous chunk's LDS reads are done
    if (tid < RW_CH) {
      float g = 0.0f;
      int t = 0;
      if (tid < n) {
        g = ds_tk[clampi(slot_src[lo + tid], 0, N - 1)];
        t = clampi(row_map[lo + tid], 0, T - 1);
      }
      sg[tid] = g;
      st[tid] = t;
    }
    __syncthreads();
    if (c < d) {
#pragma unroll 8
      for (int i = 0; i < n; ++i)
        acc = __builtin_fmaf(sg[i], ActIO<TA>::ld(X, (size_t)st[i] * d + c), acc);
    }
    if (tid == 0)
      for (int i = 0; i < n; ++i) accb = accb + sg[i];
  }
  if (c < d) part[((size_t)q * E + e) * d + c] = acc;
  if (blockIdx.y == 0 && tid == 0) partb[(size_t)q * E + e] = accb;
}

__global__ __launch_bounds__(256) void router_wgrad_reduce(const float* __restrict__ part,
                                                           const float* __restrict__ partb,
                                                           int E, int d, int nq,
                                                           float* __restrict__ dWr,
                                                           float* __restrict__ dbr) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  const size_t Ed = (size_t)E * d;
  if (i < Ed) {
    float acc = 0.0f;
    for (int q = 0; q < nq; ++q) acc = acc + part[(size_t)q * Ed + i];
    dWr[i] = acc;
  }
  if (i < (size_t)E) {
    float acc = 0.0f;
    for (int q = 0; q < nq; ++q) acc = acc + partb[(size_t)q * E + i];
    dbr[i] = acc;
  }
}

// slot_src[inv_map[t,j]] = t*k + j: the (token, choice) behind each slot.
__global__ __launch_bounds__(256) void slot_source(const int32_t* __restrict__ inv_map, int N,
                                                   int32_t* __restrict__ slot_src) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < N) slot_src[clampi(inv_map[i], 0, N - 1)] = i;
}

struct RouteBwdWs {
  int32_t* slot_src;
  float* ds;
  float* part;   // [nq][E][d] partial sums of dW_r
  float* partb;  // [nq][E] partial sums of db_r
};

RouteBwdWs carve_route_bwd(const moe_cfg& c, void* base, size_t* total) {
  WsCarve wc{(char*)base, 0};
  RouteBwdWs r;
  const size_t N = (size_t)c.T * c.k;
  const size_t nq = (size_t)rw_nq(c);
  r.slot_src = wc.take<int32_t>(N > 0 ? N : 1);
  r.ds = wc.take<float>(N > 0 ? N : 1);
  r.part = wc.take<float>(nq * c.E * c.d);
  r.partb = wc.take<float>(nq * c.E);
  if (total) *total = align_up(wc.off, 256);
  return r;
}

}  // namespace

size_t route_bwd_ws_bytes(const moe_cfg& c) {
  size_t total = 0;
  carve_route_bwd(c, nullptr, &total);
  return total;
}

extern "C" moe_status moe_combine_bwd(const moe_cfg* cfg, const void* dOut, const void* Y,
                                      const int32_t* inv_map, const float* topk_w, void* dY,
                                      float* dtopk_w, void* stream) {
  moe_status stc = check_cfg_shape(cfg);
  if (stc != MOE_OK) return stc;
  const moe_cfg& c = *cfg;
  if (c.T == 0) return MOE_OK;
  if (!dOut || !Y || !inv_map || !topk_w || !dY || !dtopk_w) return MOE_EINVAL;
  if (!aligned(dOut, 16) || !aligned(Y, 16) || !aligned(dY, 16) || !aligned(inv_map, 4) ||
      !aligned(topk_w, 4) || !aligned(dtopk_w, 4))
    return MOE_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  PROF_BEGIN("combine_bwd", st);
#define CBWD(TA, KT)                                                                           \
  hipLaunchKernelGGL(HIP_KERNEL_NAME(combine_bwd_kernel<TA, KT>), dim3((c.T + 3) / 4),          \
                     dim3(256), 0, st, (const TA*)dOut, (const TA*)Y, c.T, c.d, c.k, inv_map,    \
                     topk_w, (TA*)dY, dtopk_w);
  if (c.act == MOE_F32) {
    if (c.k == 8) CBWD(float, 8) else CBWD(float, 0)
  } else {
    if (c.k == 8) CBWD(bf16_t, 8) else CBWD(bf16_t, 0)
  }
#undef CBWD
  PROF_END("combine_bwd", st);
  MOE_LAUNCH_CHECK();
  return MOE_OK;
}

extern "C" moe_status moe_dispatch_bwd(const moe_cfg* cfg, const void* dX_perm,
                                       const int32_t* inv_map, float* dX, void* stream) {
  moe_status stc = check_cfg_shape(cfg);
  if (stc != MOE_OK) return stc;
  const moe_cfg& c = *cfg;
  if (c.T == 0) return MOE_OK;
  if (!dX_perm || !inv_map || !dX) return MOE_EINVAL;
  if (!aligned(dX_perm, 16) || !aligned(dX, 16) || !aligned(inv_map, 4)) return MOE_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  PROF_BEGIN("dispatch_bwd", st);
#define DBWD0(TA, KT)                                                                          \
  hipLaunchKernelGGL(HIP_KERNEL_NAME(dispatch_bwd_kernel<TA, false, float, KT>),               \
                     dim3((c.T + 3) / 4), dim3(256), 0, st, (const TA*)dX_perm, c.T, c.d, c.k,  \
                     c.E, inv_map, nullptr, nullptr, nullptr, nullptr, dX, nullptr);
  if (c.act == MOE_F32) {
    if (c.k == 8) DBWD0(float, 8) else DBWD0(float, 0)
  } else {
    if (c.k == 8) DBWD0(bf16_t, 8) else DBWD0(bf16_t, 0)
  }
#undef DBWD0
  PROF_END("dispatch_bwd", st);
  MOE_LAUNCH_CHECK();
  return MOE_OK;
}

extern "C" moe_status moe_route_bwd(const moe_cfg* cfg, const void* X, const float* Wr,
                                    const int32_t* topk_idx, const float* topk_w,
                                    const float* dtopk_w, const int32_t* row_map,
                                    const int32_t* offsets, const int32_t* inv_map,
                                    const void* dX_perm, void* dX, int dx_dtype, float* dWr,
                                    float* dbr, void* ws, size_t ws_bytes, void* stream) {
  moe_status stc = check_cfg_shape(cfg);
  if (stc != MOE_OK) return stc;
  const moe_cfg& c = *cfg;
  if (dx_dtype != MOE_F32 && dx_dtype != MOE_BF16) return MOE_EINVAL;
  if (!dWr || !dbr || !offsets) return MOE_EINVAL;
  if (c.T > 0 && (!X || !Wr || !topk_idx || !topk_w || !dtopk_w || !row_map || !inv_map ||
                  !dX_perm || !dX))
    return MOE_EINVAL;
  if (!aligned(X, 16) || !aligned(dX_perm, 16) || !aligned(dX, 16) || !aligned(dWr, 4) ||
      !aligned(dbr, 4) || !aligned(Wr, 16))
    return MOE_EINVAL;
  if (ws_bytes < route_bwd_ws_bytes(c) || !ws) return MOE_EWORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  RouteBwdWs w = carve_route_bwd(c, ws, nullptr);
  const int N = c.T * c.k;
  PROF_BEGIN("route_bwd", st);
  if (c.T > 0) {
    hipLaunchKernelGGL(slot_source, dim3((N + 255) / 256), dim3(256), 0, st, inv_map, N,
                       w.slot_src);
#define DBWD(TA, TO)                                                                          \
  {                                                                                           \
    if (c.k == 8)                                                                             \
      hipLaunchKernelGGL(HIP_KERNEL_NAME(dispatch_bwd_kernel<TA, true, TO, 8>),               \
                         dim3((c.T + 3) / 4), dim3(256), 0, st, (const TA*)dX_perm, c.T, c.d,  \
                         c.k, c.E, inv_map, topk_idx, topk_w, dtopk_w, Wr, (TO*)dX, w.ds);    \
    else                                                                                      \
      hipLaunchKernelGGL(HIP_KERNEL_NAME(dispatch_bwd_kernel<TA, true, TO, 0>),               \
                         dim3((c.T + 3) / 4), dim3(256), 0, st, (const TA*)dX_perm, c.T, c.d,  \
                         c.k, c.E, inv_map, topk_idx, topk_w, dtopk_w, Wr, (TO*)dX, w.ds);    \
  }
    if (c.act == MOE_F32) {
      if (dx_dtype == MOE_F32) DBWD(float, float) else DBWD(float, bf16_t)
    } else {
      if (dx_dtype == MOE_F32) DBWD(bf16_t, float) else DBWD(bf16_t, bf16_t)
    }
#undef DBWD
  }
  const int nq = rw_nq(c);
  dim3 g(c.E, (c.d + 255) / 256, nq);
  if (c.act == MOE_F32)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(router_wgrad_partial<float>), g, dim3(256), 0, st,
                       (const float*)X, c.T, c.d, c.k, c.E, row_map, offsets, w.slot_src, w.ds, nq,
                       w.part, w.partb);
  else
    hipLaunchKernelGGL(HIP_KERNEL_NAME(router_wgrad_partial<bf16_t>), g, dim3(256), 0, st,
                       (const bf16_t*)X, c.T, c.d, c.k, c.E, row_map, offsets, w.slot_src, w.ds,
                       nq, w.part, w.partb);
  const size_t Ed = (size_t)c.E * c.d;
  hipLaunchKernelGGL(router_wgrad_reduce, dim3((unsigned)((Ed + 255) / 256)), dim3(256), 0, st,
                     w.part, w.partb, c.E, c.d, nq, dWr, dbr);
  PROF_END("route_bwd", st);
  MOE_LAUNCH_CHECK();
  return MOE_OK;
}
