// Router logits, capacity prices (ascending clearing price) and
// capacity-aware top-k for gfx950.
//
// This translation unit is compiled with -ffp-contract=off: every FP32 and
// FP64 operation of the price loop is rounded on its own, so the sequence
// of operations below is the definition the FP32 replica reproduces.
//
// Data flow of moe_route (one stream, no host synchronisation):
//   route_init        state words, load buffers, starting prices
//   router_logits     s[T,E] = X W_r^T + b_r, and its transpose sT[E,T]
//   score_partials    per-256-token FP64 partial sums of s and s^2
//   score_sigma       sigma_s, eps, non-finite check
//   (acp_rank, acp_select) x (max_iters + 1)   price loop, early-exit flags
//   capacity_repair   only if the final ranking still overloads an expert
//   route_finalize    info[] from the state words
#include <math.h>

#include "common.h"
#include "internal.h"

namespace {

constexpr int SIG_BLOCK = 256;   // token block of the fixed-order reduction
constexpr int SEL_THREADS = 1024;
constexpr int REP_THREADS = 1024;

// ------------------------------------------------------------------ init

__global__ void route_init(int32_t* state, int E, float* price, int mode, float gamma) {
  int tid = threadIdx.x;
  if (tid < ST_LEN) state[tid] = 0;
  for (int e = tid; e < E; e += blockDim.x) {
    if (mode == MOE_PRICE_NONE || mode == MOE_PRICE_ACP || mode == MOE_PRICE_SUBGRAD)
      price[e] = 0.0f;
    else if (mode == MOE_PRICE_WARM) price[e] = gamma * price[e];
  }
}

// ------------------------------------------------- caller-given logits
// sT[E,T] from s[T,E] through a 64x64 LDS tile (moe_route_logits).

__global__ __launch_bounds__(256) void logits_transpose(const float* __restrict__ s, int T, int E,
                                                        float* __restrict__ sT) {
  __shared__ float tile[64][65];
  const int t0 = blockIdx.x * 64, e0 = blockIdx.y * 64, tid = threadIdx.x;
  for (int i = tid; i < 64 * 64; i += 256) {
    const int tl = i >> 6, el = i & 63;
    const int t = t0 + tl, e = e0 + el;
    tile[tl][el] = (t < T && e < E) ? s[(size_t)t * E + e] : 0.0f;
  }
  __syncthreads();
  for (int i = tid; i < 64 * 64; i += 256) {
    const int el = i >> 6, tl = i & 63;
    const int t = t0 + tl, e = e0 + el;
    if (t < T && e < E) sT[(size_t)e * T + t] = tile[tl][el];
  }
}

// ------------------------------------------------------------ router GEMM
// 64 tokens x 64 experts per block, 256 threads, 4x4 outputs per thread,
// FP32 fused multiply-add accumulation over d in chunks of 32.

template <typename TX>
__global__ __launch_bounds__(256) void router_logits(const TX* __restrict__ X,
                                                     const float* __restrict__ Wr,
                                                     const float* __restrict__ br,
                                                     float* __restrict__ s, float* __restrict__ sT,
                                                     int T, int d, int E) {
  __shared__ float Xs[32][64 + 1];
  __shared__ float Ws[32][64 + 1];
  __shared__ float Ts[64][64 + 1];
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  const int t0 = blockIdx.x * 64, e0 = blockIdx.y * 64;
  float acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0f;
  for (int k0 = 0; k0 < d; k0 += 32) {
    for (int i = tid; i < 64 * 32; i += 256) {
      int r = i >> 5, c = i & 31;
      int t = t0 + r, kk = k0 + c;
      Xs[c][r] = (t < T && kk < d) ? ActIO<TX>::ld(X, (size_t)t * d + kk) : 0.0f;
      int e = e0 + r;
      Ws[c][r] = (e < E && kk < d) ? Wr[(size_t)e * d + kk] : 0.0f;
    }
    __syncthreads();
#pragma unroll 8
    for (int kk = 0; kk < 32; ++kk) {
      float a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = Xs[kk][ty * 4 + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Ws[kk][tx * 4 + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_fmaf(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    int t = t0 + ty * 4 + i;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      int e = e0 + tx * 4 + j;
      float v = acc[i][j] + ((e < E) ? br[e] : 0.0f);
      if (t < T && e < E) s[(size_t)t * E + e] = v;
      Ts[tx * 4 + j][ty * 4 + i] = v;
    }
  }
  __syncthreads();
  for (int i = tid; i < 64 * 64; i += 256) {
    int el = i >> 6, tl = i & 63;
    int e = e0 + el, t = t0 + tl;
    if (e < E && t < T) sT[(size_t)e * T + t] = Ts[el][tl];
  }
}

// -------------------------------------------- router GEMM, BF16 tokens
// W_r is split into three BF16 planes hi, mid, lo (each the round-to-
// nearest-even of what the previous planes leave over), so that
// X W_r^T = X hi^T + X mid^T + X lo^T with exact BF16 x BF16 products
// accumulated in FP32 by v_mfma_f32_32x32x16_bf16.

__global__ __launch_bounds__(256) void router_split(const float* __restrict__ Wr, int n,
                                                    bf16_t* __restrict__ W3) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float x = Wr[i];
  const bf16_t h = (bf16_t)x;
  const float r1 = x - (float)h;
  const bf16_t m = (bf16_t)r1;
  const float r2 = r1 - (float)m;
  W3[i] = h;
  W3[n + i] = m;
  W3[2 * n + i] = (bf16_t)r2;
}

// Block: 128 tokens (32 per wavefront) x 64 experts, K step KS (32, or 128
// when d % 128 == 0: four times fewer steps, each with four times the
// MFMAs behind the next step's loads).  The three weight planes of the
// block's experts go through LDS; each wavefront reads its own token
// fragments straight from HBM.  Every product is exact in FP32 and the
// accumulation runs plane by plane within each K step.
// TPB tokens per block: 128 (each wavefront 32 tokens x 64 experts) or 64
// (each wavefront 32 tokens x 32 experts, twice the blocks for batches too
// short to fill the chip with 128-token blocks).
template <int KS, int TPB>
__global__ __launch_bounds__(256) void router_logits_mfma(const bf16_t* __restrict__ X,
                                                          const bf16_t* __restrict__ W3,
                                                          const float* __restrict__ br,
                                                          float* __restrict__ s,
                                                          float* __restrict__ sT, int T, int d,
                                                          int E) {
  constexpr int LDK = KS + 8;
  constexpr int CPR = KS / 8;               // 16-byte chunks per weight row and step
  constexpr int WCH = 3 * 64 * CPR / 256;   // chunks per thread
  constexpr int KSUB = KS / 16;             // MFMA K steps per K step
  constexpr int NJ = TPB == 128 ? 2 : 1;    // 32-expert tiles per wavefront
  __shared__ __attribute__((aligned(16))) bf16_t Ws[3 * 64 * LDK];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int t0 = blockIdx.x * TPB + (TPB == 128 ? wv * 32 : (wv & 1) * 32);
  const int jb = TPB == 128 ? 0 : (wv >> 1);
  const int e0 = blockIdx.y * 64;
  const size_t plane = (size_t)E * d;
  const int fr = lane & 31, fk = (lane >> 5) * 8;
  const int trow = t0 + fr;
  const bf16_t* xr = X + (size_t)min(trow, T - 1) * d + fk;
  const bool tvalid = trow < T;
  int wrow[WCH], wcol[WCH], wpl[WCH];
  bool wok[WCH];
#pragma unroll
  for (int r = 0; r < WCH; ++r) {
    const int c = tid + 256 * r;
    wpl[r] = c / (64 * CPR);
    wrow[r] = (c % (64 * CPR)) / CPR;
    wcol[r] = (c % CPR) * 8;
    wok[r] = e0 + wrow[r] < E;
  }
  u32x4 wreg[WCH];
  bf16x8 xa[KSUB];
#define RLOAD(k0)                                                                         \
  _Pragma("unroll") for (int r = 0; r < WCH; ++r) wreg[r] =                               \
      wok[r] ? *(const u32x4*)(W3 + wpl[r] * plane + (size_t)(e0 + wrow[r]) * d + (k0) +  \
                               wcol[r])                                                   \
             : u32x4{0u, 0u, 0u, 0u};                                                     \
  _Pragma("unroll") for (int u = 0; u < KSUB; ++u) xa[u] = *(const bf16x8*)(xr + (k0) + 16 * u);
  f32x16 acc[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j)
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[j][q] = 0.0f;
  RLOAD(0);
  for (int k0 = 0; k0 < d; k0 += KS) {
#pragma unroll
    for (int r = 0; r < WCH; ++r) *(u32x4*)(Ws + (wpl[r] * 64 + wrow[r]) * LDK + wcol[r]) = wreg[r];
    bf16x8 x[KSUB];
#pragma unroll
    for (int u = 0; u < KSUB; ++u) x[u] = tvalid ? xa[u] : bf16x8{};
    __syncthreads();
    if (k0 + KS < d) { RLOAD(k0 + KS); }
#pragma unroll
    for (int j = 0; j < NJ; ++j)
#pragma unroll
      for (int pl = 0; pl < 3; ++pl)
#pragma unroll
        for (int u = 0; u < KSUB; ++u) {
          const bf16x8 w =
              *(const bf16x8*)(Ws + (pl * 64 + (jb + j) * 32 + fr) * LDK + 16 * u + fk);
          acc[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w, x[u], acc[j], 0, 0, 0);
        }
    __syncthreads();
  }
#undef RLOAD
  // lane holds token trow and experts e0 + 32 j + 8 (q/4) + 4 (lane/32) + q%4
  if (tvalid) {
#pragma unroll
    for (int j = 0; j < NJ; ++j)
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int eb = e0 + (jb + j) * 32 + g * 8 + (lane >> 5) * 4;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int e = eb + q;
          if (e < E) {
            const float v = acc[j][g * 4 + q] + br[e];
            s[(size_t)trow * E + e] = v;
            sT[(size_t)e * T + trow] = v;
          }
        }
      }
  }
}

// ------------------------------------------------- sigma_s, fixed order
// Block b owns tokens [256b, 256b+256); thread i accumulates its token's
// row from expert 0 upward in FP64, then the block halves (stride 128..1).

__global__ __launch_bounds__(SIG_BLOCK) void score_partials(const float* __restrict__ sT, int T,
                                                            int E, double* part) {
  __shared__ double v1[SIG_BLOCK];
  __shared__ double v2[SIG_BLOCK];
  const int tid = threadIdx.x;
  const int t = blockIdx.x * SIG_BLOCK + tid;
  double r1 = 0.0, r2 = 0.0;
  if (t < T) {
    // loads batched 64 at a time (one latency for E <= 64); the additions
    // keep expert order
    for (int e0 = 0; e0 < E; e0 += 64) {
      float xv[64];
#pragma unroll
      for (int i = 0; i < 64; ++i) xv[i] = sT[(size_t)min(e0 + i, E - 1) * T + t];
#pragma unroll
      for (int i = 0; i < 64; ++i) {
        if (e0 + i < E) {
          const double v = (double)xv[i];
          r1 = r1 + v;
          r2 = r2 + v * v;
        }
      }
    }
  }
  v1[tid] = r1;
  v2[tid] = r2;
  __syncthreads();
  for (int st = SIG_BLOCK / 2; st >= 1; st >>= 1) {
    if (tid < st) {
      v1[tid] = v1[tid] + v1[tid + st];
      v2[tid] = v2[tid] + v2[tid + st];
    }
    __syncthreads();
  }
  if (tid == 0) {
    part[2 * blockIdx.x] = v1[0];
    part[2 * blockIdx.x + 1] = v2[0];
  }
}

// Running sum i takes block totals i, i+256, ... in order; then halving.
// mean = S1/n, var = max(S2/n - mean*mean, 0), sigma = fl32(sqrt(var)),
// eps = fl32(fl32(1e-3) * sigma).
__global__ __launch_bounds__(SIG_BLOCK) void score_sigma(const double* part, int nb, double n,
                                                         int32_t* state) {
  __shared__ double v1[SIG_BLOCK];
  __shared__ double v2[SIG_BLOCK];
  const int tid = threadIdx.x;
  double a1 = 0.0, a2 = 0.0;
  for (int j = tid; j < nb; j += SIG_BLOCK) {
    a1 = a1 + part[2 * j];
    a2 = a2 + part[2 * j + 1];
  }
  v1[tid] = a1;
  v2[tid] = a2;
  __syncthreads();
  for (int st = SIG_BLOCK / 2; st >= 1; st >>= 1) {
    if (tid < st) {
      v1[tid] = v1[tid] + v1[tid + st];
      v2[tid] = v2[tid] + v2[tid + st];
    }
    __syncthreads();
  }
  if (tid == 0) {
    double S1 = v1[0], S2 = v2[0];
    if (!isfinite(S1) || !isfinite(S2)) {
      state[ST_STATUS] = MOE_ENAN;
      state[ST_DONE] = 1;
      return;
    }
    double mean = S1 / n;
    double m2 = mean * mean;
    double var = S2 / n - m2;
    if (var < 0.0) var = 0.0;
    float sigma = (float)sqrt(var);
    float eps = 1.0e-3f * sigma;
    state[ST_SIGMA] = __float_as_int(sigma);
    state[ST_EPS] = __float_as_int(eps);
    state[ST_EPS0] = __float_as_int(eps);
  }
}

// ----------------------------------------------------- top-L insertion
// Composite 64-bit rank key: (sortable key of a) << 32 | (0xFFFFFFFF - e),
// so the maximum is the best expert and equal keys prefer the lower e.

__device__ __forceinline__ uint64_t rank_key(float a, int e) {
  return ((uint64_t)f32_key(a) << 32) | (uint64_t)(0xFFFFFFFFu - (uint32_t)e);
}

template <int L>
__device__ __forceinline__ void insert_top(uint64_t (&v)[L], uint64_t x) {
#pragma unroll
  for (int j = 0; j < L; ++j) {
    uint64_t hi = x > v[j] ? x : v[j];
    uint64_t lo = x > v[j] ? v[j] : x;
    v[j] = hi;
    x = lo;
  }
}

template <int L>
__device__ __forceinline__ uint64_t pick(const uint64_t (&v)[L], int j) {
  uint64_t r = 0;
#pragma unroll
  for (int i = 0; i < L; ++i)
    if (i == j) r = v[i];
  return r;
}

__device__ __forceinline__ int key_expert(uint64_t v) { return (int)(0xFFFFFFFFu - (uint32_t)v); }

// The N composite keys sorted in descending order (bitonic network, N a
// power of two): the same list insert_top builds from them, with fewer
// compare-exchanges.
template <int N>
__device__ __forceinline__ void sort_desc(uint64_t (&v)[N]) {
#pragma unroll
  for (int kk = 2; kk <= N; kk <<= 1) {
#pragma unroll
    for (int j = kk >> 1; j > 0; j >>= 1) {
#pragma unroll
      for (int i = 0; i < N; ++i) {
        const int l = i ^ j;
        if (l > i) {
          const uint64_t a = v[i], b = v[l];
          const bool sw = (i & kk) == 0 ? a < b : a > b;
          v[i] = sw ? b : a;
          v[l] = sw ? a : b;
        }
      }
    }
  }
}

// Value of lane (lane ^ 1), (lane ^ 2) or of the mirrored lane in its half
// row of eight (lane ^ 7) for the quad_perm / row_half_mirror DPP controls.
template <int CTRL>
__device__ __forceinline__ uint64_t dpp64(uint64_t x) {
  const int lo = __builtin_amdgcn_mov_dpp((int)(uint32_t)x, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(uint32_t)(x >> 32), CTRL, 0xF, 0xF, false);
  return ((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo;
}

// Maximum over each group of G (4 or 8) consecutive lanes, in every lane of
// the group.  The whole wavefront must be active.
template <int G>
__device__ __forceinline__ uint64_t group_max(uint64_t x) {
  uint64_t y = dpp64<0xB1>(x);  // quad_perm [1,0,3,2]
  x = x > y ? x : y;
  y = dpp64<0x4E>(x);  // quad_perm [2,3,0,1]
  x = x > y ? x : y;
  if (G == 8) {
    y = dpp64<0x141>(x);  // row_half_mirror
    x = x > y ? x : y;
  }
  return x;
}

// One ranking pass of the price loop.  A block owns TG groups of 64 tokens
// (one token per lane) and splits the experts into RW contiguous ranges,
// one wavefront per (token group, range); each wavefront keeps its logits
// in registers and builds a partial top-L list per token.  The RW sorted
// lists of a token are then merged by RW lanes of one wavefront (one list
// per lane, k+1 rounds of a DPP maximum over the group; every wavefront
// merges 64/RW tokens) and the routing for the current prices is written;
// then every wavefront writes the margin keys mT[e][t] of its experts.  The
// block's per-expert counts go to row blockIdx.x of cnt[nblk][E] (no global
// atomics).

// Token group of sub-group tg: gbase + tg * gstride (64 tokens each);
// the block's per-expert counts go to row crow of cnt.  With a state
// pointer the pass is skipped once the price loop is done.
template <int L, int NV, int TG, int RW>
__device__ __forceinline__ void rank_pass(const float* __restrict__ sT,
                                          const float* __restrict__ price, int T, int E, int k,
                                          const int32_t* __restrict__ state,
                                          uint32_t* __restrict__ mT, int32_t* __restrict__ idx,
                                          int32_t* __restrict__ cnt, int gbase, int gstride,
                                          int crow) {
  __shared__ int hist[MOE_MAX_E];
  __shared__ float ps[MOE_MAX_E];
  // partial lists, one padding entry per row against bank conflicts of
  // the merge's reads (RW lists of one token in one read)
  __shared__ uint64_t partv[TG][RW][L][65];
  __shared__ uint32_t kthk_s[TG][64];
  __shared__ int kthe_s[TG][64];
  __shared__ float k1_s[TG][64], k2_s[TG][64];
  constexpr int NT = 64 * RW * TG;
  const int tid = threadIdx.x, lane = tid & 63, wv = (tid >> 6) & (RW - 1);
  const int tg = tid / (64 * RW);
  const int t = (gbase + tg * gstride) * 64 + lane;
  const bool valid = t < T;
  const int tl = valid ? t : T - 1;  // out-of-range lanes read a valid row, write nothing
  const int per = (E + RW - 1) / RW;
  const int e_lo = wv * per;
  const int ne = max(0, min(E, e_lo + per) - e_lo);
  const bool cached = ne <= NV;
  // the logits, the prices and the done flag are independent loads: issue
  // them together so their latencies overlap (a wavefront whose expert
  // range is empty, E < the number of ranges, reads row E - 1 and uses none)
  float sv[NV];
  if (cached) {
#pragma unroll
    for (int i = 0; i < NV; ++i)
      sv[i] = sT[(size_t)min(e_lo + min(i, max(ne - 1, 0)), E - 1) * T + tl];
  }
  const int done = state ? state[ST_DONE] : 0;
  for (int e = tid; e < E; e += NT) {
    hist[e] = 0;
    ps[e] = price[e];
  }
  if (done) return;  // uniform: every thread read the same flag
  __syncthreads();
  // the top-L list of this wavefront's experts as composite rank keys
  // (key, then lower expert first): one 64-bit comparison per step
  uint64_t V[L];
#pragma unroll
  for (int j = 0; j < L; ++j) V[j] = 0ull;
  if (cached && NV <= 2 * L) {
    // all NV keys sorted, the best L kept (for NV <= 2L fewer
    // compare-exchanges than inserting the NV keys one by one)
    uint64_t W[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const uint32_t key = i < ne ? f32_key(sv[i] - ps[min(e_lo + i, E - 1)]) : 0u;
      W[i] = ((uint64_t)key << 32) | (uint64_t)(0xFFFFFFFFu - (uint32_t)(e_lo + i));
    }
    sort_desc<NV>(W);
#pragma unroll
    for (int j = 0; j < L; ++j) V[j] = j < NV ? W[j < NV ? j : 0] : 0ull;
  } else if (cached) {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const uint32_t key = i < ne ? f32_key(sv[i] - ps[min(e_lo + i, E - 1)]) : 0u;
      insert_top<L>(V, ((uint64_t)key << 32) | (uint64_t)(0xFFFFFFFFu - (uint32_t)(e_lo + i)));
    }
  } else {
    for (int c0 = 0; c0 < ne; c0 += NV) {
#pragma unroll
      for (int i = 0; i < NV; ++i) sv[i] = sT[(size_t)(e_lo + min(c0 + i, ne - 1)) * T + tl];
#pragma unroll
      for (int i = 0; i < NV; ++i) {
        const uint32_t key = c0 + i < ne ? f32_key(sv[i] - ps[e_lo + min(c0 + i, ne - 1)]) : 0u;
        insert_top<L>(V, ((uint64_t)key << 32) |
                             (uint64_t)(0xFFFFFFFFu - (uint32_t)(e_lo + c0 + i)));
      }
    }
  }
#pragma unroll
  for (int j = 0; j < L; ++j) partv[tg][wv][j][lane] = V[j];
  __syncthreads();
  {
    // lane: list src of token tm; the k+1 best keys of the token's RW lists
    // in order (the keys are distinct: equal scores order by expert)
    constexpr int TPW = 64 / RW;
    const int src = lane % RW, tm = wv * TPW + lane / RW;
    const int tt = (gbase + tg * gstride) * 64 + tm;
    uint64_t Q[L];
#pragma unroll
    for (int j = 0; j < L; ++j) Q[j] = partv[tg][src][j][tm];
    uint64_t k1v = 0ull, k2v = 0ull;
    for (int j = 0; j <= k && j < L; ++j) {
      const uint64_t m = group_max<RW>(Q[0]);
      const bool win = Q[0] == m;
#pragma unroll
      for (int i = 0; i + 1 < L; ++i) Q[i] = win ? Q[i + 1] : Q[i];
      Q[L - 1] = win ? 0ull : Q[L - 1];
      if (j < k && src == j % RW && tt < T) {
        const int ej = key_expert(m);
        __builtin_nontemporal_store(ej, &idx[(size_t)tt * k + j]);
        atomicAdd(&hist[ej], 1);
      }
      if (j == k - 1) k1v = m;
      if (j == k) k2v = m;
    }
    if (src == 0) {
      const uint32_t kk1 = (uint32_t)(k1v >> 32);
      kthk_s[tg][tm] = kk1;
      kthe_s[tg][tm] = key_expert(k1v);
      k1_s[tg][tm] = key_f32(kk1);
      k2_s[tg][tm] = (k < E) ? key_f32((uint32_t)(k2v >> 32)) : -INFINITY;
    }
  }
  __syncthreads();
  // margins m = s - (held ? kappa2 : kappa1), stored as sortable keys
  // (non-temporal stores, like the routing above: both are rewritten every
  // update and read by the next kernel from memory, so they are kept out
  // of the L2 write-back at the kernel boundary);
  // e is held iff (key(a_te), -e) >= (key of rank k, -its expert)
  if (valid) {
    const uint32_t kk1 = kthk_s[tg][lane];
    const int ek1 = kthe_s[tg][lane];
    const float kap1 = k1_s[tg][lane], kap2 = k2_s[tg][lane];
    if (cached) {
#pragma unroll
      for (int i = 0; i < NV; ++i) {
        if (i < ne) {
          const int e = e_lo + i;
          const uint32_t key = f32_key(sv[i] - ps[e]);
          const bool held = key > kk1 || (key == kk1 && e <= ek1);
          __builtin_nontemporal_store(f32_key(sv[i] - (held ? kap2 : kap1)), &mT[(size_t)e * T + t]);
        }
      }
    } else {
      for (int i = 0; i < ne; ++i) {
        const int e = e_lo + i;
        const float s = sT[(size_t)e * T + t];
        const uint32_t key = f32_key(s - ps[e]);
        const bool held = key > kk1 || (key == kk1 && e <= ek1);
        __builtin_nontemporal_store(f32_key(s - (held ? kap2 : kap1)), &mT[(size_t)e * T + t]);
      }
    }
  }
  for (int e = tid; e < E; e += NT) cnt[(size_t)crow * E + e] = hist[e];
}

template <int L, int NV, int TG, int RW>
__global__ __launch_bounds__(64 * RW * TG) void acp_rank(
    const float* __restrict__ sT, const float* __restrict__ price, int T, int E, int k,
    const int32_t* __restrict__ state, uint32_t* __restrict__ mT, int32_t* __restrict__ idx,
    int32_t* __restrict__ cnt) {
  rank_pass<L, NV, TG, RW>(sT, price, T, E, k, state, mT, idx, cnt, blockIdx.x * TG, 1,
                           blockIdx.x);
}

// Gate weights of the final routing: softmax of the raw logits over each
// token's k chosen experts (FP32, max-subtracted).  After a non-finite
// logit no ranking has run: every token gets the defined routing
// idx[t][j] = j with NaN weights, so that nothing downstream reads
// unwritten memory and every output the routing feeds is NaN.  KT > 0:
// k == KT known at compile time, so the k index loads (and then the k
// logit loads) are in flight together instead of one behind each guard.
template <int KT>
__global__ __launch_bounds__(256) void route_weights(const float* __restrict__ logits,
                                                     int32_t* __restrict__ idx, int T, int E,
                                                     int k_rt, const int32_t* __restrict__ state,
                                                     float* __restrict__ w) {
  const int k = KT > 0 ? KT : k_rt;
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= T || state[ST_SKIP_WEIGHTS]) return;
  if (state[ST_STATUS] != MOE_OK) {
    for (int j = 0; j < k; ++j) {
      idx[(size_t)t * k + j] = j;
      w[(size_t)t * k + j] = __builtin_nanf("");
    }
    return;
  }
  float z[MOE_MAX_K];
  float mx = -INFINITY;
#pragma unroll
  for (int j = 0; j < MOE_MAX_K; ++j) {
    z[j] = j < k ? logits[(size_t)t * E + idx[(size_t)t * k + j]] : -INFINITY;
    mx = fmaxf(mx, z[j]);
  }
  float den = 0.0f;
#pragma unroll
  for (int j = 0; j < MOE_MAX_K; ++j) {
    z[j] = j < k ? expf(z[j] - mx) : 0.0f;
    den = den + z[j];
  }
#pragma unroll
  for (int j = 0; j < MOE_MAX_K; ++j)
    if (j < k) w[(size_t)t * k + j] = z[j] / den;
}

// ------------------------------------------------ block radix selection
// r-th largest (1-based) key among the items i in [0, n) for which get(i,
// key) is true.  Digits of 11, 11 and 10 bits, a 2048-bin LDS histogram
// per pass.  Requires 1 <= r <= number of such items.  Returns the key and
// writes the number of items with a strictly larger key to *greater and the
// number of items with exactly that key to *ties.

struct SelScratch {
  uint32_t hist[2048];
  int pick_digit;
  uint32_t pick_above;
};

template <typename Get>
__device__ uint32_t block_select_rth(int n, int r, Get get, SelScratch& sc, int* greater,
                                     int* ties) {
  const int tid = threadIdx.x, bd = blockDim.x;
  uint32_t prefix = 0, mask = 0;
  int rr = r;
#pragma unroll 1
  for (int pass = 0; pass < 3; ++pass) {
    const int sh = pass == 0 ? 21 : (pass == 1 ? 10 : 0);
    const uint32_t dm = pass == 2 ? 1023u : 2047u;
    for (int i = tid; i < 2048; i += bd) sc.hist[i] = 0;
    __syncthreads();
    for (int i = tid; i < n; i += bd) {
      uint32_t key;
      if (get(i, key) && (key & mask) == prefix) atomicAdd(&sc.hist[(key >> sh) & dm], 1u);
    }
    __syncthreads();
    if (tid < 64) {
      const int l = tid;
      uint32_t sum = 0;
      for (int j = 0; j < 32; ++j) sum += sc.hist[l * 32 + ((j + l) & 31)];
      uint32_t suf = sum;
      for (int off = 1; off < 64; off <<= 1) {
        uint32_t o = __shfl_down(suf, off, 64);
        if (l + off < 64) suf += o;
      }
      const uint32_t above = suf - sum;
      if (above < (uint32_t)rr && (uint32_t)rr <= suf) {
        uint32_t acc = above;
        for (int j = 31; j >= 0; --j) {
          uint32_t h = sc.hist[l * 32 + j];
          if (acc + h >= (uint32_t)rr) {
            sc.pick_digit = l * 32 + j;
            sc.pick_above = acc;
            break;
          }
          acc += h;
        }
      }
    }
    __syncthreads();
    const int dsel = sc.pick_digit;
    const uint32_t above = sc.pick_above;
    if (pass == 2) *ties = (int)sc.hist[dsel];  // the last digit's bin: the equal keys
    __syncthreads();
    rr -= (int)above;
    prefix |= (uint32_t)dsel << sh;
    mask |= dm << sh;
  }
  *greater = r - rr;
  return prefix;
}

__device__ int block_sum(int v, int* red) {
  // red: LDS int[32]
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, nw = (blockDim.x + 63) >> 6;
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_down(v, off, 64);
  __syncthreads();
  if (lane == 0) red[wv] = v;
  __syncthreads();
  int tot = 0;
  for (int i = 0; i < nw; ++i) tot += red[i];
  __syncthreads();
  return tot;
}

// Exclusive prefix count of ``flag`` over the threads of the block, in
// thread order; *total receives the block total.
__device__ int block_excl_scan(int flag, int* red, int* total) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, nw = (blockDim.x + 63) >> 6;
  uint64_t bal = __ballot(flag);
  int in_wave = __popcll(bal & ((lane == 0) ? 0ull : (~0ull >> (64 - lane))));
  __syncthreads();
  if (lane == 0) red[wv] = __popcll(bal);
  __syncthreads();
  int before = 0, tot = 0;
  for (int i = 0; i < nw; ++i) {
    if (i < wv) before += red[i];
    tot += red[i];
  }
  __syncthreads();
  *total = tot;
  return before + in_wave;
}

// --------------------------------------------------------- price update
// One block per expert.  Every wavefront first finds, from the loads of
// this iteration, whether the loop ends here; block 0 then records the
// outcome.  An overloaded expert finds the (C+1)-th largest margin key by a
// 3-pass radix selection (11, 11, 10 bits) whose keys stay in registers
// when T is at most SEL_THREADS * SEL_KPT.  Only keys at or above a floor a
// little below the expert's current price enter the histograms (the tokens
// that do not hold the expert have margins below its price); if fewer than
// C+1 keys pass the floor, the selection restarts with no floor, so the
// result is always the exact order statistic over all T margins.
constexpr int SEL_KPT = 16;

struct alignas(16) SelShared {
  uint32_t hist[2][2048];  // passes alternate: one fills while the other is cleared
  int pick_digit;
  uint32_t pick_above;
};

// Digit holding the rr-th largest key of a 2048-bin histogram, found by one
// wavefront: lane l sums bins [32 l, 32 l + 32) (eight 16-byte reads in a
// rotated order against bank conflicts), a suffix scan over the lanes finds
// the owning lane, and 32 lanes scan that lane's bins from the top.  Writes
// the digit (or -1 if fewer than rr keys were counted) and the count of
// keys in higher digits; the caller synchronises.
__device__ void wave_pick_digit(const uint32_t* hist, int rr, SelShared& sh) {
  const int l = threadIdx.x & 63;
  const uint4* h4 = (const uint4*)hist + l * 8;
  uint32_t sum = 0;
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const uint4 v = h4[(c + l) & 7];
    sum += v.x + v.y + v.z + v.w;
  }
  uint32_t suf = sum;
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t o = __shfl_down(suf, off, 64);
    if (l + off < 64) suf += o;
  }
  const uint32_t above = suf - sum;
  const uint64_t own = __ballot(above < (uint32_t)rr && (uint32_t)rr <= suf);
  if (own == 0ull) {
    if (l == 0) sh.pick_digit = -1;
    return;
  }
  const int ow = __ffsll((unsigned long long)own) - 1;
  const uint32_t base = __shfl(above, ow, 64);
  // lanes 0..31 take the owner's bins from the highest down; inclusive
  // prefix sums over them
  const uint32_t h = l < 32 ? hist[ow * 32 + 31 - l] : 0u;
  uint32_t pre = h;
  for (int off = 1; off < 32; off <<= 1) {
    const uint32_t o = __shfl_up(pre, off, 64);
    if (l >= off) pre += o;
  }
  const uint64_t hit = __ballot(l < 32 && base + pre >= (uint32_t)rr);
  const int fl = __ffsll((unsigned long long)hit) - 1;
  if (l == fl) {
    sh.pick_digit = ow * 32 + 31 - l;
    sh.pick_above = base + pre - h;
  }
}

// The price update of one overloaded expert e (all SEL_THREADS threads):
// q = (C+1)-th largest margin key of the column, then
// p_e = max(p_e, nextafter(q, +inf) + eps).  kk holds the column when
// cached (T <= SEL_THREADS * SEL_KPT); both histograms are zero on entry.
__device__ __forceinline__ void select_update(const uint32_t* __restrict__ col,
                                              uint32_t (&kk)[SEL_KPT], bool cached, int T,
                                              int C, int e, float p_e, float* __restrict__ price,
                                              float eps, SelShared& sh) {
  const int tid = threadIdx.x;
  const uint32_t pkey = f32_key(p_e);
  uint32_t floor_key = pkey > 4096u ? pkey - 4096u : 0u;
  uint32_t prefix = 0, mask = 0;
  int rr = C + 1;
#pragma unroll 1
  for (int pass = 0; pass < 3; ++pass) {
    const int sft = pass == 0 ? 21 : (pass == 1 ? 10 : 0);
    const uint32_t dm = pass == 2 ? 1023u : 2047u;
    uint32_t* H = sh.hist[pass & 1];
    if (pass == 1)  // for the third pass; the first pass's pick is done
      for (int i = tid; i < 2048; i += SEL_THREADS) sh.hist[0][i] = 0;
    for (int c0 = 0; c0 < T; c0 += SEL_THREADS * SEL_KPT) {
      if (!cached) {
#pragma unroll
        for (int i = 0; i < SEL_KPT; ++i) {
          const int j = c0 + i * SEL_THREADS + tid;
          kk[i] = j < T ? col[j] : 0u;
        }
      }
#pragma unroll
      for (int i = 0; i < SEL_KPT; ++i) {
        if ((c0 + i * SEL_THREADS + tid < T) && kk[i] >= floor_key && ((kk[i] & mask) == prefix))
          atomicAdd(&H[(kk[i] >> sft) & dm], 1u);
      }
    }
    __syncthreads();
    if (tid < 64) wave_pick_digit(H, rr, sh);
    __syncthreads();
    const int dsel = sh.pick_digit;
    const uint32_t above = sh.pick_above;
    if (dsel < 0) {
      // fewer than C+1 keys above the floor: restart over all keys with
      // cleared histograms (a second miss cannot happen while load_e > C;
      // leave the price as is)
      if (floor_key == 0u) return;
      floor_key = 0u;
      prefix = 0u;
      mask = 0u;
      rr = C + 1;
      for (int i = tid; i < 2 * 2048; i += SEL_THREADS) (&sh.hist[0][0])[i] = 0;
      __syncthreads();
      pass = -1;
      continue;
    }
    rr -= (int)above;
    prefix |= (uint32_t)dsel << sft;
    mask |= dm << sft;
  }
  if (tid == 0) {
    const float qf = key_f32(prefix);
    const float cnd = nextafterf(qf, INFINITY) + eps;
    price[e] = cnd > p_e ? cnd : p_e;
  }
}

// subgrad != 0: the projected dual subgradient rule instead (every block
// moves its expert's price by the capacity-relative excess, no selection).
__global__ __launch_bounds__(SEL_THREADS) void acp_select(
    const uint32_t* __restrict__ mT, float* __restrict__ price, int T, int E, int C, int it,
    int max_iters, int nblk, const int32_t* __restrict__ cnt, int32_t* __restrict__ state,
    int32_t* __restrict__ load_out, int subgrad) {
  __shared__ SelShared sh;
  __shared__ int ld[MOE_MAX_E];
  const int tid = threadIdx.x, lane = tid & 63;
  const int done = state[ST_DONE];
  for (int e = tid; e < E; e += SEL_THREADS) ld[e] = 0;
  for (int i = tid; i < 2 * 2048; i += SEL_THREADS) (&sh.hist[0][0])[i] = 0;
  if (done) return;  // uniform
  // this block's margin column, requested before the load count is known
  // (the latencies overlap; blocks of experts within capacity discard it)
  const uint32_t* col = mT + (size_t)blockIdx.x * T;
  const bool cached = T <= SEL_THREADS * SEL_KPT;
  // the price and increment of this block's expert (only this block
  // writes the price, at its end)
  const float p_e = price[blockIdx.x];
  const float eps = __int_as_float(state[ST_EPS]);
  uint32_t kk[SEL_KPT];
  if (cached) {
#pragma unroll
    for (int i = 0; i < SEL_KPT; ++i) {
      const int j = i * SEL_THREADS + tid;
      kk[i] = j < T ? col[j] : 0u;
    }
  }
  __syncthreads();
  // loads of this iteration: column sums of the per-block count matrix,
  // sixteen independent loads in flight per thread
  {
    const int lanes_per_e = max(1, SEL_THREADS / E);
    for (int e0 = 0; e0 < E; e0 += SEL_THREADS) {
      const int e = e0 + tid % min(E, SEL_THREADS);
      const int r0 = tid / min(E, SEL_THREADS);
      if (e < E && r0 < lanes_per_e) {
        int sum = 0;
        int r = r0;
        for (; r + 15 * lanes_per_e < nblk; r += 16 * lanes_per_e) {
          int v[16];
#pragma unroll
          for (int u = 0; u < 16; ++u) v[u] = cnt[(size_t)(r + u * lanes_per_e) * E + e];
#pragma unroll
          for (int u = 0; u < 16; ++u) sum += v[u];
        }
        for (; r < nblk; r += lanes_per_e) sum += cnt[(size_t)r * E + e];
        atomicAdd(&ld[e], sum);
      }
    }
  }
  __syncthreads();
  // every wavefront tests the loads itself (no block reduction)
  int ov = 0;
  for (int e2 = lane; e2 < E; e2 += 64) ov |= ld[e2] > C ? 1 : 0;
  const bool any_over = __ballot(ov) != 0ull;
  const int e = blockIdx.x;
  if (!any_over || it >= max_iters) {
    if (e == 0) {
      for (int i = tid; i < E; i += SEL_THREADS) load_out[i] = ld[i];
      if (tid < 64) {
        int ex = 0;
        for (int e2 = lane; e2 < E; e2 += 64) ex += max(ld[e2] - C, 0);
        for (int off = 32; off >= 1; off >>= 1) ex += __shfl_down(ex, off, 64);
        if (tid == 0) {
          state[ST_ITERS] = it;
          state[ST_CONVERGED] = !any_over;
          state[ST_OVERFLOW] = ex;
          state[ST_NEED_REPAIR] = any_over;
          state[ST_DONE] = 1;
        }
      }
    }
    return;
  }
  if (subgrad) {
    if (tid == 0) {
      const float eta = (256.0f * eps) / sqrtf((float)(it + 1));
      const float g = (float)(ld[e] - C) / (float)C;
      const float x = p_e + eta * g;
      price[e] = x > 0.0f ? x : 0.0f;
    }
    return;
  }
  if (ld[e] <= C) return;
  select_update(col, kk, cached, T, C, e, p_e, price, eps, sh);
}

// --------------------------------------------- epsilon-scaled restarts
// Between two runs of the price update.  When the previous run converged
// and some expert is priced above zero yet below capacity (a nonzero
// certificate gap), every price is lowered by four increments (a result
// that is not positive becomes +0), the increment is divided by eight and
// the update runs again from those prices; otherwise every later run is
// skipped.  The updates of finished runs are summed in ST_ITERS_PREV.
__global__ __launch_bounds__(256) void scaled_restart(int32_t* __restrict__ state,
                                                      float* __restrict__ price,
                                                      const int32_t* __restrict__ load, int E,
                                                      int C) {
  __shared__ int slack, go;
  __shared__ float eps_s;
  const int tid = threadIdx.x;
  if (tid == 0) {
    slack = 0;
    eps_s = __int_as_float(state[ST_EPS]);
  }
  __syncthreads();
  const bool active =
      !state[ST_STAGE_STOP] && state[ST_STATUS] == MOE_OK && state[ST_CONVERGED] != 0;
  if (active)
    for (int e = tid; e < E; e += blockDim.x)
      if (price[e] != 0.0f && load[e] != C) slack = 1;
  __syncthreads();
  if (tid == 0) go = active && slack;
  __syncthreads();
  if (!go) {
    if (tid == 0) state[ST_STAGE_STOP] = 1;
    return;
  }
  const float back = 4.0f * eps_s;
  for (int e = tid; e < E; e += blockDim.x) {
    const float lowered = price[e] - back;
    price[e] = lowered > 0.0f ? lowered : 0.0f;
  }
  if (tid == 0) {
    state[ST_ITERS_PREV] += state[ST_ITERS];
    state[ST_ITERS] = 0;
    state[ST_CONVERGED] = 0;
    state[ST_OVERFLOW] = 0;
    state[ST_NEED_REPAIR] = 0;
    state[ST_EPS] = __float_as_int(eps_s / 8.0f);
    state[ST_DONE] = 0;
  }
}

// ----------------------------------------------------- capacity repair
// Single block; runs only when the price loop ended with an overloaded
// expert.  Bitmasks of W = ceil(E/32) words per token live in the workspace.

struct RepairLds {
  SelScratch sc;
  int load[MOE_MAX_E];
  int props[MOE_MAX_E];
  int red[32];
  int flag;
};

template <int L>
__global__ __launch_bounds__(REP_THREADS) void capacity_repair(
    const float* __restrict__ sT, const float* __restrict__ logits,
    const float* __restrict__ price, int T, int E, int k, int C, int32_t* __restrict__ state,
    int32_t* __restrict__ idx, float* __restrict__ w, int32_t* __restrict__ load_out,
    uint32_t* __restrict__ held, uint32_t* __restrict__ tried, uint32_t* __restrict__ prop,
    int32_t* __restrict__ missing) {
  if (!state[ST_NEED_REPAIR] || state[ST_STATUS] != MOE_OK) return;
  __shared__ RepairLds S;
  const int tid = threadIdx.x, bd = blockDim.x;
  const int W = (E + 31) >> 5;
  auto keyof = [&](int t, int e) -> uint32_t { return f32_key(sT[(size_t)e * T + t] - price[e]); };
  auto has = [&](const uint32_t* m, int t, int e) -> bool {
    return (m[(size_t)t * W + (e >> 5)] >> (e & 31)) & 1u;
  };
  for (int e = tid; e < E; e += bd) {
    S.load[e] = 0;
    S.props[e] = 0;
  }
  __syncthreads();
  for (int t = tid; t < T; t += bd) {
    for (int j = 0; j < W; ++j) {
      held[(size_t)t * W + j] = 0;
      prop[(size_t)t * W + j] = 0;
    }
    for (int j = 0; j < k; ++j) {
      int e = idx[(size_t)t * k + j];
      held[(size_t)t * W + (e >> 5)] |= 1u << (e & 31);
      atomicAdd(&S.load[e], 1);
    }
    for (int j = 0; j < W; ++j) tried[(size_t)t * W + j] = held[(size_t)t * W + j];
    missing[t] = 0;
  }
  __syncthreads();
  // 1) overloaded experts keep their C best holders (key desc, token asc)
  for (int e = 0; e < E; ++e) {
    if (S.load[e] <= C) continue;
    int greater, ties;
    uint32_t kstar = block_select_rth(
        T, C,
        [&](int t, uint32_t& key) {
          if (!has(held, t, e)) return false;
          key = keyof(t, e);
          return true;
        },
        S.sc, &greater, &ties);
    const int need = C - greater;
    if (ties == need) {
      // every holder with the C-th key stays: no order among equal keys is
      // needed, each token is decided by its own key
      for (int t = tid; t < T; t += bd) {
        if (has(held, t, e) && keyof(t, e) < kstar) {
          held[(size_t)t * W + (e >> 5)] &= ~(1u << (e & 31));
          missing[t] += 1;
        }
      }
      __syncthreads();
      if (tid == 0) S.load[e] = C;
      __syncthreads();
      continue;
    }
    int run = 0;
    for (int t0 = 0; t0 < T; t0 += bd) {
      const int t = t0 + tid;
      bool h = t < T && has(held, t, e);
      uint32_t key = h ? keyof(t, e) : 0u;
      int tot;
      int rank = block_excl_scan(h && key == kstar, S.red, &tot);
      if (h && !(key > kstar || (key == kstar && run + rank < need))) {
        held[(size_t)t * W + (e >> 5)] &= ~(1u << (e & 31));
        missing[t] += 1;
      }
      run += tot;
    }
    __syncthreads();
    if (tid == 0) S.load[e] = C;
    __syncthreads();
  }
  // 2) proposal rounds
  int rounds = 0;
  for (;;) {
    if (tid == 0) S.flag = 0;
    for (int e = tid; e < E; e += bd) S.props[e] = 0;
    __syncthreads();
    int short_tokens = 0;
    for (int t = tid; t < T; t += bd) {
      int need = missing[t];
      if (need == 0) continue;
      short_tokens = 1;
      for (int q = 0; q < need; ++q) {
        uint64_t best = 0;
        for (int e = 0; e < E; ++e) {
          if (has(tried, t, e)) continue;
          uint64_t rk = ((uint64_t)keyof(t, e) << 32) | (uint64_t)(0xFFFFFFFFu - (uint32_t)e);
          if (rk > best) best = rk;
        }
        if (best == 0) {
          atomicOr(&S.flag, 1);
          break;
        }
        int e = key_expert(best);
        tried[(size_t)t * W + (e >> 5)] |= 1u << (e & 31);
        prop[(size_t)t * W + (e >> 5)] |= 1u << (e & 31);
        atomicAdd(&S.props[e], 1);
      }
    }
    const int any_short = block_sum(short_tokens, S.red);
    if (S.flag) {
      if (tid == 0) state[ST_STATUS] = MOE_ECAPACITY;
      break;
    }
    if (any_short == 0) break;
    ++rounds;
    for (int e = 0; e < E; ++e) {
      const int P = S.props[e];
      if (P == 0) continue;
      const int room = C - S.load[e];
      uint32_t kstar = 0;
      int need = 0, ties = 0;
      bool all = P <= room;
      if (!all && room > 0) {
        int greater;
        kstar = block_select_rth(
            T, room,
            [&](int t, uint32_t& key) {
              if (!has(prop, t, e)) return false;
              key = keyof(t, e);
              return true;
            },
            S.sc, &greater, &ties);
        need = room - greater;
      }
      if (all || room <= 0 || ties == need) {
        // every proposal accepted, none, or all at or above the room-th key
        // (the equal keys fit): each token is decided by its own key
        int accepted = 0;
        for (int t = tid; t < T; t += bd) {
          if (!has(prop, t, e)) continue;
          prop[(size_t)t * W + (e >> 5)] &= ~(1u << (e & 31));
          if (room > 0 && (all || keyof(t, e) >= kstar)) {
            held[(size_t)t * W + (e >> 5)] |= 1u << (e & 31);
            missing[t] -= 1;
            ++accepted;
          }
        }
        const int acc_tot = block_sum(accepted, S.red);
        if (tid == 0) S.load[e] += acc_tot;
        __syncthreads();
        continue;
      }
      int run = 0, accepted = 0;
      for (int t0 = 0; t0 < T; t0 += bd) {
        const int t = t0 + tid;
        bool p = t < T && has(prop, t, e);
        uint32_t key = p ? keyof(t, e) : 0u;
        int tot;
        int rank = block_excl_scan(p && key == kstar, S.red, &tot);
        bool acc = p && room > 0 && (all || key > kstar || (key == kstar && run + rank < need));
        if (p) prop[(size_t)t * W + (e >> 5)] &= ~(1u << (e & 31));
        if (acc) {
          held[(size_t)t * W + (e >> 5)] |= 1u << (e & 31);
          missing[t] -= 1;
        }
        accepted += acc;
        run += tot;
      }
      const int acc_tot = block_sum(accepted, S.red);
      if (tid == 0) S.load[e] += acc_tot;
      __syncthreads();
    }
  }
  __syncthreads();
  // the proposal loop leaves only through a round with no short token
  // (S.flag clear) or through a token with no untried expert (S.flag set)
  const bool failed = S.flag != 0;
  // 3) rebuild every token's list in rank order, and its gate weights
  if (!failed) {
    for (int e = tid; e < E; e += bd) S.load[e] = 0;
    __syncthreads();
    for (int t = tid; t < T; t += bd) {
      uint64_t v[L];
#pragma unroll
      for (int j = 0; j < L; ++j) v[j] = 0;
      for (int e = 0; e < E; ++e)
        if (has(held, t, e))
          insert_top<L>(v, ((uint64_t)keyof(t, e) << 32) | (uint64_t)(0xFFFFFFFFu - (uint32_t)e));
      float mx = -INFINITY;
#pragma unroll
      for (int j = 0; j < L; ++j)
        if (j < k) mx = fmaxf(mx, logits[(size_t)t * E + key_expert(v[j])]);
      float ex[L];
      float den = 0.0f;
#pragma unroll
      for (int j = 0; j < L; ++j) {
        ex[j] = 0.0f;
        if (j < k) {
          ex[j] = expf(logits[(size_t)t * E + key_expert(v[j])] - mx);
          den = den + ex[j];
        }
      }
#pragma unroll
      for (int j = 0; j < L; ++j)
        if (j < k) {
          int ej = key_expert(v[j]);
          idx[(size_t)t * k + j] = ej;
          w[(size_t)t * k + j] = ex[j] / den;
          atomicAdd(&S.load[ej], 1);
        }
    }
    __syncthreads();
    for (int e = tid; e < E; e += bd) load_out[e] = S.load[e];
  } else {
    // the repair could not place every slot: idx and load keep the
    // overloaded routing the price loop ended with, and the weights become
    // NaN so that no output computed from it passes for a valid one
    for (int t = tid; t < T; t += bd)
      for (int j = 0; j < k; ++j) w[(size_t)t * k + j] = __builtin_nanf("");
  }
  if (tid == 0) {
    state[ST_ROUNDS] = rounds;
    state[ST_REPAIRED] = 1;
  }
}

// info[] from the state words.  An empty batch has zero loads; after a
// non-finite logit the loads are those of the placeholder routing
// idx[t][j] = j (T for experts below k, zero above).
__global__ void route_finalize(const int32_t* state, int32_t* info, int32_t* load_out, int T,
                               int E, int k, int empty) {
  const int tid = threadIdx.x;
  if (empty)
    for (int e = tid; e < E; e += blockDim.x) load_out[e] = 0;
  else if (state[ST_STATUS] == MOE_ENAN)
    for (int e = tid; e < E; e += blockDim.x) load_out[e] = e < k ? T : 0;
  if (tid == 0) {
    info[MOE_INFO_ITERS] = state[ST_ITERS] + state[ST_ITERS_PREV];
    info[MOE_INFO_CONVERGED] = empty ? 1 : state[ST_CONVERGED];
    info[MOE_INFO_OVERFLOW] = state[ST_OVERFLOW];
    info[MOE_INFO_STATUS] = state[ST_STATUS];
    info[MOE_INFO_ROUNDS] = state[ST_ROUNDS];
    info[MOE_INFO_SIGMA] = state[ST_SIGMA];
    info[MOE_INFO_EPS] = state[ST_EPS];
    info[MOE_INFO_REPAIRED] = state[ST_REPAIRED];
  }
}

struct RouteWs {
  bf16_t* W3;
  float* sT;
  uint32_t* mT;
  int32_t* state;
  int32_t* cnt;
  double* part;
  uint32_t *held, *tried, *prop;
  int32_t* missing;
};

RouteWs carve_route(const moe_cfg& c, void* base, size_t* total) {
  WsCarve wc{(char*)base, 0};
  RouteWs r;
  const size_t T = (size_t)c.T, E = (size_t)c.E;
  const size_t W = (E + 31) / 32;
  const size_t nb = (T + SIG_BLOCK - 1) / SIG_BLOCK;
  r.W3 = wc.take<bf16_t>(3 * E * (size_t)c.d);
  r.sT = wc.take<float>(T * E);
  r.mT = wc.take<uint32_t>(T * E);
  r.state = wc.take<int32_t>(ST_LEN);
  r.cnt = wc.take<int32_t>(((T + 63) / 64 + 1) * E);  // one row per rank block
  r.part = wc.take<double>(2 * (nb > 0 ? nb : 1));
  r.held = wc.take<uint32_t>(T * W);
  r.tried = wc.take<uint32_t>(T * W);
  r.prop = wc.take<uint32_t>(T * W);
  r.missing = wc.take<int32_t>(T);
  if (total) *total = align_up(wc.off, 256);
  return r;
}

template <int L>
void launch_rank_select_repair(const moe_cfg& c, const RouteWs& ws, const float* logits,
                               float* price, int32_t* idx, float* w, int32_t* load,
                               int max_iters, hipStream_t st) {
  const int T = c.T, E = c.E, k = c.k, C = c.capacity;
  // one 64-token group per block: T/64 blocks keep every CU busy at
  // T = 16384 (four groups per block left three quarters of the chip idle)
  constexpr int TG = 1;
  const int nblk = (T + 64 * TG - 1) / (64 * TG);
  // eight wavefronts per token group (two per SIMD) for lists of up to 9,
  // four for the longer lists (their LDS would not fit twice)
  constexpr int RW = L <= 9 ? 8 : 4;
  const int per = (E + RW - 1) / RW;
  // one ranking and one update kernel per iteration, each exiting at once
  // after the loop has stopped; epsilon-scaled restarts repeat the loop
  const int stages = max_iters > 0 && c.price_mode != MOE_PRICE_SUBGRAD ? c.price_stages : 0;
  for (int stage = 0; stage <= stages; ++stage) {
  if (stage > 0)
    hipLaunchKernelGGL(scaled_restart, dim3(1), dim3(256), 0, st, ws.state, price, load, E, C);
  for (int it = 0; it <= max_iters; ++it) {
    const dim3 rb(64 * RW * TG);
    if (per <= 4)
      hipLaunchKernelGGL(HIP_KERNEL_NAME(acp_rank<L, 4, TG, RW>), dim3(nblk), rb, 0, st, ws.sT,
                         price, T, E, k, ws.state, ws.mT, idx, ws.cnt);
    else if (per <= 8)
      hipLaunchKernelGGL(HIP_KERNEL_NAME(acp_rank<L, 8, TG, RW>), dim3(nblk), rb, 0, st, ws.sT,
                         price, T, E, k, ws.state, ws.mT, idx, ws.cnt);
    else if (per <= 16)
      hipLaunchKernelGGL(HIP_KERNEL_NAME(acp_rank<L, 16, TG, RW>), dim3(nblk), rb, 0, st, ws.sT,
                         price, T, E, k, ws.state, ws.mT, idx, ws.cnt);
    else if (per <= 32)
      hipLaunchKernelGGL(HIP_KERNEL_NAME(acp_rank<L, 32, TG, RW>), dim3(nblk), rb, 0, st, ws.sT,
                         price, T, E, k, ws.state, ws.mT, idx, ws.cnt);
    else
      hipLaunchKernelGGL(HIP_KERNEL_NAME(acp_rank<L, 64, TG, RW>), dim3(nblk), rb, 0, st, ws.sT,
                         price, T, E, k, ws.state, ws.mT, idx, ws.cnt);
    hipLaunchKernelGGL(acp_select, dim3(E), dim3(SEL_THREADS), 0, st, ws.mT, price, T, E, C, it,
                       max_iters, nblk, ws.cnt, ws.state, load,
                       (int)(c.price_mode == MOE_PRICE_SUBGRAD));
  }
  }
  if (k == 8)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(route_weights<8>), dim3((T + 255) / 256), dim3(256), 0, st,
                       logits, idx, T, E, k, ws.state, w);
  else
    hipLaunchKernelGGL(HIP_KERNEL_NAME(route_weights<0>), dim3((T + 255) / 256), dim3(256), 0, st,
                       logits, idx, T, E, k, ws.state, w);
  hipLaunchKernelGGL(HIP_KERNEL_NAME(capacity_repair<L>), dim3(1), dim3(REP_THREADS), 0, st,
                     ws.sT, logits, price, T, E, k, C, ws.state, idx, w, load, ws.held, ws.tried,
                     ws.prop, ws.missing);
}

moe_status route_from_scores(const moe_cfg& c, const RouteWs& w, const float* logits,
                             float* price, int32_t* topk_idx, float* topk_w, int32_t* load,
                             int32_t* info, hipStream_t st);

// s = X W_r^T + b_r and its transpose sT in the workspace.
void launch_router(const moe_cfg& c, const RouteWs& w, const void* X, const float* Wr,
                   const float* br, float* logits, hipStream_t st) {
  dim3 g((c.T + 63) / 64, (c.E + 63) / 64);
  PROF_BEGIN("router_logits", st);
  if (c.act == MOE_F32)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(router_logits<float>), g, dim3(256), 0, st,
                       (const float*)X, Wr, br, logits, w.sT, c.T, c.d, c.E);
  else if (c.d % 32 != 0)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(router_logits<bf16_t>), g, dim3(256), 0, st,
                       (const bf16_t*)X, Wr, br, logits, w.sT, c.T, c.d, c.E);
  else {
    const int n = c.E * c.d;
    hipLaunchKernelGGL(router_split, dim3((n + 255) / 256), dim3(256), 0, st, Wr, n, w.W3);
    // 128-token blocks once they give at least two blocks per CU, 64 below
    const int eg = (c.E + 63) / 64;
    const bool big = (size_t)((c.T + 127) / 128) * eg >= 512;
    const dim3 g(big ? (c.T + 127) / 128 : (c.T + 63) / 64, eg);
    if (c.d % 128 == 0) {
      if (big)
        hipLaunchKernelGGL(HIP_KERNEL_NAME(router_logits_mfma<128, 128>), g, dim3(256), 0, st,
                           (const bf16_t*)X, w.W3, br, logits, w.sT, c.T, c.d, c.E);
      else
        hipLaunchKernelGGL(HIP_KERNEL_NAME(router_logits_mfma<128, 64>), g, dim3(256), 0, st,
                           (const bf16_t*)X, w.W3, br, logits, w.sT, c.T, c.d, c.E);
    } else {
      if (big)
        hipLaunchKernelGGL(HIP_KERNEL_NAME(router_logits_mfma<32, 128>), g, dim3(256), 0, st,
                           (const bf16_t*)X, w.W3, br, logits, w.sT, c.T, c.d, c.E);
      else
        hipLaunchKernelGGL(HIP_KERNEL_NAME(router_logits_mfma<32, 64>), g, dim3(256), 0, st,
                           (const bf16_t*)X, w.W3, br, logits, w.sT, c.T, c.d, c.E);
    }
  }
  PROF_END("router_logits", st);
}


moe_status route_check(const moe_cfg* cfg, const float* logits, float* price, int32_t* topk_idx,
                       float* topk_w, int32_t* load, int32_t* info, void* ws, size_t ws_bytes) {
  moe_status stc = check_cfg_shape(cfg);
  if (stc != MOE_OK) return stc;
  const moe_cfg& c = *cfg;
  if (c.price_mode < MOE_PRICE_NONE || c.price_mode > MOE_PRICE_SUBGRAD) return MOE_EINVAL;
  if (c.max_iters < 0) return MOE_EINVAL;
  if (!price || !load || !info) return MOE_EINVAL;
  if (c.T > 0 && (!logits || !topk_idx || !topk_w)) return MOE_EINVAL;
  if (!aligned(logits, 4) || !aligned(price, 4) || !aligned(topk_idx, 4) ||
      !aligned(topk_w, 4) || !aligned(load, 4) || !aligned(info, 4))
    return MOE_EINVAL;
  if (ws_bytes < route_ws_bytes(c) || !ws) return MOE_EWORKSPACE;
  return MOE_OK;
}

}  // namespace

size_t route_ws_bytes(const moe_cfg& c) {
  size_t total = 0;
  carve_route(c, nullptr, &total);
  return total;
}

extern "C" moe_status moe_route(const moe_cfg* cfg, const void* X, const float* Wr,
                                const float* br, float* logits, float* price, int32_t* topk_idx,
                                float* topk_w, int32_t* load, int32_t* info, void* ws,
                                size_t ws_bytes, void* stream) {
  moe_status stc = route_check(cfg, logits, price, topk_idx, topk_w, load, info, ws, ws_bytes);
  if (stc != MOE_OK) return stc;
  const moe_cfg& c = *cfg;
  if (c.T > 0 && (!X || !Wr || !br)) return MOE_EINVAL;
  if (!aligned(X, 16) || !aligned(Wr, 4) || !aligned(br, 4)) return MOE_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  RouteWs w = carve_route(c, ws, nullptr);
  hipLaunchKernelGGL(route_init, dim3(1), dim3(256), 0, st, w.state, c.E, price,
                     c.price_mode, c.warm_gamma);
  if (c.T == 0) {
    hipLaunchKernelGGL(route_finalize, dim3(1), dim3(256), 0, st, w.state, info, load, c.T, c.E,
                       c.k, 1);
    MOE_LAUNCH_CHECK();
    return MOE_OK;
  }
  launch_router(c, w, X, Wr, br, logits, st);
  return route_from_scores(c, w, logits, price, topk_idx, topk_w, load, info, st);
}

extern "C" moe_status moe_router_logits(const moe_cfg* cfg, const void* X, const float* Wr,
                                        const float* br, float* logits, void* ws,
                                        size_t ws_bytes, void* stream) {
  moe_status stc = check_cfg_shape(cfg);
  if (stc != MOE_OK) return stc;
  const moe_cfg& c = *cfg;
  if (c.T == 0) return MOE_OK;
  if (!X || !Wr || !br || !logits) return MOE_EINVAL;
  if (!aligned(X, 16) || !aligned(Wr, 4) || !aligned(br, 4) || !aligned(logits, 4))
    return MOE_EINVAL;
  if (ws_bytes < route_ws_bytes(c) || !ws) return MOE_EWORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  RouteWs w = carve_route(c, ws, nullptr);
  launch_router(c, w, X, Wr, br, logits, st);
  MOE_LAUNCH_CHECK();
  return MOE_OK;
}

namespace {

// The price loop (iters updates at most), the gate weights and the repair,
// for the list length of k.
void launch_loop(const moe_cfg& c, const RouteWs& w, const float* logits, float* price,
                 int32_t* topk_idx, float* topk_w, int32_t* load, int iters, hipStream_t st) {
  const int L = c.k + 1;
  if (L <= 3)
    launch_rank_select_repair<3>(c, w, logits, price, topk_idx, topk_w, load, iters, st);
  else if (L <= 5)
    launch_rank_select_repair<5>(c, w, logits, price, topk_idx, topk_w, load, iters, st);
  else if (L <= 9)
    launch_rank_select_repair<9>(c, w, logits, price, topk_idx, topk_w, load, iters, st);
  else
    launch_rank_select_repair<17>(c, w, logits, price, topk_idx, topk_w, load, iters, st);
}

// Everything after the logits: sigma_s, the price loop, weights, repair.
moe_status route_from_scores(const moe_cfg& c, const RouteWs& w, const float* logits,
                             float* price, int32_t* topk_idx, float* topk_w, int32_t* load,
                             int32_t* info, hipStream_t st) {
  const int nb = (c.T + SIG_BLOCK - 1) / SIG_BLOCK;
  hipLaunchKernelGGL(score_partials, dim3(nb), dim3(SIG_BLOCK), 0, st, w.sT, c.T, c.E, w.part);
  hipLaunchKernelGGL(score_sigma, dim3(1), dim3(SIG_BLOCK), 0, st, w.part, nb,
                     (double)c.T * (double)c.E, w.state);
  const int iters = (c.price_mode == MOE_PRICE_ACP || c.price_mode == MOE_PRICE_WARM ||
                     c.price_mode == MOE_PRICE_SUBGRAD)
                        ? c.max_iters
                        : 0;
  PROF_BEGIN("price_loop", st);
  launch_loop(c, w, logits, price, topk_idx, topk_w, load, iters, st);
  PROF_END("price_loop", st);
  hipLaunchKernelGGL(route_finalize, dim3(1), dim3(64), 0, st, w.state, info, load, c.T, c.E,
                     c.k, 0);
  MOE_LAUNCH_CHECK();
  return MOE_OK;
}

}  // namespace

extern "C" moe_status moe_route_logits(const moe_cfg* cfg, const float* logits, float* price,
                                       int32_t* topk_idx, float* topk_w, int32_t* load,
                                       int32_t* info, void* ws, size_t ws_bytes, void* stream) {
  moe_status stc = route_check(cfg, logits, price, topk_idx, topk_w, load, info, ws, ws_bytes);
  if (stc != MOE_OK) return stc;
  const moe_cfg& c = *cfg;
  hipStream_t st = (hipStream_t)stream;
  RouteWs w = carve_route(c, ws, nullptr);
  hipLaunchKernelGGL(route_init, dim3(1), dim3(256), 0, st, w.state, c.E, price,
                     c.price_mode, c.warm_gamma);
  if (c.T == 0) {
    hipLaunchKernelGGL(route_finalize, dim3(1), dim3(256), 0, st, w.state, info, load, c.T, c.E,
                       c.k, 1);
    MOE_LAUNCH_CHECK();
    return MOE_OK;
  }
  hipLaunchKernelGGL(logits_transpose, dim3((c.T + 63) / 64, (c.E + 63) / 64), dim3(256), 0, st,
                     logits, c.T, c.E, w.sT);
  return route_from_scores(c, w, logits, price, topk_idx, topk_w, load, info, st);
}

// The price update alone: the routing it ends with (idx, w, load) goes to
// the tail of the workspace, after what moe_route_logits needs.
namespace {
struct PriceScratch {
  int32_t* idx;
  float* w;
  int32_t* load;
};

PriceScratch carve_price_scratch(const moe_cfg& c, void* base, size_t* total) {
  const size_t head = route_ws_bytes(c);
  WsCarve wc{base ? (char*)base + head : nullptr, 0};
  PriceScratch r;
  r.idx = wc.take<int32_t>((size_t)c.T * c.k);
  r.w = wc.take<float>((size_t)c.T * c.k);
  r.load = wc.take<int32_t>((size_t)c.E);
  if (total) *total = head + align_up(wc.off, 256);
  return r;
}
}  // namespace

size_t price_ws_bytes(const moe_cfg& c) {
  size_t total = 0;
  carve_price_scratch(c, nullptr, &total);
  return total;
}

extern "C" moe_status moe_price_update(const moe_cfg* cfg, const float* logits, float* price,
                                       int32_t* info, void* ws, size_t ws_bytes, void* stream) {
  moe_status stc = check_cfg_shape(cfg);
  if (stc != MOE_OK) return stc;
  if (ws_bytes < price_ws_bytes(*cfg) || !ws) return MOE_EWORKSPACE;
  PriceScratch sc = carve_price_scratch(*cfg, ws, nullptr);
  return moe_route_logits(cfg, logits, price, sc.idx, sc.w, sc.load, info, ws, ws_bytes, stream);
}

// ------------------------------------------------ judged learned prices
// moe_route_judged: route from learned prices (warm start or replacement),
// certify the result, and on the device either keep it or route the batch
// again by the update from zero prices.  No host synchronisation: the
// fallback pass is always enqueued and every one of its kernels exits at
// once when the learned routing was kept.
namespace {

__global__ void judge_init(int32_t* state, int E, const float* __restrict__ p_hat,
                           float* __restrict__ price, int mode, float gamma) {
  const int tid = threadIdx.x;
  if (tid < ST_LEN) state[tid] = 0;
  for (int e = tid; e < E; e += blockDim.x)
    price[e] = mode == MOE_PRICE_WARM ? gamma * p_hat[e] : p_hat[e];
}

// Keep the learned routing if it is valid and its relative certificate gap
// is at most gap_tol; otherwise reset the state words and prices for the
// update from p = 0.  A non-finite logit is kept as it is (a second pass
// would meet the same logits).
__global__ void judge_decide(const double* __restrict__ cert, int32_t* state,
                             float* __restrict__ price, int E, int N, float gap_tol,
                             double* __restrict__ verdict, int reset) {
  __shared__ int keep_s;
  const int tid = threadIdx.x;
  if (tid == 0) {
    const int status = state[ST_STATUS];
    const double gap = cert[2];
    const bool ok = status == MOE_OK && gap <= (double)gap_tol;
    const bool keep = ok || status == MOE_ENAN || !reset;
    verdict[0] = (double)state[ST_OVERFLOW] / (double)(N > 0 ? N : 1);
    verdict[1] = status == MOE_OK ? gap : __builtin_nan("");
    verdict[2] = ok ? 1.0 : 0.0;
    verdict[4] = (double)(state[ST_ITERS] + state[ST_ITERS_PREV]);
    if (keep) {
      state[ST_DONE] = 1;
      state[ST_NEED_REPAIR] = 0;
      state[ST_SKIP_WEIGHTS] = 1;
      state[ST_STAGE_STOP] = 1;
    } else {
      state[ST_DONE] = 0;
      state[ST_CONVERGED] = 0;
      state[ST_ITERS] = 0;
      state[ST_OVERFLOW] = 0;
      state[ST_STATUS] = MOE_OK;
      state[ST_ROUNDS] = 0;
      state[ST_NEED_REPAIR] = 0;
      state[ST_REPAIRED] = 0;
      state[ST_SKIP_WEIGHTS] = 0;
      state[ST_ITERS_PREV] = 0;
      state[ST_STAGE_STOP] = 0;
      state[ST_EPS] = state[ST_EPS0];
    }
    keep_s = keep;
  }
  __syncthreads();
  if (!keep_s)
    for (int e = tid; e < E; e += blockDim.x) price[e] = 0.0f;
}

__global__ void judge_final(const double* __restrict__ cert, const int32_t* state,
                            double* __restrict__ verdict, int empty) {
  if (threadIdx.x != 0) return;
  if (empty) {
    verdict[0] = 0.0;
    verdict[1] = 0.0;
    verdict[2] = 1.0;
    verdict[3] = 0.0;
    verdict[4] = 0.0;
    return;
  }
  verdict[3] = state[ST_STATUS] == MOE_OK ? cert[2] : __builtin_nan("");
}

struct JudgeScratch {
  double* part;
  double* cert;
};

JudgeScratch carve_judge_scratch(const moe_cfg& c, void* base, size_t* total) {
  const size_t head = route_ws_bytes(c);
  WsCarve wc{base ? (char*)base + head : nullptr, 0};
  JudgeScratch r;
  r.part = wc.take<double>(2 * (((size_t)c.T + 63) / 64 + 1));
  r.cert = wc.take<double>(4);
  if (total) *total = head + align_up(wc.off, 256);
  return r;
}

}  // namespace

size_t judged_ws_bytes(const moe_cfg& c) {
  size_t total = 0;
  carve_judge_scratch(c, nullptr, &total);
  return total;
}

namespace {

moe_status route_learned_impl(const moe_cfg* cfg, const float* logits, const float* price_hat,
                              float gap_tol, float* price, int32_t* topk_idx, float* topk_w,
                              int32_t* load, int32_t* info, double* verdict, void* ws,
                              size_t ws_bytes, void* stream, bool device_fallback) {
  moe_status stc = check_cfg_shape(cfg);
  if (stc != MOE_OK) return stc;
  const moe_cfg& c = *cfg;
  if (c.price_mode != MOE_PRICE_WARM && c.price_mode != MOE_PRICE_GIVEN) return MOE_EINVAL;
  if (!price_hat || !verdict || !aligned(price_hat, 4) || !aligned(verdict, 8))
    return MOE_EINVAL;
  if (!(gap_tol >= 0.0f) || !(gap_tol < INFINITY)) return MOE_EINVAL;
  if (ws_bytes < judged_ws_bytes(c) || !ws) return MOE_EWORKSPACE;
  stc = route_check(cfg, logits, price, topk_idx, topk_w, load, info, ws, ws_bytes);
  if (stc != MOE_OK) return stc;
  hipStream_t st = (hipStream_t)stream;
  RouteWs w = carve_route(c, ws, nullptr);
  JudgeScratch js = carve_judge_scratch(c, ws, nullptr);
  hipLaunchKernelGGL(judge_init, dim3(1), dim3(256), 0, st, w.state, c.E, price_hat, price,
                     c.price_mode, c.warm_gamma);
  if (c.T == 0) {
    hipLaunchKernelGGL(route_finalize, dim3(1), dim3(256), 0, st, w.state, info, load, c.T, c.E,
                       c.k, 1);
    hipLaunchKernelGGL(judge_final, dim3(1), dim3(64), 0, st, js.cert, w.state, verdict, 1);
    MOE_LAUNCH_CHECK();
    return MOE_OK;
  }
  hipLaunchKernelGGL(logits_transpose, dim3((c.T + 63) / 64, (c.E + 63) / 64), dim3(256), 0, st,
                     logits, c.T, c.E, w.sT);
  // 1) the learned pass: warm-started update, or p_hat alone plus repair
  stc = route_from_scores(c, w, logits, price, topk_idx, topk_w, load, info, st);
  if (stc != MOE_OK) return stc;
  launch_certify(c, logits, price, topk_idx, js.part, js.cert, st);
  hipLaunchKernelGGL(judge_decide, dim3(1), dim3(256), 0, st, js.cert, w.state, price, c.E,
                     c.T * c.k, gap_tol, verdict, device_fallback ? 1 : 0);
  if (device_fallback) {
    // 2) the fallback: the update from p = 0 (nothing runs if the learned
    //    routing was kept)
    moe_cfg c0 = c;
    c0.price_mode = MOE_PRICE_ACP;
    launch_loop(c0, w, logits, price, topk_idx, topk_w, load, c.max_iters, st);
    hipLaunchKernelGGL(route_finalize, dim3(1), dim3(64), 0, st, w.state, info, load, c.T, c.E,
                       c.k, 0);
    launch_certify(c, logits, price, topk_idx, js.part, js.cert, st);
  }
  hipLaunchKernelGGL(judge_final, dim3(1), dim3(64), 0, st, js.cert, w.state, verdict, 0);
  MOE_LAUNCH_CHECK();
  return MOE_OK;
}

}  // namespace

extern "C" moe_status moe_route_judged(const moe_cfg* cfg, const float* logits,
                                       const float* price_hat, float gap_tol, float* price,
                                       int32_t* topk_idx, float* topk_w, int32_t* load,
                                       int32_t* info, double* verdict, void* ws, size_t ws_bytes,
                                       void* stream) {
  return route_learned_impl(cfg, logits, price_hat, gap_tol, price, topk_idx, topk_w, load, info,
                            verdict, ws, ws_bytes, stream, true);
}

extern "C" moe_status moe_route_learned(const moe_cfg* cfg, const float* logits,
                                        const float* price_hat, float gap_tol, float* price,
                                        int32_t* topk_idx, float* topk_w, int32_t* load,
                                        int32_t* info, double* verdict, void* ws,
                                        size_t ws_bytes, void* stream) {
  return route_learned_impl(cfg, logits, price_hat, gap_tol, price, topk_idx, topk_w, load, info,
                            verdict, ws, ws_bytes, stream, false);
}
