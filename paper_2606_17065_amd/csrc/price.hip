// Batch statistics of router logits for the learned price (eight features
// per expert), the duality certificate of a routing, and the squared-error
// loss of predicted prices.
//
// moe_logit_stats data flow (one stream):
//   ls_rows      per token: k-th and (k+1)-th best score, and the expert
//                holding rank k (defines the plain top-k set at p = 0)
//   ls_cols      64-token x 64-expert tiles: margins m0, transposed sortable
//                keys of s and m0, per-tile FP64 column partials
//   ls_expert    per expert: fold the tile partials (fixed order), (C+1)-th
//                largest s and m0 by radix select
//   ls_features  global mean / std (fixed tree over experts), features
#include <math.h>

#include "common.h"
#include "internal.h"

namespace {

constexpr int LS_TILE = 64;
constexpr int NSTAT = 6;  // sum s, sum s^2, max s, sum m0, sum m0^2, load0

template <int L>
__device__ __forceinline__ void top_insert(uint32_t (&K)[L], int (&X)[L], uint32_t key, int e) {
  // sorted by (key descending, expert ascending).  An entry pushed down
  // the list can meet an equal key of a higher expert inserted after it,
  // so the expert index takes part in every comparison, not only the key.
#pragma unroll
  for (int j = 0; j < L; ++j) {
    const bool gt = key > K[j] || (key == K[j] && e < X[j]);
    const uint32_t hi = gt ? key : K[j], lo = gt ? K[j] : key;
    const int eh = gt ? e : X[j], el = gt ? X[j] : e;
    K[j] = hi;
    X[j] = eh;
    key = lo;
    e = el;
  }
}

// Top-L of experts [e_lo, e_hi) of one token's row, a_e = row[e] (- p[e]
// when PRICED), sorted by (key descending, expert ascending), experts
// inserted in ascending order.  The row is read 32 values at a time with
// in-bounds (clamped) addresses, so the loads of a batch are in flight
// together.
template <int L, bool PRICED>
__device__ __forceinline__ void row_top_range(const float* __restrict__ row, const float* p,
                                              int e_lo, int e_hi, uint32_t (&K)[L],
                                              int (&X)[L]) {
  for (int e0 = e_lo; e0 < e_hi; e0 += 32) {
    float v[32];
#pragma unroll
    for (int i = 0; i < 32; ++i) v[i] = row[min(e0 + i, e_hi - 1)];
#pragma unroll
    for (int i = 0; i < 32; ++i) {
      if (e0 + i < e_hi) {
        const float a = PRICED ? v[i] - p[e0 + i] : v[i];
        top_insert<L>(K, X, f32_key(a), e0 + i);
      }
    }
  }
}

// RS consecutive lanes share one token: each scans a contiguous range of
// the experts, then the lists are merged across the RS lanes (butterfly of
// exchanges, each inserting the partner's entries); every lane ends with
// the token's full list.  Entries compare by (key, expert), so the result
// is the same list a single in-order scan gives.  Call with every lane of
// the wavefront (the exchanges are cross-lane); inactive lanes pass an
// empty range.
constexpr int RS = 4;

template <int L, bool PRICED>
__device__ __forceinline__ void row_top_split(const float* __restrict__ row, const float* p,
                                              int E, int sub, bool active, uint32_t (&K)[L],
                                              int (&X)[L]) {
  const int chunk = (E + RS - 1) / RS;
  const int e_lo = min(E, sub * chunk), e_hi = min(E, e_lo + chunk);
  if (active && e_hi > e_lo) row_top_range<L, PRICED>(row, p, e_lo, e_hi, K, X);
#pragma unroll
  for (int o = 1; o < RS; o <<= 1) {
    uint32_t K2[L];
    int X2[L];
#pragma unroll
    for (int j = 0; j < L; ++j) {
      K2[j] = (uint32_t)__shfl_xor((int)K[j], o, 64);
      X2[j] = __shfl_xor(X[j], o, 64);
    }
#pragma unroll
    for (int j = 0; j < L; ++j) top_insert<L>(K, X, K2[j], X2[j]);
  }
}

// RS threads per token: the best k+1 experts at zero prices.
template <int L>
__global__ __launch_bounds__(256) void ls_rows(const float* __restrict__ s, int T, int E, int k,
                                               uint32_t* __restrict__ kkey,
                                               int32_t* __restrict__ kexp,
                                               float* __restrict__ kap) {
  const int g = blockIdx.x * 256 + threadIdx.x;
  const int t = g / RS, sub = g % RS;
  uint32_t K[L];
  int X[L];
#pragma unroll
  for (int j = 0; j < L; ++j) {
    K[j] = 0u;
    X[j] = E;
  }
  row_top_split<L, false>(s + (size_t)min(t, T - 1) * E, nullptr, E, sub, t < T, K, X);
  if (t >= T || sub != 0) return;
  uint32_t k1 = K[0], k2 = K[0];
  int e1 = X[0];
#pragma unroll
  for (int j = 0; j < L; ++j) {
    if (j == k - 1) {
      k1 = K[j];
      e1 = X[j];
    }
    if (j == k) k2 = K[j];
  }
  kkey[t] = k1;
  kexp[t] = e1;
  kap[2 * t] = key_f32(k1);
  kap[2 * t + 1] = key_f32(k2);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Block (token tile, 64-expert group), 256 threads = 4 waves; lane = token
// within the tile, wave w handles experts w, w+4, ...  FP64 partials per
// (tile, expert) are wave reductions in a fixed butterfly order.
__global__ __launch_bounds__(256) void ls_cols(const float* __restrict__ s, int T, int E,
                                               const uint32_t* __restrict__ kkey,
                                               const int32_t* __restrict__ kexp,
                                               const float* __restrict__ kap,
                                               uint32_t* __restrict__ sT, uint32_t* __restrict__ mT,
                                               double* __restrict__ part) {
  __shared__ float tile[LS_TILE][LS_TILE + 1];
  const int t0 = blockIdx.x * LS_TILE, e0 = blockIdx.y * LS_TILE, tid = threadIdx.x;
  for (int i = tid; i < LS_TILE * LS_TILE; i += 256) {
    const int tl = i >> 6, el = i & 63;
    const int t = t0 + tl, e = e0 + el;
    tile[tl][el] = (t < T && e < E) ? s[(size_t)t * E + e] : 0.0f;
  }
  __syncthreads();
  const int lane = tid & 63, wv = tid >> 6;
  const int t = t0 + lane;
  const bool valid = t < T;
  const uint32_t kk = valid ? kkey[t] : 0u;
  const int ke = valid ? kexp[t] : 0;
  const float kap1 = valid ? kap[2 * t] : 0.0f, kap2 = valid ? kap[2 * t + 1] : 0.0f;
  for (int el = wv; el < LS_TILE; el += 4) {
    const int e = e0 + el;
    if (e >= E) break;
    const float v = tile[lane][el];
    const uint32_t key = f32_key(v);
    const bool held = key > kk || (key == kk && e <= ke);
    const float m = v - (held ? kap2 : kap1);
    if (valid) {
      sT[(size_t)e * T + t] = key;
      mT[(size_t)e * T + t] = f32_key(m);
    }
    const double dv = valid ? (double)v : 0.0, dm = valid ? (double)m : 0.0;
    const double r0 = wave_sum(dv);
    const double r1 = wave_sum(dv * dv);
    const double r2 = wave_max(valid ? dv : -INFINITY);
    const double r3 = wave_sum(dm);
    const double r4 = wave_sum(dm * dm);
    const double r5 = wave_sum((valid && held) ? 1.0 : 0.0);
    if (lane == 0) {
      double* p = part + ((size_t)blockIdx.x * E + e) * NSTAT;
      p[0] = r0;
      p[1] = r1;
      p[2] = r2;
      p[3] = r3;
      p[4] = r4;
      p[5] = r5;
    }
  }
}

// r-th largest key (1-based, r <= n) of col[0..n) by four 8-bit radix
// passes; 1024 threads.  With KPT > 0 the column is loaded once into
// registers (n <= 1024 * KPT), otherwise it is re-read every pass.
// Wavefront aggregation: when every counted key of a wavefront falls in one
// bin (the usual case in the first passes, where the logits of a column
// share sign and exponent) one atomic adds them all.
__device__ __forceinline__ void hist_add(bool ok, uint32_t dg, int lane, int* hist) {
  const unsigned long long act = __ballot(ok);
  if (act == 0ull) return;
  const int first = __ffsll((long long)act) - 1;
  const uint32_t d0 = (uint32_t)__shfl((int)dg, first, 64);
  const unsigned long long same = __ballot(ok && dg == d0);
  if (same == act) {
    if (lane == first) atomicAdd(&hist[d0], __popcll(act));
  } else if (ok) {
    atomicAdd(&hist[dg], 1);
  }
}

template <int KPT>
__device__ uint32_t block_rth_key(const uint32_t* __restrict__ col, int n, int r, int* hist,
                                  int* sh) {
  const int tid = threadIdx.x, lane = tid & 63;
  constexpr int NT = 1024;
  uint32_t kk[KPT > 0 ? KPT : 1];
  if (KPT > 0) {
#pragma unroll
    for (int j = 0; j < KPT; ++j) {
      const int i = j * NT + tid;
      kk[j] = i < n ? col[i] : 0u;
    }
  }
  uint32_t prefix = 0u, mask = 0u;
  int need = r;
  for (int shift = 24; shift >= 0; shift -= 8) {
    for (int i = tid; i < 256; i += NT) hist[i] = 0;
    __syncthreads();
    if (KPT > 0) {
#pragma unroll
      for (int j = 0; j < KPT; ++j) {
        const int i = j * NT + tid;
        hist_add(i < n && (kk[j] & mask) == prefix, (kk[j] >> shift) & 255u, lane, hist);
      }
    } else {
      for (int i0 = 0; i0 < n; i0 += NT) {
        const int i = i0 + tid;
        const uint32_t key = i < n ? col[i] : 0u;
        hist_add(i < n && (key & mask) == prefix, (key >> shift) & 255u, lane, hist);
      }
    }
    __syncthreads();
    if (tid < 64) {
      // wavefront 0: lane l owns bins 4l..4l+3; suffix sums over the lanes
      // find the bin holding the need-th largest key
      int c[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) c[u] = hist[4 * tid + u];
      const int loc = c[0] + c[1] + c[2] + c[3];
      int suf = loc;
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const int o = __shfl_down(suf, off, 64);
        if (tid + off < 64) suf += o;
      }
      const int above = suf - loc;
      if (above < need && need <= suf) {
        int acc = above, dg = 4 * tid;
#pragma unroll
        for (int u = 3; u >= 0; --u) {
          if (acc + c[u] >= need) {
            dg = 4 * tid + u;
            break;
          }
          acc += c[u];
        }
        sh[0] = dg;
        sh[1] = need - acc;
      }
    }
    __syncthreads();
    prefix |= (uint32_t)sh[0] << shift;
    mask |= 255u << shift;
    need = sh[1];
    __syncthreads();
  }
  return prefix;
}

// One block per expert: fold the tile partials and select the (C+1)-th
// largest s and m0 of the expert's column.
__global__ __launch_bounds__(1024) void ls_expert(const uint32_t* __restrict__ sT,
                                                  const uint32_t* __restrict__ mT,
                                                  const double* __restrict__ part, int ntile,
                                                  int T, int E, int C, double* __restrict__ col,
                                                  float* __restrict__ q) {
  __shared__ int hist[256];
  __shared__ int sh[2];
  __shared__ double red[1024];
  const int e = blockIdx.x, tid = threadIdx.x;
  // each statistic: thread i folds tiles i, i+1024, ... in order, then a
  // fixed halving tree (deterministic, independent of scheduling)
  for (int st = 0; st < NSTAT; ++st) {
    double a = st == 2 ? -INFINITY : 0.0;
    for (int b = tid; b < ntile; b += 1024) {
      const double v = part[((size_t)b * E + e) * NSTAT + st];
      a = st == 2 ? fmax(a, v) : a + v;
    }
    red[tid] = a;
    __syncthreads();
    for (int h = 512; h >= 1; h >>= 1) {
      if (tid < h) red[tid] = st == 2 ? fmax(red[tid], red[tid + h]) : red[tid] + red[tid + h];
      __syncthreads();
    }
    if (tid == 0) col[e * NSTAT + st] = red[0];
    __syncthreads();
  }
  const int r = C + 1 < T ? C + 1 : T;
  uint32_t ks, km;
  if (T <= 1024 * 16) {
    ks = block_rth_key<16>(sT + (size_t)e * T, T, r, hist, sh);
    km = block_rth_key<16>(mT + (size_t)e * T, T, r, hist, sh);
  } else if (T <= 1024 * 64) {
    ks = block_rth_key<64>(sT + (size_t)e * T, T, r, hist, sh);
    km = block_rth_key<64>(mT + (size_t)e * T, T, r, hist, sh);
  } else {
    ks = block_rth_key<0>(sT + (size_t)e * T, T, r, hist, sh);
    km = block_rth_key<0>(mT + (size_t)e * T, T, r, hist, sh);
  }
  if (tid == 0) {
    q[2 * e] = key_f32(ks);
    q[2 * e + 1] = key_f32(km);
  }
}

// One block: global mean / std over all T*E logits (expert totals summed
// by a fixed tree), then the eight features of every expert.
__global__ __launch_bounds__(1024) void ls_features(const double* __restrict__ col,
                                                    const float* __restrict__ q, int T, int E,
                                                    int C, float* __restrict__ feats,
                                                    float* __restrict__ sigma_out) {
  __shared__ double g[2];
  __shared__ double r1[1024], r2[1024];
  const int tid = threadIdx.x;
  // expert sums by a fixed halving tree (E <= 1024)
  r1[tid] = tid < E ? col[tid * NSTAT + 0] : 0.0;
  r2[tid] = tid < E ? col[tid * NSTAT + 1] : 0.0;
  __syncthreads();
  for (int h = 512; h >= 1; h >>= 1) {
    if (tid < h) {
      r1[tid] = r1[tid] + r1[tid + h];
      r2[tid] = r2[tid] + r2[tid + h];
    }
    __syncthreads();
  }
  if (tid == 0) {
    const double s1 = r1[0], s2 = r2[0];
    const double n = (double)T * (double)E;
    const double mu = s1 / n;
    double var = s2 / n - mu * mu;
    var = var > 0.0 ? var : 0.0;
    double sg = sqrt(var);
    if (!(sg > 0.0)) sg = 1.0;
    g[0] = mu;
    g[1] = sg;
    if (sigma_out) sigma_out[0] = (float)sg;
  }
  __syncthreads();
  const double mu = g[0], sg = g[1], Tn = (double)T;
  for (int e = tid; e < E; e += blockDim.x) {
    const double* c = col + e * NSTAT;
    const double ms = c[0] / Tn, mm = c[3] / Tn;
    double vs = c[1] / Tn - ms * ms, vm = c[4] / Tn - mm * mm;
    vs = vs > 0.0 ? vs : 0.0;
    vm = vm > 0.0 ? vm : 0.0;
    float* f = feats + (size_t)e * 8;
    f[0] = (float)((ms - mu) / sg);
    f[1] = (float)(sqrt(vs) / sg);
    f[2] = (float)((c[2] - mu) / sg);
    f[3] = (float)(((double)q[2 * e] - mu) / sg);
    f[4] = (float)(c[5] / (double)C);
    f[5] = (float)(mm / sg);
    f[6] = (float)((double)q[2 * e + 1] / sg);
    f[7] = (float)(sqrt(vm) / sg);
  }
}

struct StatsWs {
  uint32_t *kkey, *sT, *mT;
  int32_t* kexp;
  float *kap, *q;
  double *part, *col;
};

StatsWs carve_stats(const moe_cfg& c, void* base, size_t* total) {
  WsCarve wc{(char*)base, 0};
  StatsWs w;
  const size_t T = (size_t)c.T, E = (size_t)c.E;
  const size_t ntile = (T + LS_TILE - 1) / LS_TILE;
  w.kkey = wc.take<uint32_t>(T);
  w.kexp = wc.take<int32_t>(T);
  w.kap = wc.take<float>(2 * T);
  w.sT = wc.take<uint32_t>(T * E);
  w.mT = wc.take<uint32_t>(T * E);
  w.part = wc.take<double>(ntile * E * NSTAT);
  w.col = wc.take<double>(E * NSTAT);
  w.q = wc.take<float>(2 * E);
  if (total) *total = align_up(wc.off, 256);
  return w;
}

// ------------------------------------------------------------ certificate
// Per token: primal term sum_j s[t, idx_j] and the dual term
// topk_sum(s_t - p) (FP64 values of the FP32 ranking); 256-token block
// partials, folded in block order by cert_final.

template <int L>
__global__ __launch_bounds__(256) void cert_tokens(const float* __restrict__ s,
                                                   const float* __restrict__ p,
                                                   const int32_t* __restrict__ idx, int T, int E,
                                                   int k, double* __restrict__ part) {
  __shared__ double sp[256], sd[256];
  __shared__ float ps[MOE_MAX_E];
  const int tid = threadIdx.x, t = blockIdx.x * (256 / RS) + tid / RS, sub = tid % RS;
  for (int e = tid; e < E; e += 256) ps[e] = p[e];
  __syncthreads();
  double prim = 0.0, dual = 0.0;
  uint32_t K[L];
  int X[L];
#pragma unroll
  for (int j = 0; j < L; ++j) {
    K[j] = 0u;
    X[j] = 0;
  }
  const float* row = s + (size_t)min(t, T - 1) * E;
  row_top_split<L, true>(row, ps, E, sub, t < T, K, X);
  if (t < T && sub == 0) {
#pragma unroll
    for (int j = 0; j < L; ++j)
      if (j < k) dual += (double)row[X[j]] - (double)p[X[j]];
    for (int j = 0; j < k; ++j) {
      const int e = idx[(size_t)t * k + j];
      prim += (e >= 0 && e < E) ? (double)row[e] : 0.0;
    }
  }
  sp[tid] = prim;
  sd[tid] = dual;
  __syncthreads();
  for (int h = 128; h >= 1; h >>= 1) {
    if (tid < h) {
      sp[tid] += sp[tid + h];
      sd[tid] += sd[tid + h];
    }
    __syncthreads();
  }
  if (tid == 0) {
    part[2 * blockIdx.x] = sp[0];
    part[2 * blockIdx.x + 1] = sd[0];
  }
}

// Fixed order: thread i folds block partials i, i + 256, ... in order, then
// the 256 sums are halved (stride 128..1); the prices are summed in order.
__global__ __launch_bounds__(256) void cert_final(const double* __restrict__ part, int nb,
                                                  const float* __restrict__ p, int E, int C,
                                                  double* __restrict__ cert) {
  __shared__ double sp[256], sd[256];
  const int tid = threadIdx.x;
  double a = 0.0, b = 0.0;
  for (int j = tid; j < nb; j += 256) {
    a += part[2 * j];
    b += part[2 * j + 1];
  }
  sp[tid] = a;
  sd[tid] = b;
  __syncthreads();
  for (int h = 128; h >= 1; h >>= 1) {
    if (tid < h) {
      sp[tid] += sp[tid + h];
      sd[tid] += sd[tid + h];
    }
    __syncthreads();
  }
  if (tid != 0) return;
  double prim = sp[0], dual = sd[0], ps = 0.0;
  for (int e = 0; e < E; ++e) ps += (double)p[e];
  dual += (double)C * ps;
  cert[0] = prim;
  cert[1] = dual;
  const double den = fabs(dual) > 0.0 ? fabs(dual) : 1.0;
  cert[2] = (dual - prim) / den;
}

// ------------------------------------------------------------------- mse
// loss = mean_r (phat_r - y_r)^2 with y_r = target_r / sigma[r / group];
// dphat_r = 2 (phat_r - y_r) / rows.  One block, fixed-order reduction.
__global__ __launch_bounds__(1024) void mse_kernel(int rows, int group,
                                                   const float* __restrict__ phat,
                                                   const float* __restrict__ target,
                                                   const float* __restrict__ sigma,
                                                   float* __restrict__ dphat,
                                                   float* __restrict__ loss) {
  __shared__ double red[1024];
  const int tid = threadIdx.x;
  double acc = 0.0;
  for (int r = tid; r < rows; r += 1024) {
    const float y = sigma ? target[r] / sigma[r / group] : target[r];
    const float d = phat[r] - y;
    acc += (double)d * (double)d;
    if (dphat) dphat[r] = 2.0f * d / (float)rows;
  }
  red[tid] = acc;
  __syncthreads();
  for (int h = 512; h >= 1; h >>= 1) {
    if (tid < h) red[tid] += red[tid + h];
    __syncthreads();
  }
  if (tid == 0 && loss) loss[0] = (float)(red[0] / (double)rows);
}

}  // namespace

size_t stats_ws_bytes(const moe_cfg& c) {
  size_t total = 0;
  carve_stats(c, nullptr, &total);
  return total;
}

size_t cert_ws_bytes(const moe_cfg& c) {
  return align_up(sizeof(double) * 2 * (((size_t)c.T + 63) / 64 + 1), 256);
}

extern "C" moe_status moe_logit_stats(const moe_cfg* cfg, const float* logits, float* feats,
                                      float* sigma, void* ws, size_t ws_bytes, void* stream) {
  moe_status stc = check_cfg_shape(cfg);
  if (stc != MOE_OK) return stc;
  const moe_cfg& c = *cfg;
  if (c.T < 1 || !logits || !feats) return MOE_EINVAL;
  if (c.k >= c.E) return MOE_EUNSUPPORTED;
  if (!aligned(logits, 4) || !aligned(feats, 4) || !aligned(sigma, 4)) return MOE_EINVAL;
  if (!ws || ws_bytes < stats_ws_bytes(c)) return MOE_EWORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  StatsWs w = carve_stats(c, ws, nullptr);
  const int L = c.k + 1;
  const dim3 gr((unsigned)(((size_t)c.T * RS + 255) / 256));
  if (L <= 3)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(ls_rows<3>), gr, dim3(256), 0, st, logits, c.T, c.E, c.k,
                       w.kkey, w.kexp, w.kap);
  else if (L <= 5)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(ls_rows<5>), gr, dim3(256), 0, st, logits, c.T, c.E, c.k,
                       w.kkey, w.kexp, w.kap);
  else if (L <= 9)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(ls_rows<9>), gr, dim3(256), 0, st, logits, c.T, c.E, c.k,
                       w.kkey, w.kexp, w.kap);
  else
    hipLaunchKernelGGL(HIP_KERNEL_NAME(ls_rows<17>), gr, dim3(256), 0, st, logits, c.T, c.E, c.k,
                       w.kkey, w.kexp, w.kap);
  const int ntile = (c.T + LS_TILE - 1) / LS_TILE;
  hipLaunchKernelGGL(ls_cols, dim3(ntile, (c.E + LS_TILE - 1) / LS_TILE), dim3(256), 0, st,
                     logits, c.T, c.E, w.kkey, w.kexp, w.kap, w.sT, w.mT, w.part);
  hipLaunchKernelGGL(ls_expert, dim3(c.E), dim3(1024), 0, st, w.sT, w.mT, w.part, ntile, c.T,
                     c.E, c.capacity, w.col, w.q);
  hipLaunchKernelGGL(ls_features, dim3(1), dim3(1024), 0, st, w.col, w.q, c.T, c.E, c.capacity,
                     feats, sigma);
  MOE_LAUNCH_CHECK();
  return MOE_OK;
}

extern "C" moe_status moe_route_certify(const moe_cfg* cfg, const float* logits,
                                        const float* price, const int32_t* topk_idx,
                                        double* cert, void* ws, size_t ws_bytes, void* stream) {
  moe_status stc = check_cfg_shape(cfg);
  if (stc != MOE_OK) return stc;
  const moe_cfg& c = *cfg;
  if (!price || !cert || (c.T > 0 && (!logits || !topk_idx))) return MOE_EINVAL;
  if (!aligned(logits, 4) || !aligned(price, 4) || !aligned(topk_idx, 4) || !aligned(cert, 8))
    return MOE_EINVAL;
  if (!ws || ws_bytes < cert_ws_bytes(c)) return MOE_EWORKSPACE;
  launch_certify(c, logits, price, topk_idx, (double*)ws, cert, stream);
  MOE_LAUNCH_CHECK();
  return MOE_OK;
}

void launch_certify(const moe_cfg& c, const float* logits, const float* price,
                    const int32_t* topk_idx, double* part, double* cert, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  const int nb = (c.T + 256 / RS - 1) / (256 / RS);  // 64 tokens per block
  if (nb > 0) {
    const int L = c.k;
    if (L <= 2)
      hipLaunchKernelGGL(HIP_KERNEL_NAME(cert_tokens<2>), dim3(nb), dim3(256), 0, st, logits,
                         price, topk_idx, c.T, c.E, c.k, part);
    else if (L <= 4)
      hipLaunchKernelGGL(HIP_KERNEL_NAME(cert_tokens<4>), dim3(nb), dim3(256), 0, st, logits,
                         price, topk_idx, c.T, c.E, c.k, part);
    else if (L <= 8)
      hipLaunchKernelGGL(HIP_KERNEL_NAME(cert_tokens<8>), dim3(nb), dim3(256), 0, st, logits,
                         price, topk_idx, c.T, c.E, c.k, part);
    else
      hipLaunchKernelGGL(HIP_KERNEL_NAME(cert_tokens<16>), dim3(nb), dim3(256), 0, st, logits,
                         price, topk_idx, c.T, c.E, c.k, part);
  }
  hipLaunchKernelGGL(cert_final, dim3(1), dim3(256), 0, st, part, nb, price, c.E, c.capacity,
                     cert);
}

extern "C" moe_status moe_price_mse(int rows, int group, const float* price_hat,
                                    const float* target, const float* sigma, float* dprice,
                                    float* loss, void* stream) {
  if (rows < 1 || group < 1 || !price_hat || !target) return MOE_EINVAL;
  if (!aligned(price_hat, 4) || !aligned(target, 4) || !aligned(sigma, 4) ||
      !aligned(dprice, 4) || !aligned(loss, 4))
    return MOE_EINVAL;
  hipLaunchKernelGGL(mse_kernel, dim3(1), dim3(1024), 0, (hipStream_t)stream, rows, group,
                     price_hat, target, sigma, dprice, loss);
  MOE_LAUNCH_CHECK();
  return MOE_OK;
}
