// Price MLP 8 -> 256 -> 256 -> 1 (exact-erf GELU after both hidden layers,
// softplus head), its backward and an Adam step, in FP32 on the GPU.
//
// The products are small (rows = experts x batches, widths 8 and 256), so
// they run on one FP32 SIMT tile kernel with arbitrary operand strides:
//   C(m, n) = sum_k A(m, k) B(n, k),  A(m,k) = A[m*sam + k*sak],
//                                     B(n,k) = B[n*sbn + k*sbk]
// Every reduction over rows (weight and bias gradients) is split into
// fixed row chunks whose partials are folded in chunk order, so results do
// not depend on scheduling.
#include <math.h>

#include "common.h"
#include "internal.h"

namespace {

constexpr int H = 256;
constexpr int NF = 8;
constexpr int OFF_W1 = 0;
constexpr int OFF_B1 = OFF_W1 + H * NF;
constexpr int OFF_W2 = OFF_B1 + H;
constexpr int OFF_B2 = OFF_W2 + H * H;
constexpr int OFF_W3 = OFF_B2 + H;
constexpr int OFF_B3 = OFF_W3 + H;
constexpr int NPARAM = OFF_B3 + 1;
constexpr int ROW_CHUNK = 256;  // rows per partial of a row reduction

__device__ __forceinline__ float gelu(float u) {
  return 0.5f * u * (1.0f + erff(u * 0.70710678118654752f));
}
__device__ __forceinline__ float gelu_grad(float u) {
  return 0.5f * (1.0f + erff(u * 0.70710678118654752f)) +
         u * expf(-0.5f * u * u) * 0.39894228040143268f;
}
__device__ __forceinline__ float softplus(float z) {
  return z > 20.0f ? z : log1pf(expf(z));
}
__device__ __forceinline__ float sigmoid(float z) { return 1.0f / (1.0f + expf(-z)); }

enum { EPI_STORE = 0, EPI_BIAS_GELU = 1, EPI_GELU_GRAD = 2 };

// 64x64 output tile per block, 256 threads with 4x4 outputs each, K in
// chunks of 16 staged through LDS.  blockIdx.z selects a K range of
// kchunk; EPI_STORE writes that range's partial to out + z*M*ldo.
template <int EPI>
__global__ __launch_bounds__(256) void mlp_gemm(const float* __restrict__ A, int sam, int sak,
                                                const float* __restrict__ B, int sbn, int sbk,
                                                int M, int N, int K, int kchunk,
                                                const float* __restrict__ bias,
                                                const float* __restrict__ aux,
                                                float* __restrict__ out, float* __restrict__ out2,
                                                int ldo) {
  __shared__ float As[16][68], Bs[16][68];
  const int tid = threadIdx.x;
  const int m0 = blockIdx.x * 64, n0 = blockIdx.y * 64;
  const int kb = blockIdx.z * kchunk, ke = min(K, kb + kchunk);
  const int tx = tid & 15, ty = tid >> 4;
  float acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0f;
  for (int k0 = kb; k0 < ke; k0 += 16) {
    for (int i = tid; i < 16 * 64; i += 256) {
      int ml, kl;
      if (sak == 1) {
        kl = i & 15;
        ml = i >> 4;
      } else {
        ml = i & 63;
        kl = i >> 6;
      }
      const int m = m0 + ml, kk = k0 + kl;
      As[kl][ml] = (m < M && kk < ke) ? A[(size_t)m * sam + (size_t)kk * sak] : 0.0f;
    }
    for (int i = tid; i < 16 * 64; i += 256) {
      int nl, kl;
      if (sbk == 1) {
        kl = i & 15;
        nl = i >> 4;
      } else {
        nl = i & 63;
        kl = i >> 6;
      }
      const int n = n0 + nl, kk = k0 + kl;
      Bs[kl][nl] = (n < N && kk < ke) ? B[(size_t)n * sbn + (size_t)kk * sbk] : 0.0f;
    }
    __syncthreads();
#pragma unroll
    for (int kl = 0; kl < 16; ++kl) {
      float a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kl][ty * 4 + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[kl][tx * 4 + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
  float* o = out + (EPI == EPI_STORE ? (size_t)blockIdx.z * M * ldo : 0);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int m = m0 + ty * 4 + i;
    if (m >= M) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int n = n0 + tx * 4 + j;
      if (n >= N) continue;
      const size_t at = (size_t)m * ldo + n;
      if (EPI == EPI_STORE) {
        o[at] = acc[i][j];
      } else if (EPI == EPI_BIAS_GELU) {
        const float u = acc[i][j] + bias[n];
        o[at] = u;
        out2[at] = gelu(u);
      } else {
        o[at] = acc[i][j] * gelu_grad(aux[at]);
      }
    }
  }
}

// out[i] = sum over z of part[z*count + i], z ascending.
__global__ __launch_bounds__(256) void fold_splits(const float* __restrict__ part, int nsplit,
                                                   int count, float* __restrict__ out) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= count) return;
  float a = 0.0f;
  for (int z = 0; z < nsplit; ++z) a += part[(size_t)z * count + i];
  out[i] = a;
}

// part[split*N + n] = sum over rows r of the split (ascending) of
// X[r*N + n] * (w ? w[r] : 1).
__global__ __launch_bounds__(256) void col_partials(const float* __restrict__ X,
                                                    const float* __restrict__ w, int R, int N,
                                                    float* __restrict__ part) {
  const int n = blockIdx.x * 256 + threadIdx.x, sp = blockIdx.y;
  if (n >= N) return;
  const int r0 = sp * ROW_CHUNK, r1 = min(R, r0 + ROW_CHUNK);
  float a = 0.0f;
  for (int r = r0; r < r1; ++r) {
    const float x = X[(size_t)r * N + n];
    a = w ? fmaf(x, w[r], a) : a + x;
  }
  part[(size_t)sp * N + n] = a;
}

__device__ __forceinline__ float wave_sum_f(float v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// One wave per row: z = a2 . w3 + b3; phat = sigma * softplus(z).
__global__ __launch_bounds__(256) void head_fwd(const float* __restrict__ a2,
                                                const float* __restrict__ params, int R,
                                                const float* __restrict__ sigma,
                                                float* __restrict__ z_out,
                                                float* __restrict__ phat) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (row >= R) return;
  const float* a = a2 + (size_t)row * H;
  const float* w3 = params + OFF_W3;
  float acc = 0.0f;
#pragma unroll
  for (int i = 0; i < H / 64; ++i) acc = fmaf(a[i * 64 + lane], w3[i * 64 + lane], acc);
  acc = wave_sum_f(acc);
  if (lane == 0) {
    const float z = acc + params[OFF_B3];
    z_out[row] = z;
    phat[row] = (sigma ? sigma[0] : 1.0f) * softplus(z);
  }
}

// One wave per row: dz = dphat * sigma * sigmoid(z); du2 = dz w3 gelu'(u2).
__global__ __launch_bounds__(256) void head_bwd(const float* __restrict__ dphat,
                                                const float* __restrict__ z,
                                                const float* __restrict__ sigma,
                                                const float* __restrict__ params,
                                                const float* __restrict__ u2, int R,
                                                float* __restrict__ dz_out,
                                                float* __restrict__ du2) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (row >= R) return;
  const float dz = dphat[row] * (sigma ? sigma[0] : 1.0f) * sigmoid(z[row]);
  if (lane == 0) dz_out[row] = dz;
  const float* w3 = params + OFF_W3;
#pragma unroll
  for (int i = 0; i < H / 64; ++i) {
    const int j = i * 64 + lane;
    du2[(size_t)row * H + j] = dz * w3[j] * gelu_grad(u2[(size_t)row * H + j]);
  }
}

__global__ __launch_bounds__(256) void adam_kernel(int n, float* __restrict__ p,
                                                   const float* __restrict__ g,
                                                   float* __restrict__ m, float* __restrict__ v,
                                                   float lr, float b1, float b2, float eps,
                                                   float c1, float c2) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float mh = mi / c1, vh = vi / c2;
  p[i] = p[i] - lr * mh / (sqrtf(vh) + eps);
}

struct MlpActs {
  float *u1, *a1, *u2, *a2, *z;
};

MlpActs acts_of(float* acts, int R) {
  MlpActs a;
  const size_t RH = (size_t)R * H;
  a.u1 = acts;
  a.a1 = acts + RH;
  a.u2 = acts + 2 * RH;
  a.a2 = acts + 3 * RH;
  a.z = acts + 4 * RH;
  return a;
}

int nsplit_of(int R) { return (R + ROW_CHUNK - 1) / ROW_CHUNK; }

struct MlpBwdWs {
  float *dz, *du2, *du1, *part;
};

MlpBwdWs carve_mlp(int R, void* base, size_t* total) {
  WsCarve wc{(char*)base, 0};
  MlpBwdWs w;
  const size_t RH = (size_t)R * H;
  w.dz = wc.take<float>((size_t)R);
  w.du2 = wc.take<float>(RH);
  w.du1 = wc.take<float>(RH);
  w.part = wc.take<float>((size_t)nsplit_of(R) * H * H);
  if (total) *total = align_up(wc.off, 256);
  return w;
}

void gemm(int epi, const float* A, int sam, int sak, const float* B, int sbn, int sbk, int M,
          int N, int K, int kchunk, const float* bias, const float* aux, float* out, float* out2,
          int ldo, hipStream_t st) {
  const dim3 g((M + 63) / 64, (N + 63) / 64, (K + kchunk - 1) / kchunk);
  if (epi == EPI_STORE)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(mlp_gemm<EPI_STORE>), g, dim3(256), 0, st, A, sam, sak, B,
                       sbn, sbk, M, N, K, kchunk, bias, aux, out, out2, ldo);
  else if (epi == EPI_BIAS_GELU)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(mlp_gemm<EPI_BIAS_GELU>), g, dim3(256), 0, st, A, sam, sak,
                       B, sbn, sbk, M, N, K, kchunk, bias, aux, out, out2, ldo);
  else
    hipLaunchKernelGGL(HIP_KERNEL_NAME(mlp_gemm<EPI_GELU_GRAD>), g, dim3(256), 0, st, A, sam, sak,
                       B, sbn, sbk, M, N, K, kchunk, bias, aux, out, out2, ldo);
}

// Sum over rows (chunked, chunk order) of X[R,N] (optionally weighted).
void row_sum(const float* X, const float* w, int R, int N, float* part, float* out,
             hipStream_t st) {
  const int ns = nsplit_of(R);
  hipLaunchKernelGGL(col_partials, dim3((N + 255) / 256, ns), dim3(256), 0, st, X, w, R, N, part);
  hipLaunchKernelGGL(fold_splits, dim3((N + 255) / 256), dim3(256), 0, st, part, ns, N, out);
}

}  // namespace

extern "C" moe_status moe_price_mlp_sizes(int rows, int32_t* n_params, size_t* acts_floats,
                                          size_t* ws_bytes) {
  if (rows < 0) return MOE_EINVAL;
  if (n_params) *n_params = NPARAM;
  if (acts_floats) *acts_floats = (size_t)rows * (4 * H + 1);
  if (ws_bytes) carve_mlp(rows, nullptr, ws_bytes);
  return MOE_OK;
}

extern "C" moe_status moe_price_mlp_forward(int rows, const float* feats, const float* params,
                                            const float* sigma, float* price_hat, float* acts,
                                            void* stream) {
  if (rows < 0 || (rows > 0 && (!feats || !params || !price_hat || !acts))) return MOE_EINVAL;
  if (!aligned(feats, 4) || !aligned(params, 4) || !aligned(sigma, 4) ||
      !aligned(price_hat, 4) || !aligned(acts, 4))
    return MOE_EINVAL;
  if (rows == 0) return MOE_OK;
  hipStream_t st = (hipStream_t)stream;
  MlpActs a = acts_of(acts, rows);
  gemm(EPI_BIAS_GELU, feats, NF, 1, params + OFF_W1, NF, 1, rows, H, NF, NF, params + OFF_B1,
       nullptr, a.u1, a.a1, H, st);
  gemm(EPI_BIAS_GELU, a.a1, H, 1, params + OFF_W2, H, 1, rows, H, H, H, params + OFF_B2, nullptr,
       a.u2, a.a2, H, st);
  hipLaunchKernelGGL(head_fwd, dim3((rows + 3) / 4), dim3(256), 0, st, a.a2, params, rows, sigma,
                     a.z, price_hat);
  MOE_LAUNCH_CHECK();
  return MOE_OK;
}

extern "C" moe_status moe_price_mlp_backward(int rows, const float* feats, const float* params,
                                             const float* sigma, const float* acts,
                                             const float* dprice, float* dparams, void* ws,
                                             size_t ws_bytes, void* stream) {
  if (rows < 1 || !feats || !params || !acts || !dprice || !dparams) return MOE_EINVAL;
  if (!aligned(feats, 4) || !aligned(params, 4) || !aligned(sigma, 4) || !aligned(acts, 4) ||
      !aligned(dprice, 4) || !aligned(dparams, 4))
    return MOE_EINVAL;
  size_t need = 0;
  carve_mlp(rows, nullptr, &need);
  if (!ws || ws_bytes < need) return MOE_EWORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  MlpActs a = acts_of(const_cast<float*>(acts), rows);
  MlpBwdWs w = carve_mlp(rows, ws, nullptr);
  const int ns = nsplit_of(rows);
  hipLaunchKernelGGL(head_bwd, dim3((rows + 3) / 4), dim3(256), 0, st, dprice, a.z, sigma, params,
                     a.u2, rows, w.dz, w.du2);
  // w3: sum_r dz_r a2[r];  b3: sum_r dz_r;  b2: sum_r du2[r]
  row_sum(a.a2, w.dz, rows, H, w.part, dparams + OFF_W3, st);
  row_sum(w.dz, nullptr, rows, 1, w.part, dparams + OFF_B3, st);
  row_sum(w.du2, nullptr, rows, H, w.part, dparams + OFF_B2, st);
  // W2[j,i] = sum_r du2[r,j] a1[r,i]   (K = rows, split by ROW_CHUNK)
  gemm(EPI_STORE, w.du2, 1, H, a.a1, 1, H, H, H, rows, ROW_CHUNK, nullptr, nullptr, w.part,
       nullptr, H, st);
  hipLaunchKernelGGL(fold_splits, dim3(H * H / 256), dim3(256), 0, st, w.part, ns, H * H,
                     dparams + OFF_W2);
  // du1 = (du2 W2) * gelu'(u1)
  gemm(EPI_GELU_GRAD, w.du2, H, 1, params + OFF_W2, 1, H, rows, H, H, H, nullptr, a.u1, w.du1,
       nullptr, H, st);
  row_sum(w.du1, nullptr, rows, H, w.part, dparams + OFF_B1, st);
  // W1[j,c] = sum_r du1[r,j] F[r,c]
  gemm(EPI_STORE, w.du1, 1, H, feats, 1, NF, H, NF, rows, ROW_CHUNK, nullptr, nullptr, w.part,
       nullptr, NF, st);
  hipLaunchKernelGGL(fold_splits, dim3((H * NF + 255) / 256), dim3(256), 0, st, w.part, ns,
                     H * NF, dparams + OFF_W1);
  MOE_LAUNCH_CHECK();
  return MOE_OK;
}

extern "C" moe_status moe_adam_step(int n, float* params, const float* grads, float* m, float* v,
                                    float lr, float beta1, float beta2, float eps, int step,
                                    void* stream) {
  if (n < 0 || step < 1 || (n > 0 && (!params || !grads || !m || !v))) return MOE_EINVAL;
  if (!(beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f && beta2 < 1.0f)) return MOE_EINVAL;
  if (!aligned(params, 4) || !aligned(grads, 4) || !aligned(m, 4) || !aligned(v, 4))
    return MOE_EINVAL;
  if (n == 0) return MOE_OK;
  const float c1 = (float)(1.0 - pow((double)beta1, (double)step));
  const float c2 = (float)(1.0 - pow((double)beta2, (double)step));
  hipLaunchKernelGGL(adam_kernel, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream, n,
                     params, grads, m, v, lr, beta1, beta2, eps, c1, c2);
  MOE_LAUNCH_CHECK();
  return MOE_OK;
}
