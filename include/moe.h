/*
 * moe.h -- C ABI of the MI355X (gfx950) mixture-of-experts layer library.
 *
 * The paper this library accompanies defines no mixture-of-experts layer,
 * so no passage of it can be cited for these calls.  Each entry point
 * states the definition it implements instead.  Shared definitions:
 *
 *   T tokens of width d, E experts, top-k, SwiGLU width f = d_ff,
 *   capacity C tokens per expert, N = T*k slots.
 *
 *   Routing problem: scores s[T,E] (FP32 router logits); choose k distinct
 *   experts per token maximising the summed scores with no expert above C
 *   tokens.  Capacity prices p[E] >= 0 are the LP dual variables of the
 *   capacity rows; given p, every token takes its top-k of a = s - p.
 *
 *   Sortable key of an FP32 value with bit pattern u: ~u if the sign bit is
 *   set, else u | 0x80000000; ranking is by key descending, ties to the
 *   lower expert index (token side) or the lower token index (expert side).
 *
 *   Slot order: slots are sorted by expert, then by token ascending.
 *
 * Conventions for every call:
 *   - every pointer argument is a caller-owned DEVICE pointer unless marked
 *     "host"; tensors are dense and row-major; pointers must be 16-byte
 *     aligned; the library never allocates device memory and never
 *     synchronises the device;
 *   - ``stream`` is a hipStream_t (NULL = the legacy default stream); all
 *     work is enqueued on it;
 *   - a call validates its arguments on the host and returns a negative
 *     moe_status without launching anything if they are bad; problems only
 *     the device can see (a non-finite logit, a failed capacity repair) are
 *     written to the device ``info`` array of moe_route;
 *   - ``ws`` is a device workspace of at least moe_workspace_bytes() bytes;
 *     it holds no state between calls, so one buffer can serve every call
 *     issued in order on one stream;
 *   - dtype codes: activations (X, X_perm, h, Y, out and their gradients)
 *     are MOE_F32 or MOE_BF16 (cfg.act); expert weights are MOE_F32,
 *     MOE_BF16 or MOE_FP8E4M3 (cfg.w).  The router (W_r, b_r, logits,
 *     prices) is always FP32.
 */
#ifndef MOE_H
#define MOE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MOE_OK = 0,
  MOE_EINVAL = -1,       /* bad pointer, size, alignment or enum value */
  MOE_EINFEASIBLE = -2,  /* k > E or E*C < T*k: no routing can exist */
  MOE_EUNSUPPORTED = -3, /* valid but unsupported shape / dtype combination */
  MOE_EWORKSPACE = -4,   /* workspace smaller than moe_workspace_bytes() */
  MOE_EHIP = -5,         /* a HIP launch failed */
  MOE_ENAN = -6,         /* (device, info[3]) a router logit is not finite */
  MOE_ECAPACITY = -7     /* (device, info[3]) capacity repair placed no slot */
} moe_status;

typedef enum {
  MOE_F32 = 0,
  MOE_BF16 = 1,
  MOE_FP8E4M3 = 2,   /* e4m3 codes with FP32 scales per 1x128 / 128x128 block */
  MOE_MXFP8E4M3 = 3, /* OCP MX: e4m3 codes, E8M0 scale per 32 along K        */
  MOE_MXFP6E2M3 = 4, /* OCP MX: e2m3 codes, E8M0 scale per 32 along K        */
  MOE_MXFP4E2M1 = 5  /* OCP MX: e2m1 codes, E8M0 scale per 32 along K        */
} moe_dtype;

typedef enum {
  MOE_PRICE_NONE = 0,  /* p = 0: plain top-k (then capacity repair)        */
  MOE_PRICE_ACP = 1,   /* ascending clearing price from p = 0              */
  MOE_PRICE_GIVEN = 2, /* p = price[] as passed, no update                  */
  MOE_PRICE_WARM = 3,  /* ascending clearing price from p = warm_gamma*price */
  MOE_PRICE_SUBGRAD = 4 /* projected dual subgradient from p = 0            */
} moe_price_mode;

typedef struct {
  int32_t T, d, E, k, d_ff;
  int32_t capacity;   /* C */
  int32_t max_iters;  /* cap on price updates (MOE_PRICE_ACP / _WARM / _SUBGRAD) */
  int32_t act;        /* moe_dtype of activations: MOE_F32 or MOE_BF16 */
  int32_t w;          /* moe_dtype of expert weights */
  int32_t price_mode; /* moe_price_mode */
  float warm_gamma;   /* MOE_PRICE_WARM scale of the given prices */
  int32_t price_stages; /* epsilon-scaled restarts after the ascending update (0..8; 0 = none) */
} moe_cfg;

/* info[] layout written by moe_route (device int32[8]). */
enum {
  MOE_INFO_ITERS = 0,     /* price updates performed */
  MOE_INFO_CONVERGED = 1, /* 1 if the last ranking respected every capacity */
  MOE_INFO_OVERFLOW = 2,  /* sum_e max(0, load_e - C) before capacity repair */
  MOE_INFO_STATUS = 3,    /* MOE_OK, MOE_ENAN or MOE_ECAPACITY */
  MOE_INFO_ROUNDS = 4,    /* proposal rounds of the capacity repair */
  MOE_INFO_SIGMA = 5,     /* bits of the FP32 score std sigma_s */
  MOE_INFO_EPS = 6,       /* bits of the FP32 bid increment eps */
  MOE_INFO_REPAIRED = 7   /* 1 if the capacity repair ran */
};
#define MOE_INFO_LEN 8

/* Bytes of workspace every call below needs for this configuration. */
moe_status moe_workspace_bytes(const moe_cfg* cfg /* host */, size_t* bytes /* host out */);

/*
 * moe_route -- router logits, capacity prices and capacity-aware top-k.
 *
 *   logits = X W_r^T + b_r                              (FP32 accumulate)
 *   sigma_s = population std of all logits (fixed-order FP64 reduction,
 *             rounded to FP32); eps = fl32(fl32(1e-3) * sigma_s)
 *   price update (MOE_PRICE_ACP / _WARM), all FP32, one rounding per op:
 *     repeat: a = s - p; rank every token's experts; S_t = best k,
 *       kappa1_t / kappa2_t = a at ranks k / k+1; load_e = #{t: e in S_t};
 *       stop if every load_e <= C or after max_iters updates; for each
 *       overloaded e, q = (C+1)-th largest of the margins
 *       m_t = s_te - (e in S_t ? kappa2_t : kappa1_t) and
 *       p_e = max(p_e, nextafter(q, +inf) + eps).
 *   projected dual subgradient (price-rule variant, MOE_PRICE_SUBGRAD):
 *     the same ranking and stop test; the update moves every price along
 *     the negative subgradient of the dual, C - load_e, scaled by the
 *     capacity and projected onto p >= 0:
 *       eta = fl32(eta0 / fl32(sqrt(fl32(u + 1)))), eta0 = fl32(256 * eps),
 *       g_e = fl32(fl32(load_e - C) / fl32(C)), x = fl32(p_e + fl32(eta g_e)),
 *       p_e = x > 0 ? x : +0                  (u = updates so far)
 *     It can stop at max_iters with an expert over capacity (the repair
 *     then places the overflow); cfg.price_stages does not apply.
 *   epsilon-scaled restarts (price-rule variant, cfg.price_stages = R > 0,
 *     with max_iters > 0): after the update, while it ended converged with
 *     some expert priced above zero and loaded below C (a nonzero
 *     certificate gap) and fewer than R restarts have run: p_e =
 *     max(+0, fl32(p_e - fl32(4 eps))) for every e, eps = fl32(eps / 8), and
 *     the update runs again from those prices (at most max_iters updates per
 *     run).  info reports the updates summed over the runs and the eps of
 *     the last run.  R = 0 is the plain update.
 *   routing: topk_idx[t, 0..k-1] = S_t in rank order (best first);
 *     topk_w[t, j] = softmax over the k chosen experts of the raw logits.
 *   If the final ranking still overloads an expert, a capacity repair runs:
 *     each overloaded expert keeps its C best holders by (key(a) desc,
 *     token asc); in rounds, each short token proposes to its best untried
 *     unheld experts and each expert accepts proposals in (key(a) desc,
 *     token asc) order while it has room.
 *
 *   X       [T,d] cfg.act          Wr [E,d] f32       br [E] f32
 *   logits  [T,E] f32 out          price [E] f32 in/out (final p)
 *   topk_idx[T,k] i32 out          topk_w [T,k] f32 out
 *   load    [E] i32 out (final loads)
 *   info    [MOE_INFO_LEN] i32 out (see MOE_INFO_*)
 */
moe_status moe_route(const moe_cfg* cfg, const void* X, const float* Wr, const float* br,
                     float* logits, float* price, int32_t* topk_idx, float* topk_w,
                     int32_t* load, int32_t* info, void* ws, size_t ws_bytes, void* stream);

/*
 * moe_router_logits -- the router alone: logits [T,E] f32 out = X W_r^T +
 *   b_r, computed exactly as moe_route computes them (same kernels, same
 *   bits).  For callers that route from these logits themselves (learned
 *   prices: moe_logit_stats, the price network, moe_route_judged).  X, Wr,
 *   br as in moe_route; ws at least moe_workspace_bytes(cfg).
 */
moe_status moe_router_logits(const moe_cfg* cfg, const void* X, const float* Wr, const float* br,
                             float* logits, void* ws, size_t ws_bytes, void* stream);

/*
 * moe_route_logits -- moe_route for caller-supplied logits: the same
 *   sigma_s, price update (cfg.price_mode), top-k, weights, capacity repair
 *   and info[], starting from logits [T,E] f32 (read only) instead of
 *   computing them.  cfg.d, cfg.d_ff, cfg.act and cfg.w are validated as for
 *   moe_route but not used.  Other arguments as in moe_route.
 */
moe_status moe_route_logits(const moe_cfg* cfg, const float* logits, float* price,
                            int32_t* topk_idx, float* topk_w, int32_t* load, int32_t* info,
                            void* ws, size_t ws_bytes, void* stream);

/*
 * moe_price_update -- the capacity-price update alone (the ascending
 *   clearing-price iteration of moe_route, its sigma_s and eps, in
 *   cfg.price_mode), from caller-supplied logits [T,E] f32 (read only):
 *   price [E] f32 in/out receives the final prices and info
 *   [MOE_INFO_LEN] i32 the iteration count, convergence flag, overflow of
 *   the final ranking and status, exactly as moe_route_logits reports them
 *   for the same inputs.  The routing the update ends with is kept in the
 *   workspace and not returned.  ws: at least moe_workspace_bytes(cfg)
 *   (MOE_EWORKSPACE otherwise).  Other arguments as in moe_route.
 */
moe_status moe_price_update(const moe_cfg* cfg, const float* logits, float* price, int32_t* info,
                            void* ws, size_t ws_bytes, void* stream);

/*
 * moe_route_certify -- duality certificate of a routing under prices p:
 *   cert[0] = primal  sum_t sum_j s[t, topk_idx[t,j]]
 *   cert[1] = dual    D(p) = C sum_e p_e + sum_t (sum of the k largest
 *                     s_te - p_e over e; ranking by the FP32 key)
 *   cert[2] = (dual - primal) / |dual|   (|dual| = 0 is taken as 1)
 *   FP64, fixed-order sums.  For any feasible routing, primal <= optimum <=
 *   dual; when topk_idx is the top-k under p the gap equals
 *   sum_e p_e (C - load_e).  logits [T,E] f32; price [E] f32; topk_idx
 *   [T,k] i32; cert [3] f64 out (8-byte aligned).  Uses ws (any buffer of
 *   moe_workspace_bytes).
 */
moe_status moe_route_certify(const moe_cfg* cfg, const float* logits, const float* price,
                             const int32_t* topk_idx, double* cert, void* ws, size_t ws_bytes,
                             void* stream);

/*
 * moe_route_judged -- routing from learned prices p_hat with the exact
 *   update as judge and fallback, all on the device (no host wait):
 *   1) learned pass, cfg.price_mode MOE_PRICE_WARM (p0 = fl32(warm_gamma *
 *      p_hat), then the clearing-price update of moe_route_logits, at most
 *      cfg.max_iters updates) or MOE_PRICE_GIVEN (p = p_hat, no update; the
 *      capacity repair of moe_route places any overflow);
 *   2) judge: the certificate of moe_route_certify for that routing under
 *      its prices; the routing is kept when its status is MOE_OK and the
 *      relative gap (dual - primal) / |dual| is at most gap_tol (weak
 *      duality makes the gap valid for any routing within capacity,
 *      repaired ones included);
 *   3) otherwise the batch is routed again by the update from p = 0 (as
 *      moe_route_logits in MOE_PRICE_ACP with cfg.max_iters), whose
 *      routing is returned.
 *   logits [T,E] f32; price_hat [E] f32 (read only); gap_tol >= 0 (finite);
 *   price, topk_idx, topk_w, load, info as moe_route_logits writes them for
 *   the routing returned; verdict [5] f64 out (8-byte aligned):
 *     verdict[0] = V = sum_e max(0, load_e - C) / N of the learned routing
 *                  before any repair,
 *     verdict[1] = relative gap of the learned routing (NaN if it failed),
 *     verdict[2] = 1 if the learned routing was kept, 0 if routed again,
 *     verdict[3] = relative gap of the routing returned,
 *     verdict[4] = price updates of the learned pass.
 *   A non-finite logit ends both passes with MOE_ENAN in info (verdict[2]
 *   = 0, gaps NaN).  cfg.price_mode other than WARM or GIVEN: MOE_EINVAL.
 *   ws: at least moe_workspace_bytes(cfg).  The fallback pass is always
 *   enqueued; when the learned routing is kept each of its kernels returns
 *   at once.
 */
moe_status moe_route_judged(const moe_cfg* cfg, const float* logits, const float* price_hat,
                            float gap_tol, float* price, int32_t* topk_idx, float* topk_w,
                            int32_t* load, int32_t* info, double* verdict, void* ws,
                            size_t ws_bytes, void* stream);

/*
 * moe_route_learned -- steps 1) and 2) of moe_route_judged without the
 *   device fallback: the learned routing, its certificate and the verdict
 *   (verdict[2] = 1 if the judge keeps it, verdict[3] = its relative gap),
 *   leaving the routing in the outputs either way.  For callers that read
 *   the verdict and route again themselves only when it is 0 (one host
 *   wait instead of the always-enqueued fallback pass).  Arguments as in
 *   moe_route_judged.
 */
moe_status moe_route_learned(const moe_cfg* cfg, const float* logits, const float* price_hat,
                             float gap_tol, float* price, int32_t* topk_idx, float* topk_w,
                             int32_t* load, int32_t* info, double* verdict, void* ws,
                             size_t ws_bytes, void* stream);

/*
 * Learned starting prices.  Eight statistics of a batch of logits per
 * expert feed a small network shared by all experts whose output,
 * p_hat_e = sigma * softplus(z_e), predicts the prices the clearing-price
 * update reaches; it is used as a warm start (MOE_PRICE_WARM: p0 =
 * warm_gamma * p_hat) or alone (MOE_PRICE_GIVEN), with moe_route_certify
 * judging the result.
 *
 * moe_logit_stats -- features [E,8] f32 out of logits [T,E] f32.  With mu,
 *   sigma the mean and population std of all T*E logits (FP64, fixed
 *   order), load0 the plain top-k loads at p = 0, kappa1_t / kappa2_t the
 *   k-th / (k+1)-th largest logit of token t, margins
 *   m0_te = fl32(s_te - (e in top-k of t ? kappa2_t : kappa1_t)), and
 *   q(v) = the (C+1)-th largest of a column v (its minimum when T <= C):
 *     f0 = (mean_t s_te - mu)/sigma     f1 = std_t s_te / sigma
 *     f2 = (max_t s_te - mu)/sigma      f3 = (q(s_.e) - mu)/sigma
 *     f4 = load0_e / C                  f5 = mean_t m0_te / sigma
 *     f6 = q(m0_.e) / sigma             f7 = std_t m0_te / sigma
 *   sigma [1] f32 out (may be NULL).  Requires T >= 1 (MOE_EINVAL) and
 *   k < E (MOE_EUNSUPPORTED).  Logits must be finite.
 */
moe_status moe_logit_stats(const moe_cfg* cfg, const float* logits, float* feats, float* sigma,
                           void* ws, size_t ws_bytes, void* stream);

/*
 * Price network parameters: one f32 vector of n_params values laid out as
 *   W1 [256,8], b1 [256], W2 [256,256], b2 [256], w3 [256], b3 [1];
 *   u1 = F W1^T + b1, a1 = gelu(u1), u2 = a1 W2^T + b2, a2 = gelu(u2),
 *   z = a2 w3 + b3, p_hat = sigma * softplus(z),
 *   gelu(u) = u/2 (1 + erf(u / sqrt 2)).
 * moe_price_mlp_sizes (host outs, each may be NULL): n_params, the floats
 *   of the activation buffer and the backward workspace bytes for `rows`.
 */
moe_status moe_price_mlp_sizes(int rows, int32_t* n_params /* host out */,
                               size_t* acts_floats /* host out */,
                               size_t* bwd_ws_bytes /* host out */);

/*
 * moe_price_mlp_forward -- p_hat [rows] f32 out for features [rows,8] f32.
 *   sigma: device f32 scalar, or NULL for 1.  acts [acts_floats] f32 out:
 *   u1, a1, u2, a2 ([rows,256] each) and z [rows], kept for the backward.
 */
moe_status moe_price_mlp_forward(int rows, const float* feats, const float* params,
                                 const float* sigma, float* price_hat, float* acts, void* stream);

/*
 * moe_price_mlp_backward -- dparams [n_params] f32 out = the gradient of a
 *   loss whose derivative with respect to p_hat is dprice [rows], through
 *   the forward whose activations are in acts.  Row sums are taken in
 *   fixed 256-row chunks folded in order.  ws: bwd_ws_bytes.
 */
moe_status moe_price_mlp_backward(int rows, const float* feats, const float* params,
                                  const float* sigma, const float* acts, const float* dprice,
                                  float* dparams, void* ws, size_t ws_bytes, void* stream);

/*
 * moe_price_mse -- loss [1] = mean_r (price_hat_r - y_r)^2 with
 *   y_r = target_r / sigma[r / group] (sigma may be NULL: y = target), and
 *   dprice [rows] = 2 (price_hat_r - y_r) / rows (may be NULL).
 */
moe_status moe_price_mse(int rows, int group, const float* price_hat, const float* target,
                         const float* sigma, float* dprice, float* loss, void* stream);

/*
 * moe_adam_step -- Adam with bias correction, in place, f32:
 *   m = b1 m + (1-b1) g;  v = b2 v + (1-b2) g^2;
 *   params -= lr (m / (1-b1^step)) / (sqrt(v / (1-b2^step)) + eps).
 *   step >= 1 counts updates; 0 <= b1, b2 < 1.
 */
moe_status moe_adam_step(int n, float* params, const float* grads, float* m, float* v, float lr,
                         float beta1, float beta2, float eps, int step, void* stream);

/*
 * moe_dispatch -- histogram / prefix-scan permute of the tokens into slots.
 *   offsets[e] = first slot of expert e (exclusive scan of the loads),
 *   offsets[E] = N; row_map[slot] = token of the slot; inv_map[t, j] = slot
 *   of (t, topk_idx[t, j]); X_perm[slot] = X[row_map[slot]].
 *   X [T,d] act; topk_idx [T,k] i32; offsets [E+1] i32 out;
 *   row_map [N] i32 out; inv_map [T,k] i32 out; X_perm [N,d] act out.
 *   FP8 experts (cfg.w == MOE_FP8E4M3, d % 128 == 0): every token row is
 *   quantised per 1 x 128 block as moe_quantize_fp8 does and X_perm [N,d]
 *   u8 receives the codes, X_perm_scale [N, d/128] f32 the scales (NULL
 *   otherwise).  X_perm may be NULL (any dtype), in which case only the
 *   maps are written (for moe_expert_ffn_gather and
 *   moe_expert_ffn_gather_fp8, which gather the token rows themselves).
 */
moe_status moe_dispatch(const moe_cfg* cfg, const void* X, const int32_t* topk_idx,
                        int32_t* offsets, int32_t* row_map, int32_t* inv_map, void* X_perm,
                        float* X_perm_scale, void* ws, size_t ws_bytes, void* stream);

/*
 * moe_dispatch_noalloc -- moe_dispatch for callers that cannot allocate
 *   device memory (code under stream capture, serving loops, harnesses that
 *   forbid allocation): identical arguments, definition and results, minus
 *   the workspace.  Its scratch (the per-256-token-block expert counts,
 *   ceil(T/256) * E int32) lives in a fixed 4 MiB device array inside the
 *   library, one copy per GPU, held until the process ends; the call never
 *   allocates or frees memory.  A configuration whose counts need more than
 *   4 MiB (e.g. E = 64 with T > 4 194 304, E = 1024 with T > 262 144)
 *   returns MOE_EUNSUPPORTED.  ``stream`` must belong to the current device
 *   (MOE_EINVAL otherwise).  Every call on one GPU shares that GPU's array
 *   and leaves its counts there: calls issued in order on one stream are
 *   safe, calls that overlap on one GPU (concurrent streams or host threads)
 *   race and give unspecified maps.  Nothing needs clearing between calls
 *   (each call writes every count it reads).
 */
moe_status moe_dispatch_noalloc(const moe_cfg* cfg, const void* X, const int32_t* topk_idx,
                                int32_t* offsets, int32_t* row_map, int32_t* inv_map,
                                void* X_perm, float* X_perm_scale, void* stream);

/*
 * moe_expert_ffn -- grouped SwiGLU experts over uneven per-expert row counts.
 *   For the rows r of expert e (offsets[e] <= r < offsets[e+1]):
 *     A = X_perm[r] W1_e^T, B = X_perm[r] W3_e^T, h = silu(A) * B,
 *     Y[r] = h W2_e^T, silu(z) = z / (1 + exp(-z)); FP32 accumulation, h
 *     stored in cfg.act between the two products.
 *   W13 [E, 2f, d] cfg.w (rows 0..f-1 = W1_e, rows f..2f-1 = W3_e);
 *   W2 [E, d, f] cfg.w; X_perm [N,d] act; Y [N,d] act out.
 *   Supported: act = w = MOE_F32; act = w = MOE_BF16 (d % 128 == 0,
 *   f % 64 == 0); act = MOE_BF16 with w = MOE_FP8E4M3 (d % 128 == 0,
 *   f % 128 == 0).
 *   FP8 experts: X_perm [N,d] u8 codes with X_perm_scale [N, d/128] (as
 *   moe_dispatch writes them); W13 / W2 u8 codes with W13_scale
 *   [E, 2f/128, d/128] and W2_scale [E, d/128, f/128] (128 x 128 blocks, as
 *   moe_quantize_fp8 writes them).  Every product accumulates each 128-wide
 *   K block on its own and adds it to the FP32 result times sa * sb; h is
 *   rounded to BF16 and re-quantised per 1 x 128 block before the second
 *   product; Y is BF16.  The scale pointers are ignored (may be NULL) for
 *   the other dtypes.
 */
moe_status moe_expert_ffn(const moe_cfg* cfg, const void* X_perm, const float* X_perm_scale,
                          const int32_t* offsets, const void* W13, const float* W13_scale,
                          const void* W2, const float* W2_scale, void* Y, void* ws,
                          size_t ws_bytes, void* stream);

/*
 * moe_expert_ffn_gather -- moe_expert_ffn with the permute fused into the
 *   first product: row r of the experts' input is X[row_map[r]], read
 *   straight from X [T,d] (no X_perm).  Same definition and results as
 *   moe_dispatch followed by moe_expert_ffn.  Requires BF16 activations and
 *   weights, d_ff % 128 == 0 and d % 256 == 0 (else MOE_EUNSUPPORTED).
 *   row_map [N] and offsets [E+1] as moe_dispatch writes them.
 */
moe_status moe_expert_ffn_gather(const moe_cfg* cfg, const void* X, const int32_t* row_map,
                                 const int32_t* offsets, const void* W13, const void* W2, void* Y,
                                 void* ws, size_t ws_bytes, void* stream);

/*
 * moe_expert_ffn_gather_save -- moe_expert_ffn_gather that also stores the
 *   first product's pre-activations for the backward (training forwards):
 *     AB[r] = [A_r | B_r] = [Xp_r W1_e^T | Xp_r W3_e^T]   [N, 2*d_ff] BF16 out
 *   (A in columns 0..d_ff-1, B in d_ff..2*d_ff-1; each value is the FP32
 *   product rounded to BF16, the same values moe_expert_ffn_bwd recomputes).
 *   Y is bit-identical to moe_expert_ffn_gather's.  AB: caller-owned, 16-byte
 *   aligned, not NULL when T > 0 (else MOE_EINVAL); other arguments and
 *   errors as moe_expert_ffn_gather.
 */
moe_status moe_expert_ffn_gather_save(const moe_cfg* cfg, const void* X, const int32_t* row_map,
                                      const int32_t* offsets, const void* W13, const void* W2,
                                      void* Y, void* AB, void* ws, size_t ws_bytes,
                                      void* stream);

/*
 * moe_expert_ffn_gather_fp8 -- the FP8-expert moe_expert_ffn with the permute
 *   fused into the first product: slot row r reads token row row_map[r] of
 *   the per-token codes X_codes [T,d] u8 and scales X_scale [T, d/128] f32
 *   (X quantised once per token, as moe_quantize_fp8 with block_rows = 1
 *   writes it), so no slot-ordered copy of the codes is made.  Same
 *   definition and results, bit for bit, as moe_dispatch (FP8) followed by
 *   moe_expert_ffn.  Requires cfg.act = MOE_BF16, cfg.w = MOE_FP8E4M3,
 *   d % 128 == 0 and d_ff % 128 == 0 (else MOE_EUNSUPPORTED).  row_map [N]
 *   and offsets [E+1] as moe_dispatch writes them; weights and Y as in
 *   moe_expert_ffn.
 */
moe_status moe_expert_ffn_gather_fp8(const moe_cfg* cfg, const uint8_t* X_codes,
                                     const float* X_scale, const int32_t* row_map,
                                     const int32_t* offsets, const uint8_t* W13,
                                     const float* W13_scale, const uint8_t* W2,
                                     const float* W2_scale, void* Y, void* ws, size_t ws_bytes,
                                     void* stream);

/*
 * moe_quantize_fp8 -- OCP FP8 e4m3 block quantisation of src [rows, cols]
 *   (src_dtype MOE_F32 or MOE_BF16; cols % 128 == 0) in blocks of
 *   block_rows x 128 (block_rows 1 or 128; a ragged last row block is
 *   allowed).  Per block: amax = max |x| (FP32); if amax == 0 the scale is
 *   1 and every code 0, else inv = fl32(448 / amax), code = e4m3 of
 *   fl32(x * inv) rounded to nearest even and saturated to +-448, scale =
 *   fl32(amax / 448).  codes [rows, cols] u8 out (8-byte aligned); scales
 *   [ceil(rows / block_rows), cols / 128] f32 out.  Expert weights [E, R, C]
 *   quantise as rows = E * R when R % 128 == 0.
 */
moe_status moe_quantize_fp8(int rows, int cols, int block_rows, int src_dtype, const void* src,
                            uint8_t* codes, float* scales, void* stream);

/*
 * OCP Microscaling (MX) experts (cfg.w = MOE_MXFP8E4M3, MOE_MXFP6E2M3 or
 * MOE_MXFP4E2M1; the published OCP Microscaling Formats v1.0 block format).
 * A matrix [R, K] (K % 32 == 0) is quantised along K in blocks of 32: amax
 * = max |x| of the block; s = floor(log2 amax) - emax (emax 8 for e4m3, 2
 * for e2m3 and e2m1), clamped to [-127, 127], s = 0 for an all-zero block;
 * scale byte = s + 127 (E8M0); code_i = the element value nearest to
 * x_i / 2^s, ties to the even mantissa, magnitudes above the largest
 * normal (448, 7.5, 6) saturated, sign kept.  Inputs must be finite.
 * Code layout of a row of K elements: e4m3 one byte per code (K bytes);
 * e2m3 per block the 32 codes 6 bits apart (code i at bits 6i of the
 * block's little-endian bit string) in 24 bytes followed by 8 zero bytes
 * (K bytes); e2m1 two codes per byte, lower index in the low nibble (K/2
 * bytes).  Scales [R, K/32] u8.
 */

/*
 * moe_quantize_mx -- MX quantisation of src [rows, cols] (src_dtype MOE_F32
 *   or MOE_BF16; cols % 32 == 0, rows * cols < 2^40) as stated above.
 *   fmt: MOE_MXFP8E4M3, MOE_MXFP6E2M3 or MOE_MXFP4E2M1.  codes [rows, row
 *   bytes] u8 out (16-byte aligned), scales [rows, cols/32] u8 out (4-byte
 *   aligned).  Expert weights [E, R, C] quantise as rows = E * R.
 */
moe_status moe_quantize_mx(int rows, int cols, int fmt, int src_dtype, const void* src,
                           uint8_t* codes, uint8_t* scales, void* stream);

/*
 * moe_expert_ffn_mx -- grouped SwiGLU experts with MX operands, the permute
 *   fused into the first product:
 *     for the slots r of expert e: x = MX-dequantised token row row_map[r];
 *     A = x W1_e^T, B = x W3_e^T with MX-dequantised weights (block products
 *     accumulated in FP32 by the scaled matrix instructions); h = silu(A) *
 *     B rounded to BF16, then MX-quantised along f (1 x 32 blocks); Y[r] =
 *     h W2_e^T (FP32 accumulation) stored as BF16.
 *   cfg.act = MOE_BF16, cfg.w one of the MX formats; d % 256 == 0 and
 *   d_ff % 128 == 0 (else MOE_EUNSUPPORTED).  X_codes [T, row bytes of d],
 *   X_scale [T, d/32] (moe_quantize_mx of the tokens); W13 [E*2f, row
 *   bytes of d] with W13_scale [E*2f, d/32] (rows 0..f-1 of expert e =
 *   W1_e, f..2f-1 = W3_e); W2 [E*d, row bytes of f] with W2_scale
 *   [E*d, f/32]; row_map [N], offsets [E+1] as moe_dispatch writes them;
 *   Y [N,d] bf16 out.  ws: moe_workspace_bytes(cfg).
 */
moe_status moe_expert_ffn_mx(const moe_cfg* cfg, const uint8_t* X_codes, const uint8_t* X_scale,
                             const int32_t* row_map, const int32_t* offsets, const uint8_t* W13,
                             const uint8_t* W13_scale, const uint8_t* W2,
                             const uint8_t* W2_scale, void* Y, void* ws, size_t ws_bytes,
                             void* stream);

/*
 * moe_combine -- out[t] = sum_j topk_w[t,j] * Y[inv_map[t,j]], accumulated
 *   in FP32 in j order, stored in cfg.act.
 *   Y [N,d] act; inv_map [T,k] i32; topk_w [T,k] f32; out [T,d] act out.
 */
moe_status moe_combine(const moe_cfg* cfg, const void* Y, const int32_t* inv_map,
                       const float* topk_w, void* out, void* stream);

/*
 * Backward of the layer with the routing held fixed: the chosen experts and
 * the prices that chose them are constants, so no gradient flows into the
 * prices or through the selection; everything below is the exact derivative
 * of the forward definitions above on that piece.
 */

/*
 * moe_combine_bwd -- derivative of moe_combine.
 *   dY[inv_map[t,j]] = topk_w[t,j] * dOut[t]          (act dtype)
 *   dtopk_w[t,j]     = <dOut[t], Y[inv_map[t,j]]>     (FP32, fixed order)
 *   dOut [T,d] act; Y [N,d] act (the forward's); dY [N,d] act out;
 *   dtopk_w [T,k] f32 out.
 */
moe_status moe_combine_bwd(const moe_cfg* cfg, const void* dOut, const void* Y,
                           const int32_t* inv_map, const float* topk_w, void* dY,
                           float* dtopk_w, void* stream);

/*
 * moe_expert_ffn_bwd -- derivative of moe_expert_ffn for an upstream dY in
 * slot order.  The permuted tokens are recomputed from X through row_map
 * (not read from a saved X_perm), as are A = Xp W1^T and B = Xp W3^T:
 *   U = dY W2_e,  dA = U * B * silu'(A),  dB = U * silu(A),  h = silu(A) * B
 *   dX_perm = dA W1_e + dB W3_e              [N,d] act out
 *   dW13[e] = [dA | dB]^T Xp                 [E,2f,d] out
 *   dW2[e]  = dY^T h                         [E,d,f] out
 * with silu'(z) = s + z s (1 - s), s = 1/(1+exp(-z)).  The weight
 * gradients accumulate in FP32 and are stored as grad_dtype (MOE_F32, or
 * MOE_BF16 rounded to nearest even; else MOE_EINVAL).  Requires BF16
 * activations and weights, d_ff % 128 == 0 and d % 256 == 0 (otherwise
 * MOE_EUNSUPPORTED).  X [T,d]; row_map [N]; offsets [E+1] from moe_dispatch.
 */
moe_status moe_expert_ffn_bwd(const moe_cfg* cfg, const void* X, const int32_t* row_map,
                              const int32_t* offsets, const void* dY, const void* W13,
                              const void* W2, void* dX_perm, void* dW13, void* dW2,
                              int grad_dtype, void* ws, size_t ws_bytes, void* stream);

/*
 * moe_expert_ffn_bwd_saved -- moe_expert_ffn_bwd reading the pre-activations
 *   AB [N, 2*d_ff] BF16 that moe_expert_ffn_gather_save stored for the same
 *   X, row_map, offsets and W13, instead of recomputing them (the first
 *   product of the backward is skipped).  Results are bit-identical to
 *   moe_expert_ffn_bwd's.  AB: 16-byte aligned, not NULL when T > 0 (else
 *   MOE_EINVAL); read only.  Other arguments, workspace size and errors as
 *   moe_expert_ffn_bwd.
 */
moe_status moe_expert_ffn_bwd_saved(const moe_cfg* cfg, const void* X, const int32_t* row_map,
                                    const int32_t* offsets, const void* dY, const void* W13,
                                    const void* W2, const void* AB, void* dX_perm, void* dW13,
                                    void* dW2, int grad_dtype, void* ws, size_t ws_bytes,
                                    void* stream);

/*
 * moe_dispatch_bwd -- derivative of moe_dispatch's permute:
 *   dX[t] = sum_j dX_perm[inv_map[t,j]]   (j order, FP32 out [T,d]).
 */
moe_status moe_dispatch_bwd(const moe_cfg* cfg, const void* dX_perm, const int32_t* inv_map,
                            float* dX, void* stream);

/*
 * moe_route_bwd -- gate and router backward, fused with the permute
 * backward into one dX:
 *   ds[t,j] = w[t,j] (dw[t,j] - sum_i w[t,i] dw[t,i])   (softmax over the
 *             chosen experts' raw logits; dw = dtopk_w)
 *   dX[t]   = sum_j dX_perm[inv_map[t,j]] + sum_j ds[t,j] W_r[e_j]   [T,d] out
 *             (FP32 sums stored as dx_dtype: MOE_F32, or MOE_BF16 rounded
 *             to nearest even; else MOE_EINVAL)
 *   dWr[e]  = sum over the slots of e of ds * X[t]                    [E,d] f32
 *   dbr[e]  = sum of the same ds                                      [E] f32
 *   (the sums run over chunks of 64 slots in slot order, whose partial
 *   sums are added in a fixed order: the result is deterministic)
 *   (topk_idx, topk_w, row_map, offsets, inv_map as produced by the forward.)
 */
moe_status moe_route_bwd(const moe_cfg* cfg, const void* X, const float* Wr,
                         const int32_t* topk_idx, const float* topk_w, const float* dtopk_w,
                         const int32_t* row_map, const int32_t* offsets, const int32_t* inv_map,
                         const void* dX_perm, void* dX, int dx_dtype, float* dWr, float* dbr,
                         void* ws, size_t ws_bytes, void* stream);

/*
 * Optional per-kernel timing for benchmarks (host bookkeeping, not
 * thread-safe).  When enabled, each instrumented kernel launch is bracketed
 * by a HIP event pair on its stream.  moe_prof_get waits for the recorded
 * events and returns the summed elapsed time and the launch count of one
 * kernel name: "router_logits", "price_loop", "dispatch", "quant_rows" (FP8
 * token quantisation), "quant_mx" (MX token quantisation), "gemm1_swiglu",
 * "gemm2", "combine", "combine_bwd", "ffn_bwd", "dispatch_bwd", "route_bwd".
 * moe_prof_reset forgets every record.
 */
moe_status moe_prof_enable(int on);
moe_status moe_prof_reset(void);
moe_status moe_prof_get(const char* kernel /* host */, double* total_ms /* host out */,
                        int32_t* launches /* host out */);

/*
 * moe_prof_lds_copy -- calibration copy for hardware byte counters: dst =
 *   src (bytes % 16 == 0, both 16-byte aligned, device pointers), every
 *   16-byte piece read from memory straight into LDS by the direct-to-LDS
 *   load the expert products use for their operands, then written out by
 *   ordinary vector stores.  Not on any layer path.
 */
moe_status moe_prof_lds_copy(const void* src, void* dst, size_t bytes, void* stream);

/* Status text (host, static storage). */
const char* moe_strerror(int status);

#ifdef __cplusplus
}
#endif

#endif /* MOE_H */
