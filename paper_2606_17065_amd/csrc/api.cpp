// Host-side pieces of the C ABI shared by all entry points: shape checks,
// workspace sizing and status text.
#include <stdint.h>

#include <algorithm>

#include "../../include/moe.h"
#include "internal.h"

bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

int act_bytes(int dtype) {
  switch (dtype) {
    case MOE_F32: return 4;
    case MOE_BF16: return 2;
    case MOE_FP8E4M3: return 1;
    default: return 0;
  }
}

moe_status check_cfg_shape(const moe_cfg* c) {
  if (!c) return MOE_EINVAL;
  if (c->T < 0 || c->d < 1 || c->E < 1 || c->k < 1 || c->d_ff < 1 || c->capacity < 0)
    return MOE_EINVAL;
  if (c->act != MOE_F32 && c->act != MOE_BF16) return MOE_EINVAL;
  if (c->w < MOE_F32 || c->w > MOE_MXFP4E2M1) return MOE_EINVAL;
  if (c->price_stages < 0 || c->price_stages > 8) return MOE_EINVAL;
  if (c->k > c->E) return MOE_EINFEASIBLE;
  if ((int64_t)c->E * (int64_t)c->capacity < (int64_t)c->T * (int64_t)c->k) return MOE_EINFEASIBLE;
  if (c->E > 1024 || c->k > 16) return MOE_EUNSUPPORTED;
  if ((int64_t)c->T * (int64_t)c->k >= (int64_t)1 << 31) return MOE_EUNSUPPORTED;
  if ((int64_t)c->T * (int64_t)c->E >= (int64_t)1 << 31) return MOE_EUNSUPPORTED;
  if (c->d % 8 != 0) return MOE_EUNSUPPORTED;
  return MOE_OK;
}

extern "C" moe_status moe_workspace_bytes(const moe_cfg* cfg, size_t* bytes) {
  if (!bytes) return MOE_EINVAL;
  moe_status st = check_cfg_shape(cfg);
  if (st != MOE_OK) return st;
  size_t b = std::max(price_ws_bytes(*cfg), dispatch_ws_bytes(*cfg));
  b = std::max(b, ffn_ws_bytes(*cfg));
  b = std::max(b, route_bwd_ws_bytes(*cfg));
  b = std::max(b, cert_ws_bytes(*cfg));
  b = std::max(b, judged_ws_bytes(*cfg));
  if (cfg->T >= 1 && cfg->k < cfg->E) b = std::max(b, stats_ws_bytes(*cfg));
  if (cfg->act == MOE_BF16 && cfg->w == MOE_BF16 && cfg->d_ff % 128 == 0 && cfg->d % 256 == 0)
    b = std::max(b, ffn_bwd_ws_bytes(*cfg));
  *bytes = b;
  return MOE_OK;
}

extern "C" const char* moe_strerror(int status) {
  switch (status) {
    case MOE_OK: return "ok";
    case MOE_EINVAL: return "invalid argument (pointer, size, alignment or enum)";
    case MOE_EINFEASIBLE: return "infeasible routing: k > E or E*capacity < T*k";
    case MOE_EUNSUPPORTED: return "unsupported shape or dtype combination";
    case MOE_EWORKSPACE: return "workspace smaller than moe_workspace_bytes()";
    case MOE_EHIP: return "HIP launch failed";
    case MOE_ENAN: return "non-finite router logit";
    case MOE_ECAPACITY: return "capacity repair could not place every slot";
    default: return "unknown status";
  }
}
