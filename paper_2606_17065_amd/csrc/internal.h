// Declarations shared between the translation units of libmoe (not ABI).
#pragma once

#include <stddef.h>

#include "../../include/moe.h"

// Workspace bytes each entry point carves from the caller's buffer.
size_t route_ws_bytes(const moe_cfg& c);
size_t price_ws_bytes(const moe_cfg& c);
size_t dispatch_ws_bytes(const moe_cfg& c);
size_t ffn_ws_bytes(const moe_cfg& c);
size_t ffn_bwd_ws_bytes(const moe_cfg& c);
size_t route_bwd_ws_bytes(const moe_cfg& c);
size_t stats_ws_bytes(const moe_cfg& c);
size_t cert_ws_bytes(const moe_cfg& c);
size_t judged_ws_bytes(const moe_cfg& c);

// Certificate of a routing under prices (moe_route_certify without the
// checks): part holds 2 * (ceil(T / 64) + 1) doubles, cert[3] receives
// primal, dual and the relative gap.
void launch_certify(const moe_cfg& c, const float* logits, const float* price,
                    const int32_t* topk_idx, double* part, double* cert, void* stream);

// Host-side argument checks shared by several entry points.
moe_status check_cfg_shape(const moe_cfg* c);
bool aligned(const void* p, size_t a);
int act_bytes(int dtype);

// Per-kernel event timing (moe_prof_*): record around a launch on ``stream``.
bool prof_on();
void prof_mark(const char* name, void* stream, bool begin);
#define PROF_BEGIN(name, stream) \
  if (prof_on()) prof_mark(name, (void*)(stream), true)
#define PROF_END(name, stream) \
  if (prof_on()) prof_mark(name, (void*)(stream), false)
