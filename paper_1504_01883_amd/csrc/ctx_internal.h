// Host-side helpers of runtime.cpp used by the other host sources (the
// serving loop). Nothing here is part of the public ABI (include/lbpf.h).
#pragma once

#include <stddef.h>

#include "../../include/lbpf.h"

namespace lbpf {

// Charge `bytes` of device memory to the context's budget; false (nothing
// charged) when it would be exceeded.
bool ctx_charge(lbpf_ctx *ctx, size_t bytes);
// Give back bytes charged earlier.
void ctx_refund(lbpf_ctx *ctx, size_t bytes);
// HIP device of the context.
int ctx_device(const lbpf_ctx *ctx);

}  // namespace lbpf
