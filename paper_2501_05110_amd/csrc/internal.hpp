// Host-side helpers of vfp.cpp shared with the other translation units that
// define C ABI entry points (not part of the ABI).
#pragma once
#include "vfp.h"

namespace vfp {
// Records a message for vfp_last_error() on this thread and returns code.
int api_fail(int code, const char* fmt, ...);
// Device ordinal a ready context is bound to (-1 before its first set-up call).
int ctx_device(const vfp_ctx* c);
}  // namespace vfp
