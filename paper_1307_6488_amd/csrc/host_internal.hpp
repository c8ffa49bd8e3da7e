// host_internal.hpp -- host-side pieces of chemora.hip shared with the
// library's other host translation units (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include "chemora.h"

namespace chemora {
namespace host {

// Records a formatted message for chemora_last_error() and returns code.
int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
void clear_error();

// The checks chemora_rk4_step makes of its params, patch and dt (everything
// but the scratch pointer); host only, no HIP call.
int check_step(const chemora_params* params, const chemora_patch* patch, double dt);

// The four stages of chemora_rk4_step on caller-checked arguments, with the
// stage buffers and the accumulator at scratch[0 .. 3*24*sf).
int rk4_step(const chemora_params* params, const chemora_patch* patch, double dt, double* scratch, hipStream_t s);

}  // namespace host
}  // namespace chemora
