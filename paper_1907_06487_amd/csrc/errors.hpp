// Error reporting shared by the C ABI's source files: the message of the
// last failure on the calling thread (race_last_error) and its code.
#pragma once

#include <hip/hip_runtime_api.h>

#include <string>

namespace race {

// Records msg for race_last_error and returns code.
int set_error(int code, const std::string& msg);
// Records "what: <HIP error string>" and returns RACE_EHIP.
int set_hip_error(hipError_t e, const char* what);

}  // namespace race
