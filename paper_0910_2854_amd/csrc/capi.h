// capi.h -- checks of the C interface shared by its translation units
// (fish.hip, noalloc.hip).
#pragma once

#include <string>

#include "../../include/fish.h"

namespace fish {

// FISH_OK, or FISH_ERR_ARG for a scheme setting outside its range.
int check_common(double gamma, int limiter, double alpha, int precision, int gravity, int hse);

// FISH_OK when the caller's stream, allocator or device memory can belong to
// this library's HIP runtime; FISH_ERR_DEVICE with a message in *msg when the
// process has loaded a second HIP runtime and the caller passes any of them.
int check_runtime(const void* stream, bool caller_memory, std::string* msg);

// The message fish_last_error(NULL) returns on the calling thread.
void set_thread_error(const std::string& msg);

}  // namespace fish
