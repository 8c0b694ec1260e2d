// batch.h -- the batch object of the C interface (shared by the batch calls
// in fish.hip and the request server in server.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/fish.h"
#include "engine.h"

struct fish_batch {
  fish_batch_params p{};
  fish::Engine e;
  hipStream_t own_stream = nullptr;
};
