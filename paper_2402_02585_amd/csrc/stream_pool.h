// Streams lent to graph captures (host side).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <vector>

namespace gqaoa {

// Non-blocking streams of default priority lent to graph captures (the
// capture stream and the parallel branches of a plan). Creating a stream
// costs about 0.1 ms and destroying one about 0.4 ms of host time on this
// GPU, so returned streams are kept per device for the next plan until the
// process ends. take() appends n streams of the current device to *out;
// give() returns streams of `device` once no work or capture uses them.
int stream_pool_take(size_t n, std::vector<hipStream_t> *out);
void stream_pool_give(int device, const std::vector<hipStream_t> &streams);

}  // namespace gqaoa
