// probes.hpp -- launch entry of the measurement helpers in probes.hip.
#pragma once
#include <hip/hip_runtime.h>

namespace lbm {
// The AA step's access pattern without arithmetic (see probes.hip): odd = 0
// the even step's, odd = 1 the odd step's (periodic on every axis).  q in
// {14, 18, 26}, elem in {2, 4, 8} bytes; buf holds q * stride elements,
// stride >= nx ny nz.  Queued on stream.
hipError_t launch_pattern_probe(void* buf, int q, int elem, int nx, int ny, int nz,
                                long long stride, int odd, int xcd, hipStream_t stream);
}  // namespace lbm
