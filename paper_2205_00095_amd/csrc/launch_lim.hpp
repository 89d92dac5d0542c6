// Launch interface of the slope-limiter kernel (per-dimension translation units).
#pragma once
#include "limiter.hpp"

namespace dgsrhd {

// The limiter on a.U given its element averages a.avg, then the operator (a.phys) and
// the recovery into a.Wout (if set).
hipError_t launch_limiter_dim1(int p, int eos, const LimArgs& a, hipStream_t s);
hipError_t launch_limiter_dim2(int p, int eos, const LimArgs& a, hipStream_t s);
hipError_t launch_limiter_dim3(int p, int eos, const LimArgs& a, hipStream_t s);

}  // namespace dgsrhd
