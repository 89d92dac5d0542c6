// Launch interface of the slope-limiter kernels (per-dimension translation units).
#pragma once
#include "limiter.hpp"

namespace dgsrhd {

// Element averages of a.U into avg ([NV][nelem], the caller's scratch, which a.avg must
// name), then the limiter, the operator (a.phys) and the recovery into a.Wout (if set).
hipError_t launch_limiter_dim1(int p, int eos, const LimArgs& a, double* avg, hipStream_t s);
hipError_t launch_limiter_dim2(int p, int eos, const LimArgs& a, double* avg, hipStream_t s);
hipError_t launch_limiter_dim3(int p, int eos, const LimArgs& a, double* avg, hipStream_t s);

}  // namespace dgsrhd
