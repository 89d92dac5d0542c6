// Template instantiation and launch of the slope-limiter kernel for one spatial
// dimension (compiled once per dimension with -DDG_DIM=1, 2 or 3).
#include "launch_lim.hpp"

#ifndef DG_DIM
#error "DG_DIM must be defined"
#endif

namespace dgsrhd {

namespace {

template <int DIM, int P>
hipError_t run_limiter(int eos, const LimArgs& a, hipStream_t s) {
  using L = LimGeo<DIM, P>;
  const int nb = (a.m.nelem + L::EPB - 1) / L::EPB;
  if (eos == EOS_IDEAL)
    hipLaunchKernelGGL((k_limit<DIM, P, EOS_IDEAL>), dim3(nb), dim3(L::NT), 0, s, a);
  else
    hipLaunchKernelGGL((k_limit<DIM, P, EOS_TM>), dim3(nb), dim3(L::NT), 0, s, a);
  return hipGetLastError();
}

}  // namespace

#define DG_CAT2(a, b) a##b
#define DG_CAT(a, b) DG_CAT2(a, b)

hipError_t DG_CAT(launch_limiter_dim, DG_DIM)(int p, int eos, const LimArgs& a, hipStream_t s) {
  switch (p) {
    case 1: return run_limiter<DG_DIM, 1>(eos, a, s);
    case 2: return run_limiter<DG_DIM, 2>(eos, a, s);
    case 3: return run_limiter<DG_DIM, 3>(eos, a, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace dgsrhd
