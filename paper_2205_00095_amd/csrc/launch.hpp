// Internal launch interface between the host C-ABI layer and the per-dimension
// kernel translation units.
#pragma once
#include "kernels.hpp"

namespace dgsrhd {

#define DG_DECLARE_LAUNCHERS(D)                                                                          \
  hipError_t launch_element_dim##D(int p, int eos, int prec, int mode, int flux, const ElemArgs& a,       \
                                   hipStream_t s);                                                        \
  hipError_t launch_enforce_dim##D(int p, double* U, const MeshArgs& m, const Tables& t,                  \
                                   const PhysParams& q, Counters* c, hipStream_t s);                      \
  hipError_t launch_con2prim_dim##D(int eos, const double* U, double* W, long long ntot, int npe,         \
                                    const PhysParams& q, Counters* c, hipStream_t s);                     \
  hipError_t launch_prim3_to_cons_dim##D(int eos, const double* S, double* U, long long ntot,             \
                                         const PhysParams& q, Counters* c, hipStream_t s);

DG_DECLARE_LAUNCHERS(1)
DG_DECLARE_LAUNCHERS(2)
DG_DECLARE_LAUNCHERS(3)

#undef DG_DECLARE_LAUNCHERS

}  // namespace dgsrhd
