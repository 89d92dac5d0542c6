// Internal launch interface of the adjoint kernels (one unit per dimension).
#pragma once
#include "adjoint.hpp"

namespace dgsrhd {

#define DG_DECLARE_ADJ_LAUNCHERS(D)                                                                             \
  hipError_t launch_vjp_dim##D(int p, int eos, int mode, int flux, const VjpArgs& a, hipStream_t s);           \
  hipError_t launch_enforce_vjp_dim##D(int p, const double* Pst, const double* lin, double* lout,              \
                                       const unsigned* flag, const MeshArgs& m, const Tables& t,                \
                                       const PhysParams& q, hipStream_t s);                                     \
  hipError_t launch_objective_dim##D(int eos, const double* U, double* partial, double* grad, long long ntot,   \
                                     int npe, int n1, const Tables& t, double jac, const PhysParams& q,          \
                                     int nblocks, hipStream_t s);                                               \
  hipError_t launch_prim3_vjp_dim##D(int eos, const double* S, const double* lamU, double* lamS,                \
                                     long long ntot, const PhysParams& q, hipStream_t s);

DG_DECLARE_ADJ_LAUNCHERS(1)
DG_DECLARE_ADJ_LAUNCHERS(2)
DG_DECLARE_ADJ_LAUNCHERS(3)

#undef DG_DECLARE_ADJ_LAUNCHERS

}  // namespace dgsrhd
