// Template instantiation and launch of the adjoint kernels for one spatial
// dimension (compiled with -DDG_DIM=1, 2 or 3).
#include "launch_adj.hpp"

#ifndef DG_DIM
#error "DG_DIM must be defined"
#endif

namespace dgsrhd {

namespace {

template <int DIM, int P, int EOS, int MODE, int FLUX>
hipError_t run_vjp(const VjpArgs& a, hipStream_t s) {
  using T = TileGeo<DIM, P>;
  const int nb = ((a.m.nex + T::TX - 1) / T::TX) * ((a.m.ney + T::TY - 1) / T::TY) *
                 ((a.m.nez + T::TZ - 1) / T::TZ);
  hipLaunchKernelGGL((k_rhs_vjp<DIM, P, EOS, MODE, FLUX>), dim3(nb), dim3(T::NT), 0, s, a);
  return hipGetLastError();
}

template <int DIM, int P, int EOS, int MODE>
hipError_t vjp_by_flux(int flux, const VjpArgs& a, hipStream_t s) {
  return flux == FLUX_HLL ? run_vjp<DIM, P, EOS, MODE, FLUX_HLL>(a, s) : run_vjp<DIM, P, EOS, MODE, FLUX_HLLC>(a, s);
}

template <int DIM, int P>
hipError_t vjp_by(int eos, int mode, int flux, const VjpArgs& a, hipStream_t s) {
  if (eos == EOS_IDEAL)
    return mode == VJP_PLAIN ? vjp_by_flux<DIM, P, EOS_IDEAL, VJP_PLAIN>(flux, a, s)
                             : vjp_by_flux<DIM, P, EOS_IDEAL, VJP_STAGE>(flux, a, s);
  return mode == VJP_PLAIN ? vjp_by_flux<DIM, P, EOS_TM, VJP_PLAIN>(flux, a, s)
                           : vjp_by_flux<DIM, P, EOS_TM, VJP_STAGE>(flux, a, s);
}

template <int DIM, int P>
hipError_t run_enforce_vjp(const double* Pst, const double* lin, double* lout, const unsigned* flag,
                           const MeshArgs& m, const Tables& t, const PhysParams& q, hipStream_t s) {
  using G = Geo<DIM, P>;
  const int nb = (m.nelem + G::EPB - 1) / G::EPB;
  hipLaunchKernelGGL((k_enforce_vjp<DIM, P>), dim3(nb), dim3(G::NT), 0, s, Pst, lin, lout, m, t, q, flag);
  return hipGetLastError();
}

}  // namespace

#define DG_CAT2(a, b) a##b
#define DG_CAT(a, b) DG_CAT2(a, b)

hipError_t DG_CAT(launch_vjp_dim, DG_DIM)(int p, int eos, int mode, int flux, const VjpArgs& a, hipStream_t s) {
  switch (p) {
    case 0: return vjp_by<DG_DIM, 0>(eos, mode, flux, a, s);
    case 1: return vjp_by<DG_DIM, 1>(eos, mode, flux, a, s);
    case 2: return vjp_by<DG_DIM, 2>(eos, mode, flux, a, s);
    case 3: return vjp_by<DG_DIM, 3>(eos, mode, flux, a, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t DG_CAT(launch_enforce_vjp_dim, DG_DIM)(int p, const double* Pst, const double* lin, double* lout,
                                                  const unsigned* flag, const MeshArgs& m, const Tables& t,
                                                  const PhysParams& q, hipStream_t s) {
  switch (p) {
    case 0: return run_enforce_vjp<DG_DIM, 0>(Pst, lin, lout, flag, m, t, q, s);
    case 1: return run_enforce_vjp<DG_DIM, 1>(Pst, lin, lout, flag, m, t, q, s);
    case 2: return run_enforce_vjp<DG_DIM, 2>(Pst, lin, lout, flag, m, t, q, s);
    case 3: return run_enforce_vjp<DG_DIM, 3>(Pst, lin, lout, flag, m, t, q, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t DG_CAT(launch_objective_dim, DG_DIM)(int eos, const double* U, double* partial, double* grad,
                                                long long ntot, int npe, int n1, const Tables& t, double jac,
                                                const PhysParams& q, int nblocks, hipStream_t s) {
  if (eos == EOS_IDEAL)
    hipLaunchKernelGGL((k_objective<EOS_IDEAL, DG_DIM>), dim3(nblocks), dim3(256), 0, s, U, partial, grad, ntot, npe,
                       n1, t, jac, q);
  else
    hipLaunchKernelGGL((k_objective<EOS_TM, DG_DIM>), dim3(nblocks), dim3(256), 0, s, U, partial, grad, ntot, npe,
                       n1, t, jac, q);
  return hipGetLastError();
}

hipError_t DG_CAT(launch_prim3_vjp_dim, DG_DIM)(int eos, const double* S, const double* lamU, double* lamS,
                                                long long ntot, const PhysParams& q, hipStream_t s) {
  const int nb = (int)((ntot + 255) / 256);
  if (eos == EOS_IDEAL)
    hipLaunchKernelGGL((k_prim3_vjp<EOS_IDEAL, DG_DIM>), dim3(nb), dim3(256), 0, s, S, lamU, lamS, ntot, q);
  else
    hipLaunchKernelGGL((k_prim3_vjp<EOS_TM, DG_DIM>), dim3(nb), dim3(256), 0, s, S, lamU, lamS, ntot, q);
  return hipGetLastError();
}

}  // namespace dgsrhd
