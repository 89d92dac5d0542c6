// Template instantiation and launch of the gfx950 kernels for one spatial
// dimension.  Compiled once per dimension with -DDG_DIM=1, 2 or 3 so the three
// translation units build in parallel.
#include "launch.hpp"

#ifndef DG_DIM
#error "DG_DIM must be defined"
#endif

namespace dgsrhd {

namespace {

template <int DIM, int P, int EOS, int PREC, int MODE, int FLUX>
hipError_t run_element(const ElemArgs& a, hipStream_t s) {
  using T = TileGeo<DIM, P>;
  const int nb = ((a.m.nex + T::TX - 1) / T::TX) * ((a.m.ney + T::TY - 1) / T::TY) *
                 ((a.m.nez + T::TZ - 1) / T::TZ);
  hipLaunchKernelGGL((k_element<DIM, P, EOS, PREC, MODE, FLUX>), dim3(nb), dim3(T::NT), 0, s, a);
  return hipGetLastError();
}

template <int DIM, int P, int EOS, int PREC, int MODE>
hipError_t by_flux(int flux, const ElemArgs& a, hipStream_t s) {
  return flux == FLUX_HLL ? run_element<DIM, P, EOS, PREC, MODE, FLUX_HLL>(a, s)
                          : run_element<DIM, P, EOS, PREC, MODE, FLUX_HLLC>(a, s);
}

template <int DIM, int P, int EOS, int PREC>
hipError_t by_mode(int mode, int flux, const ElemArgs& a, hipStream_t s) {
  if (mode == MODE_RHS_FUSED) {
    if constexpr (TileGeo<DIM, P>::kFusedRhs) return by_flux<DIM, P, EOS, PREC, MODE_RHS_FUSED>(flux, a, s);
    return hipErrorInvalidValue;
  }
  if (mode == MODE_STAGE_LIM) {
    if constexpr (P > 0) return by_flux<DIM, P, EOS, PREC, MODE_STAGE_LIM>(flux, a, s);
    return hipErrorInvalidValue;
  }
  return mode == MODE_RHS ? by_flux<DIM, P, EOS, PREC, MODE_RHS>(flux, a, s)
                          : by_flux<DIM, P, EOS, PREC, MODE_STAGE>(flux, a, s);
}

template <int DIM, int P, int EOS>
hipError_t by_prec(int prec, int mode, int flux, const ElemArgs& a, hipStream_t s) {
  if (prec == PREC_FP32_MFMA) {
    if constexpr (DIM == 2 && P == 3) return by_mode<DIM, P, EOS, PREC_FP32_MFMA>(mode, flux, a, s);
    return hipErrorInvalidValue;
  }
  return prec == PREC_FP64 ? by_mode<DIM, P, EOS, PREC_FP64>(mode, flux, a, s)
                           : by_mode<DIM, P, EOS, PREC_FP32>(mode, flux, a, s);
}

template <int DIM, int P>
hipError_t by_eos(int eos, int prec, int mode, int flux, const ElemArgs& a, hipStream_t s) {
  return eos == EOS_IDEAL ? by_prec<DIM, P, EOS_IDEAL>(prec, mode, flux, a, s)
                          : by_prec<DIM, P, EOS_TM>(prec, mode, flux, a, s);
}

template <int DIM, int P>
hipError_t run_enforce(double* U, const MeshArgs& m, const Tables& t, const PhysParams& q, Counters* c,
                       hipStream_t s) {
  using G = Geo<DIM, P>;
  const int nb = (m.nelem + G::EPB - 1) / G::EPB;
  hipLaunchKernelGGL((k_enforce<DIM, P>), dim3(nb), dim3(G::NT), 0, s, U, m, t, q, c);
  return hipGetLastError();
}

}  // namespace

#define DG_CAT2(a, b) a##b
#define DG_CAT(a, b) DG_CAT2(a, b)

hipError_t DG_CAT(launch_element_dim, DG_DIM)(int p, int eos, int prec, int mode, int flux, const ElemArgs& a,
                                              hipStream_t s) {
  switch (p) {
    case 0: return by_eos<DG_DIM, 0>(eos, prec, mode, flux, a, s);
    case 1: return by_eos<DG_DIM, 1>(eos, prec, mode, flux, a, s);
    case 2: return by_eos<DG_DIM, 2>(eos, prec, mode, flux, a, s);
    case 3: return by_eos<DG_DIM, 3>(eos, prec, mode, flux, a, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t DG_CAT(launch_enforce_dim, DG_DIM)(int p, double* U, const MeshArgs& m, const Tables& t,
                                              const PhysParams& q, Counters* c, hipStream_t s) {
  switch (p) {
    case 0: return run_enforce<DG_DIM, 0>(U, m, t, q, c, s);
    case 1: return run_enforce<DG_DIM, 1>(U, m, t, q, c, s);
    case 2: return run_enforce<DG_DIM, 2>(U, m, t, q, c, s);
    case 3: return run_enforce<DG_DIM, 3>(U, m, t, q, c, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t DG_CAT(launch_con2prim_dim, DG_DIM)(int eos, const double* U, double* W, long long ntot, int npe,
                                               const PhysParams& q, Counters* c, hipStream_t s) {
  const int nb = (int)((ntot + 255) / 256);
  if (eos == EOS_IDEAL)
    hipLaunchKernelGGL((k_con2prim<EOS_IDEAL, DG_DIM>), dim3(nb), dim3(256), 0, s, U, W, ntot, npe, q, c);
  else
    hipLaunchKernelGGL((k_con2prim<EOS_TM, DG_DIM>), dim3(nb), dim3(256), 0, s, U, W, ntot, npe, q, c);
  return hipGetLastError();
}

hipError_t DG_CAT(launch_prim3_to_cons_dim, DG_DIM)(int eos, const double* S, double* U, long long ntot,
                                                    const PhysParams& q, Counters* c, hipStream_t s) {
  const int nb = (int)((ntot + 255) / 256);
  if (eos == EOS_IDEAL)
    hipLaunchKernelGGL((k_prim3_to_cons<EOS_IDEAL, DG_DIM>), dim3(nb), dim3(256), 0, s, S, U, ntot, q, c);
  else
    hipLaunchKernelGGL((k_prim3_to_cons<EOS_TM, DG_DIM>), dim3(nb), dim3(256), 0, s, S, U, ntot, q, c);
  return hipGetLastError();
}

}  // namespace dgsrhd
