// Internal host-side context shared by the C-ABI translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <string>

#include "../../include/dgsrhd.h"
#include "launch.hpp"
#include "launch_lim.hpp"

namespace dgsrhd {
// A validated mesh description and what is derived from it on the host.
struct MeshSetup {
  dg_mesh_desc desc{};
  PhysParams q{};
  Tables t{};
  MeshArgs m{};
  int nv = 0, npe = 0;
  long long ntot = 0;
  double xi[kMaxN1] = {};      // Gauss-Legendre nodes on [-1, 1]
  double lim_inv_den = 0.0;    // 1 / sum_n w_n xi_{d,n}^2 of the slope limiter
};
}  // namespace dgsrhd

struct dg_ctx : dgsrhd::MeshSetup {
  hipStream_t stream = nullptr;
  hipEvent_t handoff = nullptr;      // orders a new stream after the work queued on the old one
  double* Wa = nullptr;
  double* Wb = nullptr;
  double* U1 = nullptr;
  double* U2 = nullptr;
  double* adj = nullptr;     // adjoint scratch (allocated on first use)
  double* avg = nullptr;     // element averages of the slope limiter (allocated with it)
  size_t adj_doubles = 0;
  dgsrhd::Counters* cnt = nullptr;
  dgsrhd::Counters last{};           // counter snapshot for sync-mode error reporting
  int flip = 0;                      // tile direction of the last element launch
  std::string err;
};


namespace dgsrhd {
int fail(dg_ctx* c, int code, const char* fmt, ...);
int hipcheck(dg_ctx* c, hipError_t e, const char* what);
int finish(dg_ctx* c, const char* what);
ElemArgs base_args(dg_ctx* c);
const char* setup_mesh(const dg_mesh_desc* in, MeshSetup& s);
hipError_t launch_element(const MeshSetup& s, int mode, const ElemArgs& a, hipStream_t st);
bool fused_rhs(const MeshSetup& s);
hipError_t launch_con2prim(const MeshSetup& s, const double* U, double* W, Counters* cnt, hipStream_t st);
hipError_t L_element(dg_ctx* c, int mode, const ElemArgs& a);
hipError_t L_con2prim(dg_ctx* c, const double* U, double* W);
hipError_t L_enforce(dg_ctx* c, double* U);
hipError_t L_prim3(dg_ctx* c, const double* S, double* U);
hipError_t L_limiter(dg_ctx* c, double* U, double* Wout);
}  // namespace dgsrhd
