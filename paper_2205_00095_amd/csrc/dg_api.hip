// Host side of the C ABI declared in include/dgsrhd.h: context, basis tables,
// scratch management, launch sequencing on the caller's HIP stream, counters.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/dgsrhd.h"
#include "ctx.hpp"

using namespace dgsrhd;

namespace dgsrhd {
__global__ void k_reset_counters(Counters* cnt) {
  const int i = threadIdx.x;
  if (i < kCounterSlots) {
    Counters* c = cnt + i;
    c->c2p_fail = c->c2p_noconv = c->trace_fallback = 0ull;
    c->flagged = c->smoothed = c->bad_average = c->bad_input = 0ull;
    c->first_bad = ~0ull;
    c->limited = 0ull;
  }
}

// All slots summed (first_bad: the minimum); synchronous.
static hipError_t read_counters(const Counters* dev, Counters& out) {
  Counters h[kCounterSlots];
  hipError_t e = hipMemcpy(h, dev, sizeof(h), hipMemcpyDeviceToHost);
  out = Counters{};
  out.first_bad = ~0ull;
  if (e != hipSuccess) return e;
  for (int i = 0; i < kCounterSlots; ++i) {
    out.c2p_fail += h[i].c2p_fail;
    out.c2p_noconv += h[i].c2p_noconv;
    out.trace_fallback += h[i].trace_fallback;
    out.flagged += h[i].flagged;
    out.smoothed += h[i].smoothed;
    out.bad_average += h[i].bad_average;
    out.bad_input += h[i].bad_input;
    out.limited += h[i].limited;
    out.first_bad = h[i].first_bad < out.first_bad ? h[i].first_bad : out.first_bad;
  }
  return hipSuccess;
}

static void to_diag(const Counters& h, dg_diag* out) {
  out->c2p_fail = (long long)h.c2p_fail;
  out->c2p_noconv = (long long)h.c2p_noconv;
  out->trace_fallback = (long long)h.trace_fallback;
  out->flagged = (long long)h.flagged;
  out->smoothed = (long long)h.smoothed;
  out->bad_average = (long long)h.bad_average;
  out->bad_input = (long long)h.bad_input;
  out->first_bad_elem = (h.first_bad == ~0ull) ? -1 : (long long)h.first_bad;
  out->limited = (long long)h.limited;
}

}  // namespace dgsrhd

namespace dgsrhd {

static const char* kNoCtx = "null context";

int fail(dg_ctx* c, int code, const char* fmt, ...) {
  if (c) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    c->err = buf;
  }
  return code;
}

int hipcheck(dg_ctx* c, hipError_t e, const char* what) {
  if (e != hipSuccess) return fail(c, DG_EHIP, "%s: %s", what, hipGetErrorString(e));
  return DG_OK;
}

// Gauss-Legendre nodes/weights on [-1, 1] by Newton iteration on P_n, and the
// Lagrange tables through barycentric weights.  Fixed-size arrays (p <= 3): no
// allocation, so the allocation-free entry point can build its tables per call.
void gl_tables(int p, int dim, Tables& t, double* xout) {
  const int n = p + 1;
  double x[kMaxN1], w[kMaxN1];
  if (n == 1) {
    x[0] = 0.0;
    w[0] = 2.0;
  } else {
    for (int i = 0; i < n; ++i) {
      double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
      double dp = 1.0;
      for (int it = 0; it < 100; ++it) {
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= n; ++k) {
          const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
          p0 = p1;
          p1 = p2;
        }
        dp = n * (z * p1 - p0) / (z * z - 1.0);
        const double dz = p1 / dp;
        z -= dz;
        if (std::fabs(dz) < 1e-16) break;
      }
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      x[n - 1 - i] = z;
      w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
    if (n % 2 == 1) x[n / 2] = 0.0;
  }
  double bw[kMaxN1];
  for (int j = 0; j < n; ++j) {
    bw[j] = 1.0;
    for (int k = 0; k < n; ++k)
      if (k != j) bw[j] /= (x[j] - x[k]);
  }
  // Dm[i][j] = l_j'(x_i)
  double Dm[kMaxN1][kMaxN1] = {};
  for (int i = 0; i < n; ++i) {
    double diag = 0.0;
    for (int j = 0; j < n; ++j) {
      if (j == i) continue;
      Dm[i][j] = (bw[j] / bw[i]) / (x[i] - x[j]);
      diag -= Dm[i][j];
    }
    Dm[i][i] = diag;
  }
  std::memset(&t, 0, sizeof(t));
  for (int i = 0; i < kMaxN1; ++i) xout[i] = i < n ? x[i] : 0.0;
  double wsum = 0.0;
  for (int i = 0; i < n; ++i) {
    double lp = 1.0, lm = 1.0;
    for (int k = 0; k < n; ++k) {
      if (k == i) continue;
      lp *= (1.0 - x[k]) / (x[i] - x[k]);
      lm *= (-1.0 - x[k]) / (x[i] - x[k]);
    }
    t.lp[i] = lp;
    t.lm[i] = lm;
    t.w[i] = w[i];
    t.iw[i] = 1.0 / w[i];
    wsum += w[i];
    for (int a = 0; a < n; ++a) t.dhat[i][a] = w[a] * Dm[a][i] / w[i];
  }
  t.inv_wsum = 1.0 / std::pow(wsum, dim);
  for (int i = 0; i < n; ++i) {
    t.lp_f[i] = (float)t.lp[i];
    t.lm_f[i] = (float)t.lm[i];
    t.iw_f[i] = (float)t.iw[i];
    for (int a = 0; a < n; ++a) t.dhat_f[i][a] = (float)t.dhat[i][a];
  }
}

// Validate a mesh description and derive the physical parameters, basis tables and
// mesh arguments from it, without allocating.  Returns null, or the reason the
// description is rejected.
const char* setup_mesh(const dg_mesh_desc* in, MeshSetup& s) {
  s = MeshSetup{};
  s.desc = *in;
  dg_mesh_desc& d = s.desc;
  if (d.dim < 1 || d.dim > 3) return "dim must be 1, 2 or 3";
  if (d.p < 0 || d.p > 3) return "p must be in 0..3";
  for (int k = 0; k < 3; ++k) {
    if (k >= d.dim) d.n_elem[k] = 1;
    if (d.n_elem[k] < 1) return "n_elem must be >= 1";
    if (k < d.dim && !(d.hi[k] > d.lo[k])) return "hi must exceed lo";
    if (d.bc[k] != DG_BC_PERIODIC && d.bc[k] != DG_BC_OUTFLOW && d.bc[k] != DG_BC_REFLECT &&
        d.bc[k] != DG_BC_DIRICHLET)
      return "bc must be periodic, outflow, reflect or dirichlet";
    if (k >= d.dim) d.bc_hi[k] = 0;
    if (d.bc_hi[k] != 0 && d.bc_hi[k] != DG_BC_OUTFLOW && d.bc_hi[k] != DG_BC_REFLECT &&
        d.bc_hi[k] != DG_BC_DIRICHLET)
      return "bc_hi must be 0, outflow, reflect or dirichlet";
    if (d.bc[k] == DG_BC_PERIODIC && d.bc_hi[k] != 0) return "a periodic dimension has no separate upper end";
  }
  if (d.eos != DG_EOS_IDEAL && d.eos != DG_EOS_TM) return "unknown eos";
  if (d.eos == DG_EOS_IDEAL && !(d.gamma_ad > 1.0)) return "gamma_ad must exceed 1";
  if (!(d.c_light > 0.0)) return "c_light must be positive";
  if (d.c2p == DG_C2P_DEFAULT) d.c2p = DG_C2P_NEWTON;
  if (d.eos == DG_EOS_IDEAL && d.c2p != DG_C2P_NEWTON && d.c2p != DG_C2P_QUARTIC)
    return "ideal EOS needs the Newton or quartic solver";
  if (d.eos == DG_EOS_TM && d.c2p != DG_C2P_NEWTON && d.c2p != DG_C2P_CUBIC && d.c2p != DG_C2P_BRENT)
    return "TM EOS needs the Newton, cubic or Brent solver";
  if (d.precision != DG_FP64 && d.precision != DG_FP32_CONTRACT && d.precision != DG_FP32_MFMA)
    return "unknown precision";
  if (d.precision == DG_FP32_MFMA && !(d.dim == 2 && d.p == 3)) return "DG_FP32_MFMA is built for dim 2, p 3";
  if (d.flux != DG_FLUX_HLL && d.flux != DG_FLUX_HLLC) return "flux must be HLL or HLLC";
  if (!(d.phys_eps > 0.0)) d.phys_eps = 1e-12;
  if (d.c2p_iters < 0 || d.c2p_iters > 1000) return "c2p_iters must be in 0..1000";
  if (d.limiter != DG_LIMITER_NONE && d.limiter != DG_LIMITER_MINMOD) return "limiter must be none or minmod";
  if (d.p == 0) d.limiter = DG_LIMITER_NONE;
  const long long nelem = (long long)d.n_elem[0] * d.n_elem[1] * d.n_elem[2];
  if (nelem > (1ll << 30)) return "mesh too large";
  s.nv = d.dim + 2;
  s.npe = 1;
  for (int k = 0; k < d.dim; ++k) s.npe *= d.p + 1;
  s.ntot = nelem * s.npe;
  PhysParams& q = s.q;
  q.c = d.c_light;
  q.c2 = q.c * q.c;
  q.c4 = q.c2 * q.c2;
  q.inv_c = 1.0 / q.c;
  q.inv_c2 = 1.0 / q.c2;
  q.gam = d.gamma_ad;
  q.gm1 = d.gamma_ad - 1.0;
  q.alpha = (d.eos == DG_EOS_IDEAL) ? d.gamma_ad / (d.gamma_ad - 1.0) : 0.0;
  q.eps = d.phys_eps;
  q.c2p = d.c2p;
  q.c2p_iters = d.c2p_iters;
  gl_tables(d.p, d.dim, s.t, s.xi);
  {
    // sum over the element's nodes of w_n xi_{d,n}^2: one line's sum times the others' weights
    double den = 0.0, w1 = 0.0;
    double x[kMaxN1];
    for (int i = 0; i <= d.p; ++i) x[i] = 0.5 * (s.xi[i] - s.xi[d.p - i]);  // exact mirror symmetry
    for (int i = 0; i <= d.p; ++i) s.xi[i] = x[i];
    for (int i = 0; i <= d.p; ++i) {
      den += s.t.w[i] * s.xi[i] * s.xi[i];
      w1 += s.t.w[i];
    }
    for (int k = 1; k < d.dim; ++k) den *= w1;
    s.lim_inv_den = den > 0.0 ? 1.0 / den : 0.0;
  }
  MeshArgs& m = s.m;
  m.nex = d.n_elem[0];
  m.ney = d.n_elem[1];
  m.nez = d.n_elem[2];
  m.nelem = (int)nelem;
  m.ntot = s.ntot;
  for (int k = 0; k < 3; ++k) {
    m.two_dx[k] = (k < d.dim) ? 2.0 * d.n_elem[k] / (d.hi[k] - d.lo[k]) : 0.0;
    m.periodic[k] = (d.bc[k] == DG_BC_PERIODIC) ? 1 : 0;
    m.bclo[k] = d.bc[k];
    m.bchi[k] = d.bc_hi[k] != 0 ? d.bc_hi[k] : d.bc[k];
    for (int end = 0; end < 2; ++end) {
      const double* w = d.bc_state[k][end];
      for (int i = 0; i < 5; ++i) m.bw[k][end][i] = 0.0;
      if ((end == 0 ? m.bclo[k] : m.bchi[k]) != DG_BC_DIRICHLET || k >= d.dim) continue;
      double v2 = 0.0;
      for (int j = 0; j < d.dim; ++j) v2 += w[1 + j] * w[1 + j];
      if (!(w[0] > 0.0) || !(w[4] > 0.0) || !(v2 < d.c_light * d.c_light))
        return "a dirichlet end needs rho > 0, P > 0 and |v| < c";
      const double g = 1.0 / std::sqrt(1.0 - v2 / (d.c_light * d.c_light));
      m.bw[k][end][0] = w[0];
      for (int j = 0; j < d.dim; ++j) m.bw[k][end][1 + j] = g * w[1 + j];
      m.bw[k][end][4] = w[4];
    }
  }
  return nullptr;
}

hipError_t launch_element(const MeshSetup& s, int mode, const ElemArgs& a, hipStream_t st) {
  const int dim = s.desc.dim, p = s.desc.p, eos = s.desc.eos, prec = s.desc.precision, fl = s.desc.flux;
  if (dim == 1) return launch_element_dim1(p, eos, prec, mode, fl, a, st);
  if (dim == 2) return launch_element_dim2(p, eos, prec, mode, fl, a, st);
  return launch_element_dim3(p, eos, prec, mode, fl, a, st);
}

// Whether the element kernel of this (dim, p) has the fused right-hand side (its halo
// adds at most one recovery per lane; see TileGeo::kFusedRhs).
template <int DIM>
static bool fused_rhs_dim(int p) {
  switch (p) {
    case 0: return TileGeo<DIM, 0>::kFusedRhs;
    case 1: return TileGeo<DIM, 1>::kFusedRhs;
    case 2: return TileGeo<DIM, 2>::kFusedRhs;
    default: return TileGeo<DIM, 3>::kFusedRhs;
  }
}

bool fused_rhs(const MeshSetup& s) {
  const int dim = s.desc.dim, p = s.desc.p;
  return dim == 1 ? fused_rhs_dim<1>(p) : (dim == 2 ? fused_rhs_dim<2>(p) : fused_rhs_dim<3>(p));
}

hipError_t launch_con2prim(const MeshSetup& s, const double* U, double* W, Counters* cnt, hipStream_t st) {
  const int dim = s.desc.dim, eos = s.desc.eos;
  if (dim == 1) return launch_con2prim_dim1(eos, U, W, s.ntot, s.npe, s.q, cnt, st);
  if (dim == 2) return launch_con2prim_dim2(eos, U, W, s.ntot, s.npe, s.q, cnt, st);
  return launch_con2prim_dim3(eos, U, W, s.ntot, s.npe, s.q, cnt, st);
}

hipError_t L_element(dg_ctx* c, int mode, const ElemArgs& a0) {
  // consecutive launches walk the tiles in opposite directions (cache reuse)
  ElemArgs a = a0;
  c->flip ^= 1;
  a.rev = c->flip;
  return launch_element(*c, mode, a, c->stream);
}

hipError_t L_con2prim(dg_ctx* c, const double* U, double* W) { return launch_con2prim(*c, U, W, c->cnt, c->stream); }

hipError_t L_enforce(dg_ctx* c, double* U) {
  const int dim = c->desc.dim, p = c->desc.p;
  if (dim == 1) return launch_enforce_dim1(p, U, c->m, c->t, c->q, c->cnt, c->stream);
  if (dim == 2) return launch_enforce_dim2(p, U, c->m, c->t, c->q, c->cnt, c->stream);
  return launch_enforce_dim3(p, U, c->m, c->t, c->q, c->cnt, c->stream);
}

hipError_t L_prim3(dg_ctx* c, const double* S, double* U) {
  const int dim = c->desc.dim, eos = c->desc.eos;
  if (dim == 1) return launch_prim3_to_cons_dim1(eos, S, U, c->ntot, c->q, c->cnt, c->stream);
  if (dim == 2) return launch_prim3_to_cons_dim2(eos, S, U, c->ntot, c->q, c->cnt, c->stream);
  return launch_prim3_to_cons_dim3(eos, S, U, c->ntot, c->q, c->cnt, c->stream);
}

// Limiter + operator + recovery (Wout null: no recovery) on U, whose element averages
// the stage launch wrote into c->avg.
hipError_t L_limiter(dg_ctx* c, double* U, double* Wout) {
  LimArgs a{};
  a.U = U;
  a.avg = c->avg;
  a.Wout = Wout;
  for (int i = 0; i < kMaxN1; ++i) a.xi[i] = c->xi[i];
  a.inv_den = c->lim_inv_den;
  a.phys = c->desc.phys;
  a.m = c->m;
  a.t = c->t;
  a.q = c->q;
  a.cnt = c->cnt;
  const int dim = c->desc.dim, p = c->desc.p, eos = c->desc.eos;
  if (dim == 1) return launch_limiter_dim1(p, eos, a, c->stream);
  if (dim == 2) return launch_limiter_dim2(p, eos, a, c->stream);
  return launch_limiter_dim3(p, eos, a, c->stream);
}

ElemArgs base_args(dg_ctx* c) {
  ElemArgs a{};
  a.m = c->m;
  a.t = c->t;
  a.q = c->q;
  a.cnt = c->cnt;
  a.phys = c->desc.phys;
  return a;
}

// After a call: in sync mode wait, then report new device-side conditions.
int finish(dg_ctx* c, const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(c, DG_EHIP, "%s: %s", what, hipGetErrorString(e));
  if (!c->desc.sync_mode) return DG_OK;
  e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return fail(c, DG_EHIP, "%s: %s", what, hipGetErrorString(e));
  Counters now{};
  e = read_counters(c->cnt, now);
  if (e != hipSuccess) return fail(c, DG_EHIP, "%s: %s", what, hipGetErrorString(e));
  const Counters prev = c->last;
  c->last = now;
  if (now.bad_input > prev.bad_input)
    return fail(c, DG_ESTATE, "%s: %llu invalid primitive input nodes", what, now.bad_input - prev.bad_input);
  if (now.c2p_fail > prev.c2p_fail)
    return fail(c, DG_ECON2PRIM, "%s: %llu recovery failures (first element %llu)", what,
                now.c2p_fail - prev.c2p_fail, now.first_bad);
  if (now.bad_average > prev.bad_average)
    return fail(c, DG_EAVERAGE, "%s: %llu elements with inadmissible average", what,
                now.bad_average - prev.bad_average);
  return DG_OK;
}

}  // namespace dgsrhd

extern "C" {

int dg_init_mesh(const dg_mesh_desc* desc, void* hip_stream, dg_ctx** out) {
  if (!out) return DG_EINVAL;
  *out = nullptr;
  if (!desc) return DG_EINVAL;
  dg_ctx* c = new (std::nothrow) dg_ctx();
  if (!c) return DG_ENOMEM;
  const char* why = setup_mesh(desc, *c);
  if (why) {
    std::fprintf(stderr, "dg_init_mesh: %s\n", why);
    delete c;
    return DG_EINVAL;
  }
  c->stream = (hipStream_t)hip_stream;
  const size_t bytes = sizeof(double) * (size_t)c->nv * (size_t)c->ntot;
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = hipMalloc((void**)&c->Wa, bytes);
  if (e == hipSuccess) e = hipMalloc((void**)&c->Wb, bytes);
  if (e == hipSuccess) e = hipMalloc((void**)&c->U1, bytes);
  if (e == hipSuccess) e = hipMalloc((void**)&c->U2, bytes);
  if (e == hipSuccess) e = hipMalloc((void**)&c->cnt, sizeof(Counters) * kCounterSlots);
  if (e == hipSuccess && c->desc.limiter)
    e = hipMalloc((void**)&c->avg, sizeof(double) * (size_t)c->nv * (size_t)c->m.nelem);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&c->handoff, hipEventDisableTiming);
  if (e != hipSuccess) {
    std::fprintf(stderr, "dg_init_mesh: allocation failed: %s\n", hipGetErrorString(e));
    dg_destroy(c);
    return DG_ENOMEM;
  }
  hipLaunchKernelGGL(k_reset_counters, dim3(1), dim3(kCounterSlots), 0, c->stream, c->cnt);
  e = hipGetLastError();
  if (e != hipSuccess) {
    std::fprintf(stderr, "dg_init_mesh: %s\n", hipGetErrorString(e));
    dg_destroy(c);
    return DG_EHIP;
  }
  c->last = Counters{};
  c->last.first_bad = ~0ull;
  *out = c;
  return DG_OK;
}

// Every call of a context shares its scratch (primitive and stage buffers, counters):
// when the stream changes, the new one first waits for what is queued on the old one.
int dg_set_stream(dg_ctx* c, void* hip_stream) {
  if (!c) return DG_EINVAL;
  const hipStream_t s = (hipStream_t)hip_stream;
  if (s == c->stream) return DG_OK;
  int r = hipcheck(c, hipEventRecord(c->handoff, c->stream), "dg_set_stream");
  if (r) return r;
  r = hipcheck(c, hipStreamWaitEvent(s, c->handoff, 0), "dg_set_stream");
  if (r) return r;
  c->stream = s;
  return DG_OK;
}

size_t dg_state_size(const dg_ctx* c) { return c ? (size_t)c->nv * (size_t)c->ntot : 0; }

int dg_set_state(dg_ctx* c, int kind, const double* src, double* U) {
  if (!c) return DG_EINVAL;
  if (!src || !U) return fail(c, DG_EINVAL, "dg_set_state: null pointer");
  if (kind == DG_CONSERVED) {
    const size_t bytes = sizeof(double) * dg_state_size(c);
    int r = hipcheck(c, hipMemcpyAsync(U, src, bytes, hipMemcpyDeviceToDevice, c->stream), "dg_set_state");
    if (r) return r;
  } else if (kind == DG_PRIMITIVE) {
    int r = hipcheck(c, L_prim3(c, src, U), "dg_set_state");
    if (r) return r;
  } else {
    return fail(c, DG_EINVAL, "dg_set_state: unknown kind %d", kind);
  }
  return finish(c, "dg_set_state");
}

int dg_con2prim(dg_ctx* c, const double* U, double* W) {
  if (!c) return DG_EINVAL;
  if (!U || !W) return fail(c, DG_EINVAL, "dg_con2prim: null pointer");
  int r = hipcheck(c, L_con2prim(c, U, W), "dg_con2prim");
  if (r) return r;
  return finish(c, "dg_con2prim");
}

int dg_rhs(dg_ctx* c, const double* U, double* R) {
  if (!c) return DG_EINVAL;
  if (!U || !R) return fail(c, DG_EINVAL, "dg_rhs: null pointer");
  if (U == R) return fail(c, DG_EINVAL, "dg_rhs: U and R alias");
  ElemArgs a = base_args(c);
  a.out = R;
  int r;
  if (fused_rhs(*c)) {
    // one launch: every tile recovers its nodes and its halo elements itself
    a.Uk = U;
    r = hipcheck(c, L_element(c, MODE_RHS_FUSED, a), "dg_rhs/element");
  } else {
    r = hipcheck(c, L_con2prim(c, U, c->Wa), "dg_rhs/con2prim");
    if (r) return r;
    a.W = c->Wa;
    r = hipcheck(c, L_element(c, MODE_RHS, a), "dg_rhs/element");
  }
  if (r) return r;
  return finish(c, "dg_rhs");
}

int dg_enforce_physical(dg_ctx* c, double* U) {
  if (!c) return DG_EINVAL;
  if (!U) return fail(c, DG_EINVAL, "dg_enforce_physical: null pointer");
  int r = hipcheck(c, L_enforce(c, U), "dg_enforce_physical");
  if (r) return r;
  return finish(c, "dg_enforce_physical");
}

// SSP Runge-Kutta steps in Shu-Osher form (Sec. 2.3): every stage is
// U^(k+1) = Pi(ca U^n + cb (U^(k) + dt L(U^(k)))), one fused launch per stage.
// order 1: forward Euler; 2: the second-order SSP scheme (1/2, 1/2);
// 3: the third-order SSP scheme (3/4, 1/4; 1/3, 2/3).
// The last stage's U^n term is folded into the stage before it: that stage stores
// Z = ca U^n + cb U^(k) (with the last stage's weights) in place of U^(k), whose
// primitives it still writes, and the last stage forms Z + cb dt L(U^(k)) reading
// only Z, one state read fewer per step.
// With the slope limiter a stage is U^(k+1) = Pi(Lim(ca U^n + cb (U^(k) + dt L))):
// the stage launch writes the unlimited combination, its element averages and its
// primitives (no operator, no folding, since Lim needs the neighbours' averages of
// the finished stage), then the limiter launch finishes it, rewriting U and W only
// where it or the operator changed a node.
static int ssprk_steps(dg_ctx* c, double* U, double dt, int nsteps, int order, const char* what) {
  if (!c) return DG_EINVAL;
  if (!U) return fail(c, DG_EINVAL, "%s: null pointer", what);
  if (nsteps < 0) return fail(c, DG_EINVAL, "%s: nsteps < 0", what);
  if (order < 1 || order > 3) return fail(c, DG_EINVAL, "%s: order must be 1, 2 or 3", what);
  if (!std::isfinite(dt)) return fail(c, DG_EINVAL, "%s: dt not finite", what);
  if (nsteps == 0) return DG_OK;
  struct Stage {
    double ca, cb, dtf;  // U^(k+1) = ca U^n + cb (U^(k) + dtf dt L)
    double za, zb;       // stored: za U^n + zb U^(k+1) when za != 0
    double* in;
    double* out;
  };
  const Stage tab1[1] = {{0.0, 1.0, 1.0, 0.0, 0.0, U, U}};
  const Stage tab2[2] = {{0.0, 1.0, 1.0, 0.5, 0.5, U, c->U1}, {0.0, 1.0, 0.5, 0.0, 0.0, c->U1, U}};
  const Stage tab3[3] = {{0.0, 1.0, 1.0, 0.0, 0.0, U, c->U1},
                         {0.75, 0.25, 1.0, 1.0 / 3.0, 2.0 / 3.0, c->U1, c->U2},
                         {0.0, 1.0, 2.0 / 3.0, 0.0, 0.0, c->U2, U}};
  // the Shu-Osher weights as they stand (limiter)
  const Stage lim2[2] = {{0.0, 1.0, 1.0, 0.0, 0.0, U, c->U1}, {0.5, 0.5, 1.0, 0.0, 0.0, c->U1, U}};
  const Stage lim3[3] = {{0.0, 1.0, 1.0, 0.0, 0.0, U, c->U1},
                         {0.75, 0.25, 1.0, 0.0, 0.0, c->U1, c->U2},
                         {1.0 / 3.0, 2.0 / 3.0, 1.0, 0.0, 0.0, c->U2, U}};
  const bool lim = c->desc.limiter != DG_LIMITER_NONE;
  const Stage* tab = order == 1 ? tab1 : (order == 2 ? (lim ? lim2 : tab2) : (lim ? lim3 : tab3));
  double* Wa = c->Wa;
  double* Wb = c->Wb;
  int r = hipcheck(c, L_con2prim(c, U, Wa), what);
  if (r) return r;
  for (int s = 0; s < nsteps; ++s) {
    for (int k = 0; k < order; ++k) {
      ElemArgs a = base_args(c);
      a.dt = dt * tab[k].dtf;
      a.W = Wa;
      a.Uk = tab[k].in;
      a.Un = U;
      a.ca = tab[k].ca;
      a.cb = tab[k].cb;
      a.za = tab[k].za;
      a.zb = tab[k].zb;
      a.out = tab[k].out;
      const bool last = (s == nsteps - 1) && (k == order - 1);
      if (lim) {
        a.phys = 0;
        a.Wout = last ? nullptr : Wb;
        a.avg = c->avg;
        if ((r = hipcheck(c, L_element(c, MODE_STAGE_LIM, a), what))) return r;
        if ((r = hipcheck(c, L_limiter(c, tab[k].out, last ? nullptr : Wb), what))) return r;
      } else {
        a.Wout = last ? nullptr : Wb;
        if ((r = hipcheck(c, L_element(c, MODE_STAGE, a), what))) return r;
      }
      double* tmp = Wa; Wa = Wb; Wb = tmp;
    }
  }
  return finish(c, what);
}

int dg_ssprk3_step(dg_ctx* c, double* U, double dt) { return ssprk_steps(c, U, dt, 1, 3, "dg_ssprk3_step"); }

int dg_ssprk3_run(dg_ctx* c, double* U, double dt, int nsteps) {
  return ssprk_steps(c, U, dt, nsteps, 3, "dg_ssprk3_run");
}

int dg_ssprk_step(dg_ctx* c, double* U, double dt, int order) {
  return ssprk_steps(c, U, dt, 1, order, "dg_ssprk_step");
}

int dg_ssprk_run(dg_ctx* c, double* U, double dt, int nsteps, int order) {
  return ssprk_steps(c, U, dt, nsteps, order, "dg_ssprk_run");
}

int dg_get_diagnostics(dg_ctx* c, dg_diag* out) {
  if (!c) return DG_EINVAL;
  if (!out) return fail(c, DG_EINVAL, "dg_get_diagnostics: null pointer");
  int r = hipcheck(c, hipStreamSynchronize(c->stream), "dg_get_diagnostics");
  if (r) return r;
  Counters h{};
  r = hipcheck(c, read_counters(c->cnt, h), "dg_get_diagnostics");
  if (r) return r;
  to_diag(h, out);
  return DG_OK;
}

int dg_reset_diagnostics(dg_ctx* c) {
  if (!c) return DG_EINVAL;
  hipLaunchKernelGGL(k_reset_counters, dim3(1), dim3(kCounterSlots), 0, c->stream, c->cnt);
  int r = hipcheck(c, hipGetLastError(), "dg_reset_diagnostics");
  if (r) return r;
  c->last = Counters{};
  c->last.first_bad = ~0ull;
  return finish(c, "dg_reset_diagnostics");
}

const char* dg_last_error(const dg_ctx* c) { return c ? c->err.c_str() : kNoCtx; }

void dg_destroy(dg_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  (void)hipFree(c->Wa);
  (void)hipFree(c->Wb);
  (void)hipFree(c->U1);
  (void)hipFree(c->U2);
  (void)hipFree(c->adj);
  (void)hipFree(c->avg);
  (void)hipFree(c->cnt);
  if (c->handoff) (void)hipEventDestroy(c->handoff);
  delete c;
}

}  // extern "C"

// ------------------------------------------------------------------ dg_rhs_noalloc
// Device scratch of the allocation-free right-hand side: the counter slots at offset
// 0, the primitive staging buffer from kNoAllocWOffset.  Every GPU the library runs on
// holds its own copy until the process ends.  In host code the array's name is only a
// host-side stand-in: kernels and copies take the device address resolved per device
// by hipGetSymbolAddress (noalloc_scratch), never the name itself.
constexpr size_t kNoAllocBytes = 64ull << 20;
constexpr size_t kNoAllocWOffset = 64ull << 10;
static_assert(sizeof(dgsrhd::Counters) * dgsrhd::kCounterSlots <= kNoAllocWOffset, "counters fit before W");
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {
constexpr int kNoAllocMaxDevices = 64;
void* g_noalloc_ptr[kNoAllocMaxDevices];
std::mutex g_noalloc_mu;

// Device address of `scratch` on the current device, resolved on the first call on
// that device (with it current) and kept.
hipError_t noalloc_scratch(unsigned char** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kNoAllocMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (g_noalloc_ptr[dev] == nullptr) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (p == nullptr) return hipErrorInvalidSymbol;
    g_noalloc_ptr[dev] = p;
  }
  *out = static_cast<unsigned char*>(g_noalloc_ptr[dev]);
  return hipSuccess;
}

int noalloc_fail(int code, const char* fmt, ...) {
  char buf[256];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  std::fprintf(stderr, "dg_rhs_noalloc: %s\n", buf);
  return code;
}
}  // namespace

static_assert(DG_RHS_NOALLOC_MAX_STATE == (kNoAllocBytes - kNoAllocWOffset) / sizeof(double),
              "the header's limit is the staging part of the scratch");

extern "C" int dg_rhs_noalloc(const dg_mesh_desc* desc, void* hip_stream, const double* U, double* R,
                              dg_diag* diag) {
  if (!desc) return noalloc_fail(DG_EINVAL, "null description");
  MeshSetup s;
  const char* why = setup_mesh(desc, s);
  if (why) return noalloc_fail(DG_EINVAL, "%s", why);
  if (!U || !R) return noalloc_fail(DG_EINVAL, "null pointer");
  if (U == R) return noalloc_fail(DG_EINVAL, "U and R alias");
  // the same kernels as dg_rhs: one fused launch, or (3D, p >= 1) a recovery launch
  // staging the primitives in the scratch and the element kernel reading them
  const bool fused = fused_rhs(s);
  const size_t need = (size_t)s.nv * (size_t)s.ntot;
  if (!fused && need > (size_t)DG_RHS_NOALLOC_MAX_STATE)
    return noalloc_fail(DG_EINVAL, "the mesh needs %zu doubles of primitive staging; the static scratch holds %zu",
                        need, (size_t)DG_RHS_NOALLOC_MAX_STATE);
  unsigned char* base = nullptr;
  hipError_t e = noalloc_scratch(&base);
  if (e != hipSuccess) return noalloc_fail(DG_EHIP, "scratch address: %s", hipGetErrorString(e));
  Counters* cnt = reinterpret_cast<Counters*>(base);
  double* W = reinterpret_cast<double*>(base + kNoAllocWOffset);
  const hipStream_t st = (hipStream_t)hip_stream;
  // the counters start at zero on every call (a kernel, not a memset node)
  hipLaunchKernelGGL(k_reset_counters, dim3(1), dim3(kCounterSlots), 0, st, cnt);
  e = hipGetLastError();
  if (e == hipSuccess && !fused) e = launch_con2prim(s, U, W, cnt, st);
  if (e == hipSuccess) {
    ElemArgs a{};
    a.m = s.m;
    a.t = s.t;
    a.q = s.q;
    a.cnt = cnt;
    a.phys = s.desc.phys;
    a.out = R;
    if (fused) {
      a.Uk = U;
      e = launch_element(s, MODE_RHS_FUSED, a, st);
    } else {
      a.W = W;
      e = launch_element(s, MODE_RHS, a, st);
    }
  }
  if (e != hipSuccess) return noalloc_fail(DG_EHIP, "launch: %s", hipGetErrorString(e));
  if (!diag && !s.desc.sync_mode) return DG_OK;
  e = hipStreamSynchronize(st);
  Counters h{};
  if (e == hipSuccess) e = read_counters(cnt, h);
  if (e != hipSuccess) return noalloc_fail(DG_EHIP, "counters: %s", hipGetErrorString(e));
  if (diag) to_diag(h, diag);
  if (s.desc.sync_mode && h.c2p_fail > 0)
    return noalloc_fail(DG_ECON2PRIM, "%llu recovery failures (first element %llu)", h.c2p_fail, h.first_bad);
  return DG_OK;
}
