// Host side of the adjoint entry points: dg_rhs_vjp, the taped SSP-RK3 step and
// its vector-Jacobian product, the v_y^2 objective and the initial-data adjoint.
#include <hip/hip_runtime.h>

#include <cstring>

#include "ctx.hpp"
#include "launch_adj.hpp"

using namespace dgsrhd;

namespace {

size_t state_doubles(const dg_ctx* c) { return (size_t)c->nv * (size_t)c->ntot; }
int obj_blocks(const dg_ctx* c) { return (int)((c->ntot + 255) / 256); }

// A tape: W(U^n), W(U1), W(U2), the three pre-operator stage outputs, then a
// flag block (kTapeFlagDoubles doubles, keeping later tapes 256-byte aligned)
// whose first three unsigned ints say whether the operator changed an element in
// stage 1, 2, 3.
constexpr size_t kTapeFlagDoubles = 32;
size_t tape_doubles(const dg_ctx* c) { return 6 * state_doubles(c) + kTapeFlagDoubles; }
unsigned* tape_flags(double* tape, const dg_ctx* c) { return (unsigned*)(tape + 6 * state_doubles(c)); }
const unsigned* tape_flags(const double* tape, const dg_ctx* c) {
  return (const unsigned*)(tape + 6 * state_doubles(c));
}

// Adjoint scratch: Utmp, one tape, mu_a, mu_b, lamn, then objective partials.
enum { A_UTMP = 0, A_TAPE = 1, A_MUA = 2, A_MUB = 3, A_LAMN = 4 };

size_t adj_offset(const dg_ctx* c, int k) {
  const size_t S = state_doubles(c);
  return k == A_UTMP ? 0 : (k == A_TAPE ? S : S + tape_doubles(c) + (size_t)(k - A_MUA) * S);
}

int ensure_adj(dg_ctx* c) {
  const size_t need = adj_offset(c, A_LAMN) + state_doubles(c) + (size_t)obj_blocks(c) + 8;
  if (c->adj && c->adj_doubles >= need) return DG_OK;
  if (c->adj) {
    int r = hipcheck(c, hipStreamSynchronize(c->stream), "adjoint scratch");
    if (r) return r;
    (void)hipFree(c->adj);
    c->adj = nullptr;
  }
  if (hipMalloc((void**)&c->adj, need * sizeof(double)) != hipSuccess) {
    c->adj = nullptr;
    return fail(c, DG_ENOMEM, "adjoint scratch allocation (%zu doubles) failed", need);
  }
  c->adj_doubles = need;
  return DG_OK;
}

double* adj_state(dg_ctx* c, int k) { return c->adj + adj_offset(c, k); }
double* adj_partials(dg_ctx* c) { return c->adj + adj_offset(c, A_LAMN) + state_doubles(c); }

// Clears the operator flags of nsteps consecutive tapes (a kernel, so that a
// captured sequence holds no memset node).
__global__ void k_clear_tape_flags(double* tapes, long long tape_stride, long long flag_offset, int nsteps) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < nsteps) {
    unsigned* f = (unsigned*)(tapes + (long long)s * tape_stride + flag_offset);
    f[0] = f[1] = f[2] = 0u;
  }
}

hipError_t clear_tape_flags(dg_ctx* c, double* tapes, int nsteps) {
  if (nsteps <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_clear_tape_flags, dim3((nsteps + 255) / 256), dim3(256), 0, c->stream, tapes,
                     (long long)tape_doubles(c), (long long)(6 * state_doubles(c)), nsteps);
  return hipGetLastError();
}

hipError_t L_vjp(dg_ctx* c, int mode, const VjpArgs& a) {
  const int dim = c->desc.dim, p = c->desc.p, eos = c->desc.eos;
  const int fl = c->desc.flux;
  if (dim == 1) return launch_vjp_dim1(p, eos, mode, fl, a, c->stream);
  if (dim == 2) return launch_vjp_dim2(p, eos, mode, fl, a, c->stream);
  return launch_vjp_dim3(p, eos, mode, fl, a, c->stream);
}

hipError_t L_enforce_vjp(dg_ctx* c, const double* Pst, const double* lin, double* lout, const unsigned* flag) {
  const int dim = c->desc.dim, p = c->desc.p;
  if (dim == 1) return launch_enforce_vjp_dim1(p, Pst, lin, lout, flag, c->m, c->t, c->q, c->stream);
  if (dim == 2) return launch_enforce_vjp_dim2(p, Pst, lin, lout, flag, c->m, c->t, c->q, c->stream);
  return launch_enforce_vjp_dim3(p, Pst, lin, lout, flag, c->m, c->t, c->q, c->stream);
}

VjpArgs vjp_args(dg_ctx* c) {
  VjpArgs a{};
  a.m = c->m;
  a.t = c->t;
  a.q = c->q;
  return a;
}

__global__ void k_sum_partials(const double* partial, int n, double* out) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) acc += partial[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

// One forward step in place, recording (W(U^n), W(U1), W(U2), P1, P2, P3).  When
// have_w0 is set, W(U^n) is already in the tape (written by the previous step);
// next_w0, if not null, receives W(U^{n+1}) from the last stage's epilogue.
int step_tape(dg_ctx* c, double* U, double dt, double* tape, const char* what, bool have_w0 = false,
              double* next_w0 = nullptr) {
  const size_t S = state_doubles(c);
  double* W0 = tape;
  double* W1 = tape + S;
  double* W2 = tape + 2 * S;
  double* P1 = tape + 3 * S;
  double* P2 = tape + 4 * S;
  double* P3 = tape + 5 * S;
  unsigned* flags = tape_flags(tape, c);  // cleared by the caller
  int r;
  if (!have_w0 && (r = hipcheck(c, L_con2prim(c, U, W0), what))) return r;
  ElemArgs a = base_args(c);
  a.dt = dt;
  a.W = W0; a.Uk = U; a.Un = U; a.ca = 0.0; a.cb = 1.0; a.out = c->U1; a.Wout = W1; a.Pout = P1;
  a.opflag = flags;
  if ((r = hipcheck(c, L_element(c, MODE_STAGE, a), what))) return r;
  a.W = W1; a.Uk = c->U1; a.ca = 0.75; a.cb = 0.25; a.out = c->U2; a.Wout = W2; a.Pout = P2;
  a.opflag = flags + 1;
  if ((r = hipcheck(c, L_element(c, MODE_STAGE, a), what))) return r;
  a.W = W2; a.Uk = c->U2; a.ca = 1.0 / 3.0; a.cb = 2.0 / 3.0; a.out = U; a.Wout = next_w0; a.Pout = P3;
  a.opflag = flags + 2;
  return hipcheck(c, L_element(c, MODE_STAGE, a), what);
}

// Reverse of one taped step: lam_n = (dU^{n+1}/dU^n)^T lam_next.  In a reverse sweep
// over consecutive steps, pre_applied says that lam_next is already the adjoint of this
// step's last pre-operator state (the operator's adjoint was fused into the next step's
// first reverse stage), and prev_tape, when given, is the previous step's tape, whose
// last operator's adjoint is fused into this step's first reverse stage (so lam_n is
// then the adjoint of that step's last pre-operator state).
int step_vjp_tape(dg_ctx* c, const double* tape, double dt, const double* lam_next, double* lam_n,
                  const char* what, bool pre_applied = false, const double* prev_tape = nullptr) {
  const size_t S = state_doubles(c);
  const double* W0 = tape;
  const double* W1 = tape + S;
  const double* W2 = tape + 2 * S;
  const double* P1 = tape + 3 * S;
  const double* P2 = tape + 4 * S;
  const double* P3 = tape + 5 * S;
  double* mua = adj_state(c, A_MUA);
  double* mub = adj_state(c, A_MUB);
  double* lamn = adj_state(c, A_LAMN);
  const unsigned* flags = tape_flags(tape, c);  // operator active in stages 1, 2, 3 of the forward step
  const bool phys = c->desc.phys != 0;
  int r;
  VjpArgs a = vjp_args(c);
  a.dt = dt;
  // the operator after stage 3, when it acted: mua = Pi'(P3)^T lam_next (else
  // nothing is written and stage 3 reads lam_next)
  a.lam = lam_next;
  if (phys && !pre_applied) {
    if ((r = hipcheck(c, L_enforce_vjp(c, P3, lam_next, mua, flags + 2), what))) return r;
    a.lam_alt = mua;
    a.lam_sel = flags + 2;
  }
  // stage 3: U^{n+1} = Pi(1/3 U^n + 2/3 (U2 + dt R(U2)))
  a.W = W2; a.out = mub; a.lamn = lamn; a.lamn_init = 1;
  a.ca = 1.0 / 3.0; a.cb = 2.0 / 3.0; a.Pprev = phys ? P2 : nullptr; a.pflag = flags + 1;
  if ((r = hipcheck(c, L_vjp(c, VJP_STAGE, a), what))) return r;
  // stage 2: U2 = Pi(3/4 U^n + 1/4 (U1 + dt R(U1)))
  double* mu1 = mua;  // mu3 (mua or lam_next) is no longer read
  a.lam_alt = nullptr;
  a.lam_sel = nullptr;
  a.W = W1; a.lam = mub; a.out = mu1; a.lamn_init = 0; a.ca = 0.75; a.cb = 0.25; a.Pprev = phys ? P1 : nullptr;
  a.pflag = flags;
  if ((r = hipcheck(c, L_vjp(c, VJP_STAGE, a), what))) return r;
  // stage 1: U1 = Pi(U^n + dt R(U^n)); U^n = Pi(P3 of the previous step) when prev_tape is given
  a.W = W0; a.lam = mu1; a.out = lam_n; a.ca = 0.0; a.cb = 1.0; a.Pprev = nullptr; a.pflag = nullptr;
  if (phys && prev_tape) {
    a.Ppost = prev_tape + 5 * S;
    a.postflag = tape_flags(prev_tape, c) + 2;
  }
  return hipcheck(c, L_vjp(c, VJP_STAGE, a), what);
}

// The stepping adjoints differentiate the stage without the slope limiter.
int reject_limiter(dg_ctx* c, const char* what) {
  if (c->desc.limiter != DG_LIMITER_NONE)
    return fail(c, DG_EINVAL, "%s: the slope limiter has no adjoint here", what);
  return DG_OK;
}

}  // namespace

extern "C" {

int dg_rhs_vjp(dg_ctx* c, const double* U, const double* lamR, double* lamU) {
  if (!c) return DG_EINVAL;
  if (!U || !lamR || !lamU) return fail(c, DG_EINVAL, "dg_rhs_vjp: null pointer");
  if (lamU == lamR || lamU == U) return fail(c, DG_EINVAL, "dg_rhs_vjp: output aliases an input");
  int r = hipcheck(c, L_con2prim(c, U, c->Wa), "dg_rhs_vjp/con2prim");
  if (r) return r;
  VjpArgs a = vjp_args(c);
  a.W = c->Wa;
  a.lam = lamR;
  a.out = lamU;
  if ((r = hipcheck(c, L_vjp(c, VJP_PLAIN, a), "dg_rhs_vjp"))) return r;
  return finish(c, "dg_rhs_vjp");
}

size_t dg_tape_size(const dg_ctx* c) { return c ? tape_doubles(c) : 0; }

int dg_ssprk3_step_tape(dg_ctx* c, double* U, double dt, double* tape) {
  if (!c) return DG_EINVAL;
  if (int rl = reject_limiter(c, "dg_ssprk3_step_tape")) return rl;
  if (!U || !tape) return fail(c, DG_EINVAL, "dg_ssprk3_step_tape: null pointer");
  int r = hipcheck(c, clear_tape_flags(c, tape, 1), "dg_ssprk3_step_tape");
  if (r) return r;
  r = step_tape(c, U, dt, tape, "dg_ssprk3_step_tape");
  if (r) return r;
  return finish(c, "dg_ssprk3_step_tape");
}

int dg_ssprk3_step_vjp_tape(dg_ctx* c, const double* tape, double dt, const double* lam_next, double* lam_n) {
  if (!c) return DG_EINVAL;
  if (int rl = reject_limiter(c, "dg_ssprk3_step_vjp_tape")) return rl;
  if (!tape || !lam_next || !lam_n) return fail(c, DG_EINVAL, "dg_ssprk3_step_vjp_tape: null pointer");
  int r = ensure_adj(c);
  if (r) return r;
  if ((r = step_vjp_tape(c, tape, dt, lam_next, lam_n, "dg_ssprk3_step_vjp_tape"))) return r;
  return finish(c, "dg_ssprk3_step_vjp_tape");
}

int dg_ssprk3_run_tape(dg_ctx* c, double* U, double dt, int nsteps, double* tapes) {
  if (!c) return DG_EINVAL;
  if (int rl = reject_limiter(c, "dg_ssprk3_run_tape")) return rl;
  if (!U || !tapes) return fail(c, DG_EINVAL, "dg_ssprk3_run_tape: null pointer");
  if (nsteps < 0) return fail(c, DG_EINVAL, "dg_ssprk3_run_tape: nsteps < 0");
  const size_t T = tape_doubles(c);
  int r0 = hipcheck(c, clear_tape_flags(c, tapes, nsteps), "dg_ssprk3_run_tape");
  if (r0) return r0;
  for (int s = 0; s < nsteps; ++s) {
    double* next_w0 = (s + 1 < nsteps) ? tapes + (size_t)(s + 1) * T : nullptr;
    int r = step_tape(c, U, dt, tapes + (size_t)s * T, "dg_ssprk3_run_tape", s > 0, next_w0);
    if (r) return r;
  }
  return finish(c, "dg_ssprk3_run_tape");
}

int dg_ssprk3_run_vjp_tape(dg_ctx* c, const double* tapes, double dt, int nsteps, double* lam) {
  if (!c) return DG_EINVAL;
  if (int rl = reject_limiter(c, "dg_ssprk3_run_vjp_tape")) return rl;
  if (!tapes || !lam) return fail(c, DG_EINVAL, "dg_ssprk3_run_vjp_tape: null pointer");
  if (nsteps < 0) return fail(c, DG_EINVAL, "dg_ssprk3_run_vjp_tape: nsteps < 0");
  int r = ensure_adj(c);
  if (r) return r;
  const size_t T = tape_doubles(c);
  for (int s = nsteps - 1; s >= 0; --s) {
    const double* prev = s > 0 ? tapes + (size_t)(s - 1) * T : nullptr;
    if ((r = step_vjp_tape(c, tapes + (size_t)s * T, dt, lam, lam, "dg_ssprk3_run_vjp_tape", s < nsteps - 1, prev)))
      return r;
  }
  return finish(c, "dg_ssprk3_run_vjp_tape");
}

int dg_ssprk3_step_vjp(dg_ctx* c, const double* Un, double dt, const double* lam_next, double* lam_n) {
  if (!c) return DG_EINVAL;
  if (int rl = reject_limiter(c, "dg_ssprk3_step_vjp")) return rl;
  if (!Un || !lam_next || !lam_n) return fail(c, DG_EINVAL, "dg_ssprk3_step_vjp: null pointer");
  int r = ensure_adj(c);
  if (r) return r;
  double* Ut = adj_state(c, A_UTMP);
  double* tape = adj_state(c, A_TAPE);
  r = hipcheck(c, hipMemcpyAsync(Ut, Un, state_doubles(c) * sizeof(double), hipMemcpyDeviceToDevice, c->stream),
               "dg_ssprk3_step_vjp");
  if (r) return r;
  if ((r = hipcheck(c, clear_tape_flags(c, tape, 1), "dg_ssprk3_step_vjp"))) return r;
  if ((r = step_tape(c, Ut, dt, tape, "dg_ssprk3_step_vjp"))) return r;
  if ((r = step_vjp_tape(c, tape, dt, lam_next, lam_n, "dg_ssprk3_step_vjp"))) return r;
  return finish(c, "dg_ssprk3_step_vjp");
}

int dg_objective_vy2(dg_ctx* c, const double* U, double* J_host, double* dJdU) {
  if (!c) return DG_EINVAL;
  if (!U || !J_host) return fail(c, DG_EINVAL, "dg_objective_vy2: null pointer");
  int r = ensure_adj(c);
  if (r) return r;
  const int nb = obj_blocks(c);
  double* partial = adj_partials(c);
  double* Jdev = partial + nb;
  double jac = 1.0;
  for (int d = 0; d < c->desc.dim; ++d) jac *= 1.0 / c->m.two_dx[d];  // prod dx_d / 2
  const int dim = c->desc.dim, eos = c->desc.eos, n1 = c->desc.p + 1;
  hipError_t e;
  if (dim == 1) e = launch_objective_dim1(eos, U, partial, dJdU, c->ntot, c->npe, n1, c->t, jac, c->q, nb, c->stream);
  else if (dim == 2)
    e = launch_objective_dim2(eos, U, partial, dJdU, c->ntot, c->npe, n1, c->t, jac, c->q, nb, c->stream);
  else e = launch_objective_dim3(eos, U, partial, dJdU, c->ntot, c->npe, n1, c->t, jac, c->q, nb, c->stream);
  if ((r = hipcheck(c, e, "dg_objective_vy2"))) return r;
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, c->stream, partial, nb, Jdev);
  if ((r = hipcheck(c, hipGetLastError(), "dg_objective_vy2"))) return r;
  if ((r = hipcheck(c, hipMemcpyAsync(J_host, Jdev, sizeof(double), hipMemcpyDeviceToHost, c->stream),
                    "dg_objective_vy2")))
    return r;
  if ((r = hipcheck(c, hipStreamSynchronize(c->stream), "dg_objective_vy2"))) return r;
  return finish(c, "dg_objective_vy2");
}

int dg_set_state_vjp(dg_ctx* c, const double* src, const double* lamU, double* lamS) {
  if (!c) return DG_EINVAL;
  if (!src || !lamU || !lamS) return fail(c, DG_EINVAL, "dg_set_state_vjp: null pointer");
  const int dim = c->desc.dim, eos = c->desc.eos;
  hipError_t e;
  if (dim == 1) e = launch_prim3_vjp_dim1(eos, src, lamU, lamS, c->ntot, c->q, c->stream);
  else if (dim == 2) e = launch_prim3_vjp_dim2(eos, src, lamU, lamS, c->ntot, c->q, c->stream);
  else e = launch_prim3_vjp_dim3(eos, src, lamU, lamS, c->ntot, c->q, c->stream);
  int r = hipcheck(c, e, "dg_set_state_vjp");
  if (r) return r;
  return finish(c, "dg_set_state_vjp");
}

}  // extern "C"
