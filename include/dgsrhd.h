/*
 * dgsrhd — C ABI of the MI355X (gfx950) discontinuous-Galerkin special-relativistic
 * hydrodynamics hot path (Glines et al., "A Robust, Performance-Portable
 * Discontinuous Galerkin Method for Relativistic Hydrodynamics").
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Layout.  Every nodal array is FP64, C order
 *     [n_var][n_ez][n_ey][n_ex][nk][nj][ni]        (x node index i fastest)
 * with n_var = dim + 2 and unused dimensions of extent 1, so one element's
 * (p+1)^dim nodes of one component are contiguous.
 *   conserved:  (D, S_1..S_dim, tau)   S = M the momentum density (Sec. 2.1),
 *               tau = E - D c^2 (the energy minus the rest mass);
 *   primitive input of dg_set_state: (rho, v_1..v_dim, P), v the 3-velocity;
 *   primitive output of dg_con2prim:  (rho, u_1..u_dim, P), u = gamma v (Sec. 2.1).
 * Ownership.  Every pointer argument ending in _dev is a device pointer owned by
 * the caller (typically a torch tensor); the library only borrows it for the
 * stream-ordered duration of the call and never frees or retains it.  The
 * context owns its scratch buffers (stage states, primitive buffers, counters).
 * Streams.  All work is enqueued on the stream given to dg_init_mesh (or
 * dg_set_stream) and is asynchronous: the return code reports argument and
 * launch errors only.  Device-detected conditions (recovery failures, smoothed
 * elements, ...) accumulate in counters read by dg_get_diagnostics, which
 * synchronises the stream.  With desc.sync_mode = 1 every call synchronises and
 * also returns DG_ECON2PRIM / DG_EAVERAGE / DG_ESTATE when a counter grew.
 * Errors.  No exception or exit() crosses the ABI; negative codes below, the
 * message of the last failure from dg_last_error.  Calls that overlap on one
 * context from several host threads race; use one context per thread.
 */
#ifndef DGSRHD_H
#define DGSRHD_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dg_ctx dg_ctx;

enum {
  DG_OK = 0,
  DG_EINVAL = -1,       /* bad argument (null pointer, unsupported size, ...) */
  DG_ENOMEM = -2,       /* scratch allocation failed */
  DG_EHIP = -3,         /* HIP runtime error (launch, copy, sync) */
  DG_ECON2PRIM = -4,    /* >= 1 node had an inadmissible U (D <= 0 or q <= 0) or no root */
  DG_EAVERAGE = -5,     /* >= 1 flagged element had an inadmissible volume average */
  DG_ESTATE = -6        /* dg_set_state input had rho <= 0, P <= 0, |v| >= c or NaN */
};
enum { DG_BC_PERIODIC = 0, DG_BC_OUTFLOW = 1, DG_BC_REFLECT = 2, DG_BC_DIRICHLET = 3 };
enum { DG_EOS_IDEAL = 0, DG_EOS_TM = 1 };
enum { DG_C2P_DEFAULT = -1, DG_C2P_NEWTON = 0, DG_C2P_QUARTIC = 1, DG_C2P_CUBIC = 2, DG_C2P_BRENT = 3 };
enum { DG_FP64 = 0, DG_FP32_CONTRACT = 1, DG_FP32_MFMA = 2 };
enum { DG_FLUX_HLL = 0, DG_FLUX_HLLC = 1 };
enum { DG_LIMITER_NONE = 0, DG_LIMITER_MINMOD = 1 };
enum { DG_CONSERVED = 0, DG_PRIMITIVE = 1 };

/* Mesh and method description.  Cartesian mesh of n_elem[d] equal elements on
 * [lo[d], hi[d]] (Sec. 2.3), tensor-product Lagrange basis of order p on
 * Gauss-Legendre nodes with collocated quadrature (supported: dim 1..3,
 * p 0..3).  bc[d] is the boundary of dimension d: periodic, outflow (the
 * exterior state at a boundary face is the interior trace), a reflecting wall
 * (the interior trace with its velocity component along d negated) or Dirichlet
 * (a fixed exterior state), the boundaries of the Riemann problems of Sec. 4.
 * bc[d] applies to both ends unless bc_hi[d] (0 keeps bc[d]) names another
 * non-periodic type for the upper end.  A Dirichlet end takes its exterior state
 * from bc_state[d][end] = (rho, v_x, v_y, v_z, P), end 0 the lower, 1 the upper,
 * v the 3-velocity (components beyond dim ignored); dg_init_mesh returns DG_EINVAL
 * unless rho > 0, P > 0 and |v| < c there.  eos / gamma_ad /
 * c_light select the equation of state (Sec. 2.2).  c2p selects the recovery
 * solver of Sec. 3: ideal EOS NEWTON (Newton on the quartic in w, the default;
 * inside an SSP-RK stage started from the node's root of the previous stage,
 * elsewhere from the beta_max bound) or QUARTIC (analytic); TM EOS CUBIC (analytic root of the cubic plus one Newton
 * step), BRENT (bracketed iteration) or NEWTON (the default: inside an SSP-RK
 * stage, three Newton steps on the same cubic started from the node's primitives
 * of the previous stage and accepted only when converged on the physical root,
 * else the CUBIC result; outside a stage the same three steps started from the
 * closed-form root evaluated in FP32, accepted likewise).  precision = DG_FP32_CONTRACT
 * evaluates the volume (D-hat) and lift contractions in FP32 with FP32
 * accumulation, on deviations from an FP64 reference per line of nodes; the face
 * traces, the recovery, the fluxes, the numerical flux, the operator and the RK
 * combine stay FP64.  precision = DG_FP32_MFMA (dim 2, p 3 only; DG_EINVAL
 * elsewhere) is the same form with the volume sweeps on the matrix cores
 * (v_mfma_f32_4x4x1f32, FP32 accumulation).  phys = 1 applies
 * the physicality-enforcing operator (Sec. 2.5) after every SSP-RK stage, with
 * relative margin phys_eps (0 selects 1e-12).  flux selects the numerical flux at
 * the faces (Sec. 2.4): DG_FLUX_HLL (0, the default when the field is zeroed) or
 * DG_FLUX_HLLC, the HLLC solver of Mignone & Bodo (2005) with one contact wave
 * inside the HLL fan (exact on isolated contacts, including tangential-velocity
 * jumps); the adjoint entry points differentiate whichever flux is selected.
 * c2p_iters (0: off) fixes the iteration count of the iterative recovery solvers
 * for the recovery study of Sec. 3.3: with the ideal EOS exactly c2p_iters Newton
 * steps started from w = 1/2, the middle of the interval every start converges from
 * (no convergence test), with the TM EOS and c2p = BRENT at most c2p_iters Brent
 * steps on the bracket [0, 200^2 - 1]; no failure is counted for stopping there.  Valid
 * range 0..1000 (DG_EINVAL outside).
 * limiter = DG_LIMITER_MINMOD (p >= 1; ignored at p = 0) applies the slope limiter the
 * paper pairs with the operator for its p >= 1 shock runs (Sec. 2.3 names the minmod
 * limiter of van Leer 1979 and the scaling limiter of Moe, Rossmanith & Seal 2015)
 * after every SSP-RK stage, before the operator: per element, the slope of each
 * conserved component along each d (the coefficient of xi_d in the element's Legendre
 * expansion, from mirror pairs of nodes) is bounded by minmod with the differences to
 * the neighbouring element averages (periodic wrap; a non-periodic end takes the
 * element's own average); the least ratio of bounded to own slope over the pairs whose
 * bound moves the slope by more than 1e-10 of the component's energy scale is one
 * factor theta <= 1 by which every node's deviation from the element average is
 * scaled.  Averages are kept, and a node stays on the segment to the average.  Each
 * stage then runs as two launches (the stage, writing the unlimited combination, its
 * element averages and its primitives; the limiter with the operator, rewriting U
 * and the primitives of the nodes that changed).  The taped
 * stepping and step-adjoint entry points reject it (DG_EINVAL); dg_rhs and dg_rhs_vjp
 * do not involve it. */
typedef struct {
  int dim, p;
  int n_elem[3];
  double lo[3], hi[3];
  int bc[3];
  int eos;
  double gamma_ad;
  double c_light;
  int c2p;
  int precision;
  int phys;
  double phys_eps;
  int sync_mode;
  int flux;
  int bc_hi[3];
  double bc_state[3][2][5];
  int c2p_iters;
  int limiter;
} dg_mesh_desc;

typedef struct {
  long long c2p_fail;        /* nodes with inadmissible U, no root or P <= 0 */
  long long c2p_noconv;      /* Newton / Brent iteration cap reached */
  long long trace_fallback;  /* face traces with rho <= 0 or P <= 0 replaced by the nearest node */
  long long flagged;         /* elements flagged by the physicality operator */
  long long smoothed;        /* flagged elements that were smoothed */
  long long bad_average;     /* flagged elements left unchanged (inadmissible average) */
  long long bad_input;       /* dg_set_state nodes rejected */
  long long first_bad_elem;  /* lowest element index with a recovery failure, or -1 */
  long long limited;         /* element-stages the slope limiter scaled (theta < 1) */
} dg_diag;

/* Create a context for one mesh.  Validates desc, builds the basis tables on the
 * host in FP64 and allocates scratch (about 5 states).  hip_stream may be NULL
 * (the null stream).  On failure *out is NULL and a negative code is returned. */
int dg_init_mesh(const dg_mesh_desc* desc, void* hip_stream, dg_ctx** out);
/* Make hip_stream the context's stream for the calls that follow.  Every call on a
 * context shares its scratch, so when the stream changes the new stream is made to
 * wait (an event, no host synchronisation) for the work already queued on the old
 * one; calls on the same context are thus ordered whatever streams they use. */
int dg_set_stream(dg_ctx* ctx, void* hip_stream);

/* Number of doubles in one nodal state array (n_var * n_elements * (p+1)^dim). */
size_t dg_state_size(const dg_ctx* ctx);

/* Initial data (Sec. 2.1, Eq. primitive_to_conserved).  kind = DG_PRIMITIVE:
 * src_dev holds (rho, v, P) with v the 3-velocity, converted to U_dev; invalid
 * nodes (rho <= 0, P <= 0, |v| >= c, non-finite) are counted (bad_input) and
 * written as D = 0.  kind = DG_CONSERVED: a device copy of src_dev into U_dev.
 * src_dev and U_dev must not overlap. */
int dg_set_state(dg_ctx* ctx, int kind, const double* src_dev, double* U_dev);

/* Per-node conserved-to-primitive recovery (Sec. 3) with the configured solver:
 * U_dev -> W_dev = (rho, u, P).  Failures follow the documented convention
 * (rho = 1e-10, u = 0, P = 1e-10 c^2, counted). */
int dg_con2prim(dg_ctx* ctx, const double* U_dev, double* W_dev);

/* DG right-hand side R = dU/dt of the weak form (Sec. 2.3, 2.4): recovery at the
 * nodes, volume quadrature, primitive traces, HLL numerical flux, lift and the
 * inverse of the diagonal mass matrix.  U_dev and R_dev must not overlap. */
int dg_rhs(dg_ctx* ctx, const double* U_dev, double* R_dev);

/* Physicality-enforcing operator (Sec. 2.5), in place on U_dev. */
int dg_enforce_physical(dg_ctx* ctx, double* U_dev);

/* One third-order SSP-RK step (Sec. 2.3) of size dt, in place on U_dev, with the
 * physicality operator after each stage when desc.phys = 1. */
int dg_ssprk3_step(dg_ctx* ctx, double* U_dev, double dt);
/* nsteps such steps (the primitive state is carried between steps). */
int dg_ssprk3_run(dg_ctx* ctx, double* U_dev, double dt, int nsteps);

/* One step (nsteps steps) of the SSP Runge-Kutta scheme of the given order in
 * Shu-Osher form (Sec. 2.3; the paper pairs basis orders p = 0, 1, 2 with
 * orders 1, 2, 3 in its convergence and performance runs): order 1 forward Euler,
 * 2 the second-order SSP scheme U1 = U + dt L(U), U+ = U/2 + (U1 + dt L(U1))/2,
 * 3 the scheme of dg_ssprk3_step.  In place on U_dev, the physicality operator
 * after each stage when desc.phys = 1, one kernel launch per stage.  Returns
 * DG_EINVAL for order outside 1..3 or nsteps < 0. */
int dg_ssprk_step(dg_ctx* ctx, double* U_dev, double dt, int order);
int dg_ssprk_run(dg_ctx* ctx, double* U_dev, double dt, int nsteps, int order);

/* Vector-Jacobian product of dg_rhs: lamU_dev = (dR/dU)^T lamR_dev.  The
 * recovery is differentiated by the implicit-function theorem.  The buffers
 * must not overlap. */
int dg_rhs_vjp(dg_ctx* ctx, const double* U_dev, const double* lamR_dev, double* lamU_dev);

/* Vector-Jacobian product of one dg_ssprk3_step taken from Un_dev with size dt:
 * lam_n_dev = (dU^{n+1}/dU^n)^T lam_next_dev.  The physicality operator is
 * differentiated on its active branch.  lam_next_dev and lam_n_dev may alias. */
int dg_ssprk3_step_vjp(dg_ctx* ctx, const double* Un_dev, double dt,
                       const double* lam_next_dev, double* lam_n_dev);

/* Taped step for the adjoint of a trajectory: dg_ssprk3_step in place on U_dev,
 * also recording into tape_dev (dg_tape_size doubles, caller-owned) the
 * primitives of the three stage inputs, the three stage outputs before the
 * physicality operator and, in a trailing block, whether the operator changed
 * any element in each stage (the reverse then skips the operator's adjoint, an
 * identity, without a host synchronisation).  dg_ssprk3_step_vjp_tape applies the
 * step's vector-Jacobian product from that tape without recomputing the forward
 * step; lam_next_dev and lam_n_dev may alias. */
size_t dg_tape_size(const dg_ctx* ctx);
int dg_ssprk3_step_tape(dg_ctx* ctx, double* U_dev, double dt, double* tape_dev);
int dg_ssprk3_step_vjp_tape(dg_ctx* ctx, const double* tape_dev, double dt, const double* lam_next_dev,
                            double* lam_n_dev);
/* Segment forms for checkpointed trajectories: nsteps taped steps in place on U_dev,
 * tapes_dev holding nsteps consecutive tapes; then the nsteps step adjoints in
 * reverse order, in place on lam_dev (lambda of the segment end on entry, of its
 * start on exit). */
int dg_ssprk3_run_tape(dg_ctx* ctx, double* U_dev, double dt, int nsteps, double* tapes_dev);
int dg_ssprk3_run_vjp_tape(dg_ctx* ctx, const double* tapes_dev, double dt, int nsteps, double* lam_dev);

/* J = sum over nodes of (cell volume / 2^dim) w_i v_y,i^2 (the integral of v_y^2,
 * the Kelvin-Helmholtz diagnostic of Sec. 4) written to *J_host (synchronises),
 * and, if dJdU_dev is not NULL, its gradient with respect to U. */
int dg_objective_vy2(dg_ctx* ctx, const double* U_dev, double* J_host, double* dJdU_dev);

/* Vector-Jacobian product of dg_set_state(DG_PRIMITIVE): lam_src_dev =
 * (dU/d(rho, v, P))^T lamU_dev at the primitive state src_dev. */
int dg_set_state_vjp(dg_ctx* ctx, const double* src_dev, const double* lamU_dev,
                     double* lam_src_dev);

/* Counters since the last reset (synchronises the stream). */
int dg_get_diagnostics(dg_ctx* ctx, dg_diag* out);
int dg_reset_diagnostics(dg_ctx* ctx);

/* Message of the last failed call on ctx (never NULL). */
const char* dg_last_error(const dg_ctx* ctx);

/* Release the context and its scratch (synchronises the stream first). */
void dg_destroy(dg_ctx* ctx);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops, harnesses that forbid hipMalloc): dg_rhs without a context and
 * without any allocation.  desc is validated and its tables are built on the host
 * at every call (as dg_init_mesh would, DG_EINVAL when rejected); U_dev and R_dev
 * are as in dg_rhs (caller-owned, [n_var][elements][nodes], not overlapping) and
 * the result equals dg_rhs's bit for bit.  Scratch: a static device array of 64 MiB
 * per GPU, held from the first call on that GPU until the process ends, holding the
 * counters and, where dg_rhs stages the primitives between two launches (3D with
 * p >= 1; elsewhere one launch recovers them in the tile), that staging: there,
 * meshes whose state holds more than DG_RHS_NOALLOC_MAX_STATE doubles
 * (n_var x elements x (p+1)^dim) are rejected with DG_EINVAL.  The work is enqueued on hip_stream, which must belong to the current
 * device; the first call on each device resolves the array's address (make it
 * outside a capture).  Every call on one GPU shares that array: calls that overlap
 * on one GPU (several streams or host threads) race.  The counters restart at zero
 * at every call; with diag non-NULL, or desc->sync_mode = 1, the call synchronises
 * hip_stream and reports them (not under capture), sync_mode also returning
 * DG_ECON2PRIM after a recovery failure.  Messages go to stderr. */
#define DG_RHS_NOALLOC_MAX_STATE 8380416u
int dg_rhs_noalloc(const dg_mesh_desc* desc, void* hip_stream, const double* U_dev, double* R_dev,
                   dg_diag* diag);

#ifdef __cplusplus
}
#endif

#endif /* DGSRHD_H */
