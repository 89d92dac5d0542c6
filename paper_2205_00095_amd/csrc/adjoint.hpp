// Adjoint (vector-Jacobian product) kernels of the DG SRHD path.
//
// k_rhs_vjp    element-tile kernel, one node per lane, gather form (no atomics):
//              transposed volume contraction and nodal-flux reverse; per face point
//              the adjoint of the face flux is assembled from the lift transposes of
//              BOTH adjacent elements (the neighbour's lambda gathered from HBM), the
//              HLL flux is reversed for the element's own trace, the trace
//              interpolation is transposed in LDS, and the recovery is reversed by the
//              implicit-function theorem (a DIM+2 linear solve per node).
//              Stage mode also folds in the SSP-RK combine transpose and the
//              physicality operator's active-branch adjoint of the previous stage.
// k_enforce_vjp  the physicality operator's adjoint alone.
// k_objective / k_sum   J = int v_y^2 with a fixed-order reduction, and dJ/dU.
// k_prim3_vjp  adjoint of the (rho, v, P) -> U map of the initial data.
#pragma once
#include "kernels.hpp"
#include "physics_rev.hpp"

namespace dgsrhd {

struct VjpArgs {
  const double* W;      // primitives of the linearisation point
  const double* lam;    // adjoint of R (plain) or of the stage's pre-operator output (stage)
  const double* lam_alt;     // read instead of lam when *lam_sel != 0 (lam_sel may be null)
  const unsigned* lam_sel;
  const unsigned* pflag;     // the forward operator of the previous stage changed nothing when *pflag == 0
  double* out;          // lambda_U (plain); previous stage's adjoint or lambda_n (stage)
  double* lamn;         // running adjoint of U^n (stage mode)
  const double* Pprev;  // pre-operator state of the previous stage (stage mode), or null
  // first stage of a step (Pprev null): the output lambda_n is U^n's adjoint, U^n = Pi(Ppost)
  // the previous step's last stage output; with Ppost set the output is Pi'(Ppost)^T lambda_n,
  // the adjoint of that pre-operator state (the operator's adjoint fused into this launch)
  const double* Ppost;
  const unsigned* postflag;  // that operator changed nothing when *postflag == 0 (may be null)
  double ca, cb, dt;
  int lamn_init;        // 1: lamn is treated as zero on input
  MeshArgs m;
  Tables t;
  PhysParams q;
};

enum { VJP_PLAIN = 0, VJP_STAGE = 1 };

template <int DIM>
__device__ __forceinline__ bool is_floor_state(const double* W, const PhysParams& q) {
  bool f = (W[0] == kRhoFloor) && (W[DIM + 1] == kPFloor * q.c2);
#pragma unroll
  for (int j = 0; j < DIM; ++j) f = f && (W[1 + j] == 0.0);
  return f;
}

// Nodal fluxes F^d(W), d = 0..DIM-1, reversed with one state evaluation.
template <int EOS, int DIM>
__host__ __device__ __forceinline__ void nodal_flux_rev(const double* W, const PhysParams& q, const double (*lamF)[DIM + 2],
                                               double* lamW) {
  constexpr int NV = DIM + 2;
  StateEval<EOS, DIM> s;
  eval_state<EOS, DIM>(W, q, s);
  double lam_U[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) lam_U[k] = 0.0;
  double lam_ig = 0.0, lam_P = 0.0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    const double vd = W[1 + d] * s.ig;
    double lam_vd = 0.0;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      lam_U[k] += lamF[d][k] * vd;
      lam_vd += lamF[d][k] * s.U[k];
    }
    lam_P += lamF[d][1 + d] + lamF[d][NV - 1] * vd;
    lam_vd += lamF[d][NV - 1] * s.P;
    lamW[1 + d] += lam_vd * s.ig;
    lam_ig += lam_vd * W[1 + d];
  }
  lamW[NV - 1] += lam_P;
  eval_state_rev<EOS, DIM>(W, s, q, lam_U, 0.0, lam_ig, 0.0, 0.0, lamW);
}

// Adjoint of the physicality operator on the elements of one workgroup.  Pn is
// the node's pre-operator state; lam holds the adjoint of the operator output on
// entry and of its input on exit.  Linearised on the active branch: the
// element's argmin node, its stage-1/stage-2 case and the average.  sbuf needs
// (NV + 1) * NT doubles, sred NV * EPB doubles, sflag NT ints, svote one int per
// wave (for this call only).  All threads of
// the block must reach it.
template <int DIM, int P, int NT, int EPB>
__device__ __forceinline__ void physicality_vjp_block(const double* Pn, double* lam, bool act, int tid, int el,
                                                      int node, const Tables& t, const PhysParams& q, double* sbuf,
                                                      double* sred, int* sflag, int* svote) {
  using G = Geo<DIM, P>;
  constexpr int NV = G::NV, NPE = G::NPE, N1 = G::N1;
  const bool bad = act && !admissible<DIM>(Pn, q);
  if (!block_any<(NT + 63) / 64>(bad, svote)) return;
  double wn = t.w[node_coord<N1>(node, 0)];
  if (DIM > 1) wn *= t.w[node_coord<N1>(node, 1)];
  if (DIM > 2) wn *= t.w[node_coord<N1>(node, 2)];
#pragma unroll
  for (int v = 0; v < NV; ++v) sbuf[v * NT + tid] = wn * Pn[v];
  sflag[tid] = bad ? 1 : 0;
  __syncthreads();
  bool eflag = false;
  for (int n = 0; n < NPE; ++n) eflag |= (sflag[el * NPE + n] != 0);
  double Ub[NV];
  bool avg_ok = false;
  double si = 1.0;
  if (act && eflag) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      double acc = 0.0;
      for (int n = 0; n < NPE; ++n) acc += sbuf[v * NT + el * NPE + n];
      Ub[v] = acc * t.inv_wsum;
    }
    avg_ok = admissible<DIM>(Ub, q);
    if (avg_ok) si = node_factor<DIM>(Pn, Ub, q);
  }
  __syncthreads();
  sbuf[tid] = si;
  __syncthreads();
  double smin = 1.0;
  int istar = 0;
  if (act && eflag && avg_ok) {
    for (int n = 0; n < NPE; ++n) {
      const double sv = sbuf[el * NPE + n];
      if (sv < smin) { smin = sv; istar = n; }
    }
  }
  __syncthreads();
  double ls = 0.0;
  if (act && eflag && avg_ok) {
#pragma unroll
    for (int v = 0; v < NV; ++v) ls += lam[v] * (Pn[v] - Ub[v]);
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) sbuf[v * NT + tid] = lam[v];
  sbuf[NV * NT + tid] = ls;
  __syncthreads();
  double sumlam[NV], gP[NV];
  double lam_s = 0.0;
  const bool active = act && eflag && avg_ok && smin < 1.0;
  if (active) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      double acc = 0.0;
      for (int n = 0; n < NPE; ++n) acc += sbuf[v * NT + el * NPE + n];
      sumlam[v] = acc;
    }
    for (int n = 0; n < NPE; ++n) lam_s += sbuf[NV * NT + el * NPE + n];
    if (node == istar) {
      constexpr int ND = 2 * NV;
      Dual<ND> Ud[NV], Bd[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        Ud[v] = dconst<ND>(Pn[v]);
        Ud[v].t[v] = 1.0;
        Bd[v] = dconst<ND>(Ub[v]);
        Bd[v].t[NV + v] = 1.0;
      }
      const Dual<ND> sd = node_factor_dual<DIM, ND>(Ud, Bd, q);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        gP[v] = lam_s * sd.t[v];
        sred[v * EPB + el] = lam_s * sd.t[NV + v];
      }
    }
  }
  __syncthreads();
  if (active) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const double lamUb = (1.0 - smin) * sumlam[v] + sred[v * EPB + el];
      double r = smin * lam[v] + wn * t.inv_wsum * lamUb;
      if (node == istar) r += gP[v];
      lam[v] = r;
    }
  }
  __syncthreads();
}

// flag, when given, is the forward stage's operator flag: 0 means the operator
// changed nothing, its adjoint is the identity and nothing is written (the caller
// then reads lam_in).
template <int DIM, int P>
__global__ __launch_bounds__((Geo<DIM, P>::NT)) void k_enforce_vjp(const double* __restrict__ Pst,
                                                                   const double* __restrict__ lam_in,
                                                                   double* __restrict__ lam_out, MeshArgs m, Tables t,
                                                                   PhysParams q, const unsigned* flag) {
  using G = Geo<DIM, P>;
  if (flag && *flag == 0u) return;
  constexpr int NV = G::NV, NPE = G::NPE, NT = G::NT, EPB = G::EPB;
  __shared__ double sbuf[(NV + 1) * NT];
  __shared__ double sred[NV * EPB];
  __shared__ int sflag[NT];
  __shared__ int svote[(NT + 63) / 64];
  const int tid = threadIdx.x;
  const int el = tid / NPE, node = tid % NPE;
  const long long e = (long long)blockIdx.x * EPB + el;
  const bool act = e < m.nelem;
  const long long g = e * NPE + node;
  double Pn[NV], lam[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    Pn[v] = act ? Pst[v * m.ntot + g] : 1.0;
    lam[v] = act ? lam_in[v * m.ntot + g] : 0.0;
  }
  physicality_vjp_block<DIM, P, NT, EPB>(Pn, lam, act, tid, el, node, t, q, sbuf, sred, sflag, svote);
  if (act) {
#pragma unroll
    for (int v = 0; v < NV; ++v) lam_out[v * m.ntot + g] = lam[v];
  }
}

// Trace of the primitives at one face point (as trace_lds / trace_glb of the forward
// kernel: weights l_b(+1) over nodes n0 + b step, the nearest node on fallback) and the
// lift transpose's sum over the same line, sum_b (1/w_b) l_b(+1) lambda(n0 + b step),
// whose weights the reversal maps the same way (w_{P-b} = w_b).  Returns whether the
// trace fell back.
template <int NV, int NT, int P>
__device__ __forceinline__ bool trace_lam_lds(const double* sW, const double* sL, int n0, int step,
                                              const Tables& t, double* Wt, double* lt) {
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    double acc = 0.0, lacc = 0.0;
#pragma unroll
    for (int b = 0; b <= P; ++b) {
      acc += t.lp[b] * sW[v * NT + n0 + b * step];
      lacc += t.iw[b] * t.lp[b] * sL[v * NT + n0 + b * step];
    }
    Wt[v] = acc;
    lt[v] = lacc;
  }
  if (!(Wt[0] > 0.0) || !(Wt[NV - 1] > 0.0)) {
#pragma unroll
    for (int v = 0; v < NV; ++v) Wt[v] = sW[v * NT + n0 + P * step];
    return true;
  }
  return false;
}

template <int NV, int P>
__device__ __forceinline__ bool trace_lam_glb(const double* srcW, const double* srcL, long long ntot, int step,
                                              const Tables& t, double* Wt, double* lt) {
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    double acc = 0.0, lacc = 0.0;
#pragma unroll
    for (int b = 0; b <= P; ++b) {
      acc += t.lp[b] * srcW[v * ntot + b * step];
      lacc += t.iw[b] * t.lp[b] * srcL[v * ntot + b * step];
    }
    Wt[v] = acc;
    lt[v] = lacc;
  }
  if (!(Wt[0] > 0.0) || !(Wt[NV - 1] > 0.0)) {
#pragma unroll
    for (int v = 0; v < NV; ++v) Wt[v] = srcW[v * ntot + P * step];
    return true;
  }
  return false;
}

// Waves per SIMD the adjoint element kernel is compiled for: 3 (at most 168 VGPRs,
// a few spills) measured faster than 2 for the 2D ideal-gas kernels; elsewhere the
// spills at 3 would be heavy.  At p = 0 the tile's LDS already caps the occupancy
// below either bound, so none is asked for.
template <int DIM, int P, int EOS>
constexpr int vjp_min_waves() { return P == 0 ? 1 : (DIM == 2 && EOS == EOS_IDEAL) ? 3 : 2; }

template <int DIM, int P, int EOS, int MODE, int FLUX>
__global__ __launch_bounds__((TileGeo<DIM, P>::NT), (vjp_min_waves<DIM, P, EOS>())) void k_rhs_vjp(VjpArgs a) {
  using T = TileGeo<DIM, P>;
  constexpr int N1 = T::N1, NPE = T::NPE, NV = T::NV, NT = T::NT, EPB = T::EPB;
  constexpr int NFP = T::NFP, FPB = T::FPB, TX = T::TX, TY = T::TY;
  __shared__ double sW[NV * NT];
  __shared__ double sL[(NV + 1) * NT];
  __shared__ double sLWL[NV * FPB];  // adjoint of the left (+) trace of each face point
  __shared__ double sLWR[NV * FPB];  // adjoint of the right (-) trace
  __shared__ int sfb[FPB];           // bit 0: left trace fell back, bit 1: right trace fell back
  __shared__ double sred[(MODE == VJP_STAGE) ? NV * EPB : 1];
  __shared__ int sflag[(MODE == VJP_STAGE) ? NT : 1];
  __shared__ int svote[(NT + 63) / 64];

  const MeshArgs& m = a.m;
  const Tables& t = a.t;
  const PhysParams& q = a.q;
  const long long ntot = m.ntot;
  const int tid = threadIdx.x;
  const int el = tid / NPE, node = tid % NPE;
  const int ntx = (m.nex + TX - 1) / TX, nty = (m.ney + TY - 1) / TY, ntz = (m.nez + T::TZ - 1) / T::TZ;
  const int tile = xcd_tile(blockIdx.x, ntx * nty * ntz);
  const int o[3] = {(tile % ntx) * TX, ((tile / ntx) % nty) * TY, (tile / (ntx * nty)) * T::TZ};
  const int lc[3] = {el % TX, (el / TX) % TY, el / (TX * TY)};
  const bool act = (o[0] + lc[0] < m.nex) && (o[1] + lc[1] < m.ney) && (o[2] + lc[2] < m.nez);
  const long long e = act ? ((long long)(o[2] + lc[2]) * m.ney + (o[1] + lc[1])) * m.nex + (o[0] + lc[0]) : 0;
  const long long g = e * NPE + node;
  const double* const lam_in = (a.lam_sel && *a.lam_sel != 0u) ? a.lam_alt : a.lam;

  double W[NV], mu[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    W[v] = act ? a.W[v * ntot + g] : (v == 0 || v == NV - 1 ? 1.0 : 0.0);
    mu[v] = act ? lam_in[v * ntot + g] : 0.0;
    sW[v * NT + tid] = W[v];
    sL[v * NT + tid] = mu[v];
  }
  __syncthreads();

  // ---- volume: lamF^d at this node = (2/dx_d) sum_i dhat[i][a_d] lam_(line node i); nodal flux reverse
  double lamW[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) lamW[v] = 0.0;
  {
    double lamF[DIM][NV];
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const int id = node_coord<N1>(node, d);
      const int pt = face_pt<DIM, N1>(node, d);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        double acc = 0.0;
#pragma unroll
        for (int i = 0; i < N1; ++i) acc += t.dhat[i][id] * sL[v * NT + el * NPE + line_node<DIM, N1>(d, pt, i)];
        lamF[d][v] = m.two_dx[d] * acc;
      }
    }
    nodal_flux_rev<EOS, DIM>(W, q, lamF, lamW);
  }
  // end the volume reverse here (the compiler would otherwise sink it past the face
  // phase and keep every loaded lambda live through it)
#pragma unroll
  for (int v = 0; v < NV; ++v) pin_reg(lamW[v]);

  // ---- faces of the tile: adjoint of each face flux from the lift transposes of both
  //      adjacent elements, HLL linearised once and reversed for every side in the tile.
  //      Side A of a face point is an element in this tile (the left one when it is),
  //      side B the other one (LDS, HBM, or absent at an outflow boundary); the slot
  //      order puts the tile's boundary face points first (see TileFacePoint).
  for (int k = tid; k < FPB; k += NT) {
    const TileFacePoint<DIM, P> fc = TileFacePoint<DIM, P>::from_slot(k, o, m);
    const bool left_local = fc.left_local, right_local = fc.right_local;
    if (!left_local && !right_local) continue;
    const int d = fc.d;
    const double tdx = sel3(d, m.two_dx[0], m.two_dx[1], m.two_dx[2]);
    const int line0 = line_node<DIM, N1>(d, fc.pt, 0);
    const int stride = sel3(d, 1, N1, N1 * N1);
    const bool a_left = left_local;
    const int fwd0 = line0, bwd0 = line0 + P * stride;
    // traces and lift-transpose sums sum_b iw_b lp_b lam_(node b) of both sides
    double WA[NV], WB[NV], lA[NV], lB[NV];
    const bool fbA = trace_lam_lds<NV, NT, P>(sW, sL, (a_left ? fc.left_elem() : fc.right_elem()) * NPE +
                                              (a_left ? fwd0 : bwd0), a_left ? stride : -stride, t, WA, lA);
    bool fbB = false, have_B = true;
    if (a_left && right_local) {
      fbB = trace_lam_lds<NV, NT, P>(sW, sL, fc.right_elem() * NPE + bwd0, -stride, t, WB, lB);
    } else {
      const long long ge = a_left ? fc.right_global() : fc.left_global();
      have_B = ge >= 0;
      if (have_B) {
        const long long off = ge * NPE + (a_left ? bwd0 : fwd0);
        fbB = trace_lam_glb<NV, P>(a.W + off, lam_in + off, ntot, a_left ? -stride : stride, t, WB, lB);
      }
    }
    // the left element's lift contributes -(2/dx) sum, the right one's +(2/dx) sum
    double lamFh[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const double lb = have_B ? lB[v] : 0.0;
      lamFh[v] = tdx * (a_left ? lb - lA[v] : lA[v] - lb);
    }
    double lamWL[NV], lamWR[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) lamWL[v] = lamWR[v] = 0.0;
    if (!have_B) {
      // a boundary face: the exterior state is side A's trace (outflow), its mirror image
      // (a wall: u_d negated) or fixed; its adjoint goes back onto side A accordingly
      const int kind = a_left ? sel3(d, m.bchi[0], m.bchi[1], m.bchi[2]) : sel3(d, m.bclo[0], m.bclo[1], m.bclo[2]);
      exterior_state<DIM>(m, d, a_left, WA, WB);
      double WL[NV], WR[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        WL[v] = a_left ? WA[v] : WB[v];
        WR[v] = a_left ? WB[v] : WA[v];
      }
      if constexpr (FLUX == FLUX_HLLC)
        hllc_flux_rev<EOS, DIM>(WL, WR, d, q, lamFh, lamWL, lamWR, true, true);
      else
        hll_flux_rev<EOS, DIM>(WL, WR, d, q, lamFh, lamWL, lamWR, true, true);
      double lamM[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) lamM[v] = a_left ? lamWR[v] : lamWL[v];
      if (kind == BC_REFLECT) comp_add<DIM>(lamM + 1, d, -2.0 * comp<DIM>(lamM + 1, d));
      const double keep = kind == BC_FIXED ? 0.0 : 1.0;  // a fixed state does not depend on A
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const double lamWA = (a_left ? lamWL[v] : lamWR[v]) + keep * lamM[v];
        lamWL[v] = a_left ? lamWA : 0.0;
        lamWR[v] = a_left ? 0.0 : lamWA;
      }
    } else {
      double WL[NV], WR[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        WL[v] = a_left ? WA[v] : WB[v];
        WR[v] = a_left ? WB[v] : WA[v];
      }
      if constexpr (FLUX == FLUX_HLLC)
        hllc_flux_rev<EOS, DIM>(WL, WR, d, q, lamFh, lamWL, lamWR, left_local, right_local);
      else
        hll_flux_rev<EOS, DIM>(WL, WR, d, q, lamFh, lamWL, lamWR, left_local, right_local);
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      sLWL[v * FPB + fc.fidx] = lamWL[v];
      sLWR[v * FPB + fc.fidx] = lamWR[v];
    }
    const bool fbL = a_left ? fbA : fbB, fbR = a_left ? fbB : fbA;
    sfb[fc.fidx] = (fbL ? 1 : 0) | (fbR ? 2 : 0);
  }
  __syncthreads();

  // ---- transposed trace interpolation (or the fallback node)
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    const int id = node_coord<N1>(node, d);
    const int pt = face_pt<DIM, N1>(node, d);
    // minus face: this element is the right side
    {
      const int fpi = tile_face_index<DIM, P>(d, lc[d], lc, pt);
      const double coef = (sfb[fpi] & 2) ? (id == 0 ? 1.0 : 0.0) : t.lm[id];
#pragma unroll
      for (int v = 0; v < NV; ++v) lamW[v] += coef * sLWR[v * FPB + fpi];
    }
    // plus face: this element is the left side
    {
      const int fpi = tile_face_index<DIM, P>(d, lc[d] + 1, lc, pt);
      const double coef = (sfb[fpi] & 1) ? (id == P ? 1.0 : 0.0) : t.lp[id];
#pragma unroll
      for (int v = 0; v < NV; ++v) lamW[v] += coef * sLWL[v * FPB + fpi];
    }
  }

  // ---- recovery adjoint (implicit-function theorem); W and mu come back from LDS so
  //      they are not held in registers through the face phase
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    W[v] = sW[v * NT + tid];
    mu[v] = sL[v * NT + tid];
  }
  double lamU[NV];
  if (is_floor_state<DIM>(W, q)) {
#pragma unroll
    for (int v = 0; v < NV; ++v) lamU[v] = 0.0;
  } else {
    double J[NV][NV];
    prim_jacobian<EOS, DIM>(W, q, J);
    solve_transposed<NV>(J, lamW, lamU);
  }

  if constexpr (MODE == VJP_PLAIN) {
    if (act) {
#pragma unroll
      for (int v = 0; v < NV; ++v) a.out[v * ntot + g] = lamU[v];
    }
  } else {
    double lp[NV], acc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      lp[v] = a.cb * (mu[v] + a.dt * lamU[v]);
      const double prev = (act && !a.lamn_init) ? a.lamn[v * ntot + g] : 0.0;
      acc[v] = prev + a.ca * mu[v];
    }
    if (a.Pprev) {
      if (!a.pflag || *a.pflag != 0u) {
        double Pn[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) Pn[v] = act ? a.Pprev[v * ntot + g] : 1.0;
        __syncthreads();
        physicality_vjp_block<DIM, P, NT, EPB>(Pn, lp, act, tid, el, node, t, q, sL, sred, sflag, svote);
      }
      if (act) {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          a.out[v * ntot + g] = lp[v];
          a.lamn[v * ntot + g] = acc[v];
        }
      }
    } else {
      double tot[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) tot[v] = acc[v] + lp[v];
      if (a.Ppost && (!a.postflag || *a.postflag != 0u)) {
        double Pn[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) Pn[v] = act ? a.Ppost[v * ntot + g] : 1.0;
        __syncthreads();
        physicality_vjp_block<DIM, P, NT, EPB>(Pn, tot, act, tid, el, node, t, q, sL, sred, sflag, svote);
      }
      if (act) {
#pragma unroll
        for (int v = 0; v < NV; ++v) a.out[v * ntot + g] = tot[v];
      }
    }
  }
}

// ------------------------------------------------ objective J = int v_y^2 dA
template <int EOS, int DIM>
__global__ __launch_bounds__(256) void k_objective(const double* __restrict__ U, double* __restrict__ partial,
                                                   double* __restrict__ grad, long long ntot, int npe, int n1,
                                                   Tables t, double jac, PhysParams q) {
  constexpr int NV = DIM + 2;
  __shared__ double red[256];
  const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  double Jn = 0.0;
  if (n < ntot) {
    double u[NV], W[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) u[v] = U[v * ntot + n];
    const int st = con2prim<EOS, DIM>(u, W, q);
    const int node = (int)(n % npe);
    double wn = t.w[node % n1];
    if (DIM > 1) wn *= t.w[(node / n1) % n1];
    if (DIM > 2) wn *= t.w[node / (n1 * n1)];
    const double cw = jac * wn;
    double lamU[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) lamU[v] = 0.0;
    if constexpr (DIM >= 2) {
      double usq = 0.0;
#pragma unroll
      for (int j = 0; j < DIM; ++j) usq += W[1 + j] * W[1 + j];
      const double gm = sqrt(1.0 + usq * q.inv_c2);
      const double vy = W[2] / gm;
      Jn = cw * vy * vy;
      if (grad && (st == C2P_OK || st == C2P_NOCONV)) {
        double lamW[NV];
        lamW[0] = 0.0;
        lamW[NV - 1] = 0.0;
        const double common = 2.0 * cw * vy;
#pragma unroll
        for (int k = 0; k < DIM; ++k)
          lamW[1 + k] = common * ((k == 1 ? 1.0 / gm : 0.0) - W[2] * W[1 + k] * q.inv_c2 / (gm * gm * gm));
        double J[NV][NV];
        prim_jacobian<EOS, DIM>(W, q, J);
        solve_transposed<NV>(J, lamW, lamU);
      }
    }
    if (grad) {
#pragma unroll
      for (int v = 0; v < NV; ++v) grad[v * ntot + n] = lamU[v];
    }
  }
  red[threadIdx.x] = Jn;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// Adjoint of (rho, v, P) -> U: lam_src = (dU/d(rho, v, P))^T lamU.
template <int EOS, int DIM>
__global__ __launch_bounds__(256) void k_prim3_vjp(const double* __restrict__ S, const double* __restrict__ lamU,
                                                   double* __restrict__ lamS, long long ntot, PhysParams q) {
  constexpr int NV = DIM + 2;
  const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= ntot) return;
  double w[NV], lu[NV], out[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    w[v] = S[v * ntot + n];
    lu[v] = lamU[v * ntot + n];
    out[v] = 0.0;
  }
  double v2 = 0.0;
#pragma unroll
  for (int j = 0; j < DIM; ++j) v2 += w[1 + j] * w[1 + j];
  const double b2 = v2 * q.inv_c2;
  const bool ok = (w[0] > 0.0) && (w[NV - 1] > 0.0) && (b2 < 1.0) && isfinite(w[0]) && isfinite(w[NV - 1]) &&
                  isfinite(b2);
  if (ok) {
    const double gm = 1.0 / sqrt(1.0 - b2);
    double Wu[NV];
    Wu[0] = w[0];
    Wu[NV - 1] = w[NV - 1];
#pragma unroll
    for (int j = 0; j < DIM; ++j) Wu[1 + j] = gm * w[1 + j];
    double J[NV][NV];
    prim_jacobian<EOS, DIM>(Wu, q, J);
    double lw[NV];
#pragma unroll
    for (int c = 0; c < NV; ++c) {
      double acc = 0.0;
#pragma unroll
      for (int r = 0; r < NV; ++r) acc += J[r][c] * lu[r];
      lw[c] = acc;
    }
    out[0] = lw[0];
    out[NV - 1] = lw[NV - 1];
    double vl = 0.0;
#pragma unroll
    for (int j = 0; j < DIM; ++j) vl += w[1 + j] * lw[1 + j];
    // u = gamma v:  du_j/dv_k = gamma delta_jk + gamma^3 v_j v_k / c^2
#pragma unroll
    for (int k = 0; k < DIM; ++k) out[1 + k] = gm * lw[1 + k] + gm * gm * gm * vl * w[1 + k] * q.inv_c2;
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) lamS[v * ntot + n] = out[v];
}

}  // namespace dgsrhd
