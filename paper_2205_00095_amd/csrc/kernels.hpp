// gfx950 kernels of the DG SRHD hot path.
//
// Data layout in HBM: every nodal array is [var][element][node] with element =
// (ez * ney + ey) * nex + ex and node = (k * N1 + j) * N1 + i, so the N1^DIM nodes
// of one element and consecutive elements along x are contiguous per component.
//
// k_con2prim   one node per lane: U -> W (Sec. 3), registers only.
// k_element    one workgroup per EPB consecutive elements, one node per lane:
//                volume term (Sec. 2.3, Eq. quad-vol-flux) from nodal fluxes staged
//                in LDS; face traces of the primitives, neighbour traces gathered
//                from HBM, HLL numerical flux (Sec. 2.4) per face point into LDS;
//                lift with the inverse diagonal mass; then either write R, or
//                (stage mode) the SSP-RK combine, the physicality-enforcing
//                operator (Sec. 2.5) on the element in LDS and the recovery of the
//                next stage's primitives, all before one write of U and W.
// k_enforce    the physicality operator alone, in place.
#pragma once
#include "physics.hpp"

namespace dgsrhd {

constexpr int ipow(int b, int e) { return e == 0 ? 1 : b * ipow(b, e - 1); }

template <int DIM, int P>
struct Geo {
  static constexpr int N1 = P + 1;
  static constexpr int NPE = ipow(N1, DIM);
  static constexpr int NV = DIM + 2;
  static constexpr int NFP = ipow(N1, DIM - 1);
  static constexpr int NF = 2 * DIM;
  static constexpr int EPB = (256 / NPE) > 0 ? 256 / NPE : 1;
  static constexpr int NT = EPB * NPE;
  static constexpr int FPB = EPB * NF * NFP;
};

constexpr int kMaxN1 = 4;

struct Tables {
  double dhat[kMaxN1][kMaxN1];  // dhat[i][a] = w_a l_i'(x_a) / w_i
  double lp[kMaxN1], lm[kMaxN1];
  double w[kMaxN1], iw[kMaxN1];
  double inv_wsum;              // 1 / sum of the element's tensor weights
  float dhat_f[kMaxN1][kMaxN1];
  float lp_f[kMaxN1], lm_f[kMaxN1], iw_f[kMaxN1];
};

struct MeshArgs {
  int nex, ney, nez, nelem;
  long long ntot;               // nodes per component
  double two_dx[3];             // 2 / dx_d
  int periodic[3];
};

struct Counters {
  unsigned long long c2p_fail, c2p_noconv, trace_fallback, flagged, smoothed, bad_average, bad_input;
  unsigned long long first_bad;  // lowest failing element (ULLONG_MAX if none)
};

struct ElemArgs {
  const double* W;    // primitives of the stage input
  const double* Uk;   // stage input U^(k)          (stage mode)
  const double* Un;   // step start U^n             (stage mode)
  double* out;        // R (rhs mode) or U^(k+1) (stage mode)
  double* Wout;       // primitives of U^(k+1), or null
  double* Pout;       // U^(k+1) before the physicality operator (adjoint tape), or null
  double ca, cb, dt;  // U^(k+1) = ca U^n + cb (U^(k) + dt R)
  int phys;
  MeshArgs m;
  Tables t;
  PhysParams q;
  Counters* cnt;
};

__device__ __forceinline__ void count_c2p(Counters* cnt, int status, long long elem) {
  if (status == C2P_OK) return;
  if (status == C2P_NOCONV) atomicAdd(&cnt->c2p_noconv, 1ull);
  else atomicAdd(&cnt->c2p_fail, 1ull);
  atomicMin(&cnt->first_bad, (unsigned long long)elem);
}

// index of the node along direction d
template <int N1>
__device__ __forceinline__ int node_coord(int node, int d) {
  return d == 0 ? node % N1 : (d == 1 ? (node / N1) % N1 : node / (N1 * N1));
}

// face-point index of a node on the faces normal to d (remaining coordinates, lower dims fastest)
template <int DIM, int N1>
__device__ __forceinline__ int face_pt(int node, int d) {
  if constexpr (DIM == 1) return 0;
  const int i = node % N1, j = (node / N1) % N1, k = node / (N1 * N1);
  if constexpr (DIM == 2) return d == 0 ? j : i;
  return d == 0 ? k * N1 + j : (d == 1 ? k * N1 + i : j * N1 + i);
}

// node at position a along d through face point pt
template <int DIM, int N1>
__device__ __forceinline__ int line_node(int d, int pt, int a) {
  if constexpr (DIM == 1) return a;
  if constexpr (DIM == 2) return d == 0 ? pt * N1 + a : a * N1 + pt;
  if (d == 0) return pt * N1 + a;
  if (d == 1) return (pt / N1) * N1 * N1 + a * N1 + pt % N1;
  return a * N1 * N1 + pt;
}

// neighbour element across the face of direction d on side +1 / -1, or -1 at an outflow boundary
__device__ __forceinline__ int neighbour(const MeshArgs& m, int e, int d, int dir) {
  const int ex = e % m.nex;
  const int ey = (e / m.nex) % m.ney;
  const int ez = e / (m.nex * m.ney);
  int c[3] = {ex, ey, ez};
  const int n[3] = {m.nex, m.ney, m.nez};
  c[d] += dir;
  if (c[d] < 0 || c[d] >= n[d]) {
    if (!m.periodic[d]) return -1;
    c[d] = (c[d] + n[d]) % n[d];
  }
  return (c[2] * m.ney + c[1]) * m.nex + c[0];
}

// ------------------------------------------------------------ recovery kernel
template <int EOS, int DIM>
__global__ __launch_bounds__(256) void k_con2prim(const double* __restrict__ U, double* __restrict__ W,
                                                  long long ntot, int npe, PhysParams q, Counters* cnt) {
  constexpr int NV = DIM + 2;
  const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= ntot) return;
  double u[NV], w[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) u[v] = U[v * ntot + n];
  const int st = con2prim<EOS, DIM>(u, w, q);
  count_c2p(cnt, st, n / npe);
#pragma unroll
  for (int v = 0; v < NV; ++v) W[v * ntot + n] = w[v];
}

// (rho, v, P) with v the 3-velocity -> U (Eq. primitive_to_conserved); rejects
// rho <= 0, P <= 0, |v| >= c and non-finite input (written as D = 0, counted).
template <int EOS, int DIM>
__global__ __launch_bounds__(256) void k_prim3_to_cons(const double* __restrict__ S, double* __restrict__ U,
                                                       long long ntot, PhysParams q, Counters* cnt) {
  constexpr int NV = DIM + 2;
  const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= ntot) return;
  double w[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) w[v] = S[v * ntot + n];
  double v2 = 0.0;
#pragma unroll
  for (int j = 0; j < DIM; ++j) v2 += w[1 + j] * w[1 + j];
  const double b2 = v2 * q.inv_c2;
  bool ok = (w[0] > 0.0) && (w[NV - 1] > 0.0) && (b2 < 1.0) && isfinite(w[0]) && isfinite(w[NV - 1]) &&
            isfinite(b2);
  double out[NV];
  if (ok) {
    const double g = 1.0 / sqrt(1.0 - b2);
#pragma unroll
    for (int j = 0; j < DIM; ++j) w[1 + j] *= g;
    StateEval<EOS, DIM> s;
    eval_state<EOS, DIM>(w, q, s);
#pragma unroll
    for (int v = 0; v < NV; ++v) out[v] = s.U[v];
  } else {
    atomicAdd(&cnt->bad_input, 1ull);
#pragma unroll
    for (int v = 0; v < NV; ++v) out[v] = 0.0;
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) U[v * ntot + n] = out[v];
}

// ------------------------------------------- physicality operator (Sec. 2.5)
// Largest s_i for one node given the element average (readings: '+' under the
// root of Eq. physicality; no square on the momentum difference in b; relative
// margin eps with the stable root 2(1-eps)c/(-b + sqrt(b^2 - 4a(1-eps)c))).
template <int DIM>
__device__ __forceinline__ double node_factor(const double* Ui, const double* Ub, const PhysParams& q) {
  constexpr int NV = DIM + 2;
  const double eps = q.eps;
  const double Di = Ui[0], Ei = Ui[NV - 1] + Ui[0] * q.c2;
  const double Db = Ub[0], Eb = Ub[NV - 1] + Ub[0] * q.c2;
  const double sD = (Di >= eps * Db) ? 1.0 : (1.0 - eps) * Db / (Db - Di);
  const double sE = (Ei >= eps * Eb) ? 1.0 : (1.0 - eps) * Eb / (Eb - Ei);
  const double s1 = fmin(sD, sE);
  double U1[NV], dl[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    U1[v] = s1 * Ui[v] + (1.0 - s1) * Ub[v];
    dl[v] = U1[v] - Ub[v];
  }
  // Q(U) = t (t + 2D) - |s|^2 with t = tau/c^2, s = S/c
  const double tb = Ub[NV - 1] * q.inv_c2;
  double sb2 = 0.0, s12 = 0.0, ds2 = 0.0, sbds = 0.0;
#pragma unroll
  for (int j = 0; j < DIM; ++j) {
    const double sb = Ub[1 + j] * q.inv_c, s1j = U1[1 + j] * q.inv_c, dsj = dl[1 + j] * q.inv_c;
    sb2 += sb * sb;
    s12 += s1j * s1j;
    ds2 += dsj * dsj;
    sbds += sb * dsj;
  }
  const double Qb = tb * (tb + 2.0 * Ub[0]) - sb2;
  const double t1 = U1[NV - 1] * q.inv_c2;
  const double Q1 = t1 * (t1 + 2.0 * U1[0]) - s12;
  if (!(Q1 < eps * Qb)) return s1;
  const double dt = dl[NV - 1] * q.inv_c2, dD = dl[0];
  const double a = dt * (dt + 2.0 * dD) - ds2;
  const double b = 2.0 * (tb * dt + tb * dD + Ub[0] * dt - sbds);
  const double cp = (1.0 - eps) * Qb;
  const double disc = fmax(b * b - 4.0 * a * cp, 0.0);
  const double s2 = 2.0 * cp / (-b + sqrt(disc));
  return s1 * s2;
}

// Apply the operator to the elements of one workgroup.  Every thread holds one
// node's U in registers (act = it belongs to a real element); sbuf must hold
// NV * NT doubles and sflag NT ints.  Must be reached by all threads of the block.
template <int DIM, int P>
__device__ __forceinline__ void physicality_block(double* Un, bool act, int tid, int el, int node, long long e,
                                                  const Tables& t, const PhysParams& q, Counters* cnt,
                                                  double* sbuf, int* sflag) {
  using G = Geo<DIM, P>;
  constexpr int NV = G::NV, NPE = G::NPE, NT = G::NT, N1 = G::N1;
  const bool bad = act && !admissible<DIM>(Un, q);
  if (!__syncthreads_or(bad)) return;
  double wn = t.w[node_coord<N1>(node, 0)];
  if (DIM > 1) wn *= t.w[node_coord<N1>(node, 1)];
  if (DIM > 2) wn *= t.w[node_coord<N1>(node, 2)];
#pragma unroll
  for (int v = 0; v < NV; ++v) sbuf[v * NT + tid] = wn * Un[v];
  sflag[tid] = bad ? 1 : 0;
  __syncthreads();
  bool eflag = false;
  for (int n = 0; n < NPE; ++n) eflag |= (sflag[el * NPE + n] != 0);
  double Ub[NV];
  bool avg_ok = false;
  double s = 1.0;
  if (act && eflag) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      double acc = 0.0;
      for (int n = 0; n < NPE; ++n) acc += sbuf[v * NT + el * NPE + n];
      Ub[v] = acc * t.inv_wsum;
    }
    avg_ok = admissible<DIM>(Ub, q);
    if (avg_ok) s = node_factor<DIM>(Un, Ub, q);
    if (node == 0) {
      atomicAdd(&cnt->flagged, 1ull);
      atomicAdd(avg_ok ? &cnt->smoothed : &cnt->bad_average, 1ull);
    }
  }
  __syncthreads();
  sbuf[tid] = s;
  __syncthreads();
  if (act && eflag && avg_ok) {
    double smin = 1.0;
    for (int n = 0; n < NPE; ++n) smin = fmin(smin, sbuf[el * NPE + n]);
#pragma unroll
    for (int v = 0; v < NV; ++v) Un[v] = smin * Un[v] + (1.0 - smin) * Ub[v];
  }
  __syncthreads();
}

template <int DIM, int P>
__global__ __launch_bounds__((Geo<DIM, P>::NT)) void k_enforce(double* __restrict__ U, MeshArgs m, Tables t,
                                                             PhysParams q, Counters* cnt) {
  using G = Geo<DIM, P>;
  constexpr int NV = G::NV, NPE = G::NPE, NT = G::NT, EPB = G::EPB;
  __shared__ double sbuf[NV * NT];
  __shared__ int sflag[NT];
  const int tid = threadIdx.x;
  const int el = tid / NPE, node = tid % NPE;
  const long long e = (long long)blockIdx.x * EPB + el;
  const bool act = e < m.nelem;
  const long long g = e * NPE + node;
  double u[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) u[v] = act ? U[v * m.ntot + g] : 1.0;
  physicality_block<DIM, P>(u, act, tid, el, node, e, t, q, cnt, sbuf, sflag);
  if (act) {
#pragma unroll
    for (int v = 0; v < NV; ++v) U[v * m.ntot + g] = u[v];
  }
}

// ------------------------------------------------------------ element kernel
enum { MODE_RHS = 0, MODE_STAGE = 1 };
enum { PREC_FP64 = 0, PREC_FP32 = 1 };

template <int DIM, int P, int EOS, int PREC, int MODE>
__global__ __launch_bounds__((Geo<DIM, P>::NT)) void k_element(ElemArgs a) {
  using G = Geo<DIM, P>;
  constexpr int N1 = G::N1, NPE = G::NPE, NV = G::NV, NT = G::NT, EPB = G::EPB;
  constexpr int NFP = G::NFP, NF = G::NF, FPB = G::FPB;
  __shared__ double sW[NV * NT];
  __shared__ double sF[NV * NT];
  __shared__ double sFh[NV * FPB];
  // FP32 form: per-line FP64 reference flux (the flux at the line's first node)
  __shared__ double sFref[(PREC == PREC_FP32) ? DIM * NV * EPB * NFP : 1];
  __shared__ int sflag[(MODE == MODE_STAGE) ? NT : 1];

  const MeshArgs& m = a.m;
  const Tables& t = a.t;
  const PhysParams& q = a.q;
  const long long ntot = m.ntot;
  const int tid = threadIdx.x;
  const int el = tid / NPE, node = tid % NPE;
  const int e0 = blockIdx.x * EPB;
  const int e = e0 + el;
  const bool act = e < m.nelem;
  const long long g = (long long)e * NPE + node;

  double W[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) W[v] = act ? a.W[v * ntot + g] : (v == 0 || v == NV - 1 ? 1.0 : 0.0);
#pragma unroll
  for (int v = 0; v < NV; ++v) sW[v * NT + tid] = W[v];

  // ---- volume term: V_i = sum_d (2/dx_d) sum_a dhat[i_d][a] F^d(W at node (i with i_d -> a))
  double R[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) R[v] = 0.0;
  float Rf[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) Rf[v] = 0.0f;
  StateEval<EOS, DIM> sv;
  eval_state<EOS, DIM>(W, q, sv);
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    double F[NV];
    flux_dir<EOS, DIM>(W, sv, d, F);
    __syncthreads();
#pragma unroll
    for (int v = 0; v < NV; ++v) sF[v * NT + tid] = F[v];
    __syncthreads();
    const int id = node_coord<N1>(node, d);
    const int pt = face_pt<DIM, N1>(node, d);
    if constexpr (PREC == PREC_FP64) {
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        double acc = 0.0;
#pragma unroll
        for (int aa = 0; aa < N1; ++aa) acc += t.dhat[id][aa] * sF[v * NT + el * NPE + line_node<DIM, N1>(d, pt, aa)];
        R[v] += m.two_dx[d] * acc;
      }
    } else {
      // deviations from the line's first node, so only the variation along d enters FP32
      const int n0 = el * NPE + line_node<DIM, N1>(d, pt, 0);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const double ref = sF[v * NT + n0];
        float acc = 0.0f;
#pragma unroll
        for (int aa = 0; aa < N1; ++aa)
          acc += t.dhat_f[id][aa] * (float)(sF[v * NT + el * NPE + line_node<DIM, N1>(d, pt, aa)] - ref);
        Rf[v] += (float)m.two_dx[d] * acc;
        if (id == 0) sFref[((d * NV + v) * EPB + el) * NFP + pt] = F[v];
      }
    }
  }
  __syncthreads();

  // ---- faces: primitive traces, exterior state, HLL flux per face point
  for (int fp = tid; fp < FPB; fp += NT) {
    const int fel = fp / (NF * NFP);
    const int rem = fp - fel * NF * NFP;
    const int f = rem / NFP;
    const int pt = rem - f * NFP;
    const int fe = e0 + fel;
    if (fe >= m.nelem) continue;
    const int d = f >> 1;
    const int side = f & 1;  // 1: the + face of the element
    const double* lo = side ? t.lp : t.lm;
    const double* ln = side ? t.lm : t.lp;
    const float* lof = side ? t.lp_f : t.lm_f;
    const float* lnf = side ? t.lm_f : t.lp_f;
    double Wo[NV], Wn[NV];
    const int ob = fel * NPE;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      if constexpr (PREC == PREC_FP64) {
        double acc = 0.0;
#pragma unroll
        for (int aa = 0; aa < N1; ++aa) acc += lo[aa] * sW[v * NT + ob + line_node<DIM, N1>(d, pt, aa)];
        Wo[v] = acc;
      } else {
        const double ref = sW[v * NT + ob + line_node<DIM, N1>(d, pt, 0)];
        float acc = 0.0f;
#pragma unroll
        for (int aa = 0; aa < N1; ++aa) acc += lof[aa] * (float)(sW[v * NT + ob + line_node<DIM, N1>(d, pt, aa)] - ref);
        Wo[v] = ref + (double)acc;
      }
    }
    if (!(Wo[0] > 0.0) || !(Wo[NV - 1] > 0.0)) {
      const int nb = ob + line_node<DIM, N1>(d, pt, side ? P : 0);
#pragma unroll
      for (int v = 0; v < NV; ++v) Wo[v] = sW[v * NT + nb];
      atomicAdd(&a.cnt->trace_fallback, 1ull);
    }
    const int ne = neighbour(m, fe, d, side ? 1 : -1);
    if (ne < 0) {
#pragma unroll
      for (int v = 0; v < NV; ++v) Wn[v] = Wo[v];
    } else {
      const long long nbase = (long long)ne * NPE;
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const double* src = a.W + v * ntot + nbase;
        if constexpr (PREC == PREC_FP64) {
          double acc = 0.0;
#pragma unroll
          for (int aa = 0; aa < N1; ++aa) acc += ln[aa] * src[line_node<DIM, N1>(d, pt, aa)];
          Wn[v] = acc;
        } else {
          const double ref = src[line_node<DIM, N1>(d, pt, 0)];
          float acc = 0.0f;
#pragma unroll
          for (int aa = 0; aa < N1; ++aa) acc += lnf[aa] * (float)(src[line_node<DIM, N1>(d, pt, aa)] - ref);
          Wn[v] = ref + (double)acc;
        }
      }
      if (!(Wn[0] > 0.0) || !(Wn[NV - 1] > 0.0)) {
        const double* src = a.W + nbase + line_node<DIM, N1>(d, pt, side ? 0 : P);
#pragma unroll
        for (int v = 0; v < NV; ++v) Wn[v] = src[v * ntot];
        atomicAdd(&a.cnt->trace_fallback, 1ull);
      }
    }
    double Fh[NV];
    if (side) hll_flux<EOS, DIM>(Wo, Wn, d, q, Fh);
    else hll_flux<EOS, DIM>(Wn, Wo, d, q, Fh);
#pragma unroll
    for (int v = 0; v < NV; ++v) sFh[v * FPB + fp] = Fh[v];
  }
  __syncthreads();

  // ---- lift: S_i = -sum_d (2/dx_d)(1/w_{i_d}) [l_{i_d}(+1) Fhat^+ - l_{i_d}(-1) Fhat^-]
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    const int id = node_coord<N1>(node, d);
    const int pt = face_pt<DIM, N1>(node, d);
    const int ip = (el * NF + 2 * d + 1) * NFP + pt;
    const int im = (el * NF + 2 * d) * NFP + pt;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      if constexpr (PREC == PREC_FP64) {
        R[v] -= m.two_dx[d] * t.iw[id] * (t.lp[id] * sFh[v * FPB + ip] - t.lm[id] * sFh[v * FPB + im]);
      } else {
        const double ref = sFref[((d * NV + v) * EPB + el) * NFP + pt];
        const float fpv = (float)(sFh[v * FPB + ip] - ref);
        const float fmv = (float)(sFh[v * FPB + im] - ref);
        Rf[v] -= (float)m.two_dx[d] * t.iw_f[id] * (t.lp_f[id] * fpv - t.lm_f[id] * fmv);
      }
    }
  }
  if constexpr (PREC == PREC_FP32) {
#pragma unroll
    for (int v = 0; v < NV; ++v) R[v] = (double)Rf[v];
  }

  // ---- epilogue
  if constexpr (MODE == MODE_RHS) {
    if (act) {
#pragma unroll
      for (int v = 0; v < NV; ++v) a.out[v * ntot + g] = R[v];
    }
  } else {
    double Un[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const double un = act ? a.Un[v * ntot + g] : 1.0;
      const double uk = act ? a.Uk[v * ntot + g] : 1.0;
      Un[v] = a.ca * un + a.cb * (uk + a.dt * R[v]);
    }
    if (a.Pout && act) {
#pragma unroll
      for (int v = 0; v < NV; ++v) a.Pout[v * ntot + g] = Un[v];
    }
    if (a.phys) {
      __syncthreads();
      physicality_block<DIM, P>(Un, act, tid, el, node, e, t, q, a.cnt, sF, sflag);
    }
    if (act) {
#pragma unroll
      for (int v = 0; v < NV; ++v) a.out[v * ntot + g] = Un[v];
      if (a.Wout) {
        double Wn[NV];
        const int st = con2prim<EOS, DIM>(Un, Wn, q);
        count_c2p(a.cnt, st, e);
#pragma unroll
        for (int v = 0; v < NV; ++v) a.Wout[v * ntot + g] = Wn[v];
      }
    }
  }
}

}  // namespace dgsrhd
