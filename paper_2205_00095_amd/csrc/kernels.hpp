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
  int bclo[3], bchi[3];         // non-periodic boundary type at the lower / upper end of d
  double bw[3][2][5];           // fixed exterior primitives (rho, u_x, u_y, u_z, P) per d and end
};

// Event counters, one 128-byte set (an L2 cache line) per slot.  A workgroup counts
// into slot blockIdx.x mod kCounterSlots: device-scope atomics from every XCD on one
// cache line serialise (on failure-heavy data that cost milliseconds per stage); the
// host sums the slots (minimum for first_bad) when it reads them.
struct Counters {
  unsigned long long c2p_fail, c2p_noconv, trace_fallback, flagged, smoothed, bad_average, bad_input;
  unsigned long long first_bad;  // lowest failing element (ULLONG_MAX if none)
  unsigned long long limited;    // (element, component) pairs replaced by the slope limiter
  unsigned long long pad[7];
};
static_assert(sizeof(Counters) == 128, "one cache line per slot");
constexpr int kCounterSlots = 256;

__device__ __forceinline__ Counters* counter_slot(Counters* base) {
  return base + (blockIdx.x & (kCounterSlots - 1));
}

struct ElemArgs {
  const double* W;    // primitives of the stage input
  const double* Uk;   // stage input U^(k)          (stage mode)
  const double* Un;   // step start U^n             (stage mode)
  double* out;        // R (rhs mode) or U^(k+1) (stage mode)
  double* Wout;       // primitives of U^(k+1), or null
  double* Pout;       // U^(k+1) before the physicality operator (adjoint tape), or null
  double* avg;        // [NV][nelem] element averages of U^(k+1) (MODE_STAGE_LIM)
  double ca, cb, dt;  // U^(k+1) = ca U^n + cb (U^(k) + dt R); U^n is not read when ca = za = 0
  double za, zb;      // with za != 0 the stored output is za U^n + zb U^(k+1) (after the operator)
  int phys;
  MeshArgs m;
  Tables t;
  PhysParams q;
  Counters* cnt;
  unsigned* opflag;   // set to 1 when the operator changed an element (taped stages), or null
  int rev;            // walk each XCD's tile range backwards (see xcd_tile)
};

// Wave-aggregated event counting: one atomic per wave and counter (the counters are
// hit by many lanes at once on stress data; per-lane atomics on one address serialise).
__device__ __forceinline__ void count_wave(unsigned long long* ctr, bool flag) {
  const unsigned long long m = __ballot(flag);
  if (m == 0ull) return;
  const int leader = __ffsll((long long)m) - 1;
  if ((int)(threadIdx.x & 63) == leader) atomicAdd(ctr, (unsigned long long)__popcll(m));
}

// Block-wide OR of a predicate with one barrier: lane 0 of each wave stores its wave's
// vote in svote[wave], then every lane reads all NW of them.  Each call site needs an
// svote array of its own (a later vote on the same array could overwrite votes that
// slower waves are still reading).  All threads of the block must reach it.
template <int NW>
__device__ __forceinline__ bool block_any(bool pred, int* svote) {
  const bool w = __ballot(pred) != 0ull;
  if ((threadIdx.x & 63) == 0) svote[threadIdx.x >> 6] = w ? 1 : 0;
  __syncthreads();
  int r = 0;
#pragma unroll
  for (int i = 0; i < NW; ++i) r |= svote[i];
  return r != 0;
}

// Ordering of LDS data exchanged only among the nodes of one element.  When NPE divides
// 64 an element's nodes never straddle two waves, and a wave's LDS accesses are
// executed in program order, so it is enough that the compiler keeps that order (a
// wave-scope fence); otherwise a workgroup barrier.
template <int NPE>
__device__ __forceinline__ void element_sync() {
  if constexpr (64 % NPE == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// Sum over the wave's active lanes of a per-lane count below 16 (bitwise ballots).
__device__ __forceinline__ unsigned long long wave_sum16(unsigned x) {
  unsigned long long s = 0;
#pragma unroll
  for (int b = 0; b < 4; ++b) s += (unsigned long long)__popcll(__ballot((x >> b) & 1u)) << b;
  return s;
}

// Recovery status: counts failures / non-convergence and records an element index
// with a failure (the first failing lane of each wave offers its element to an
// atomic minimum).
__device__ __forceinline__ void count_c2p(Counters* cnt, int status, long long elem) {
  const bool fail = status != C2P_OK && status != C2P_NOCONV;
  const bool noconv = status == C2P_NOCONV;
  count_wave(&cnt->c2p_fail, fail);
  count_wave(&cnt->c2p_noconv, noconv);
  const unsigned long long m = __ballot(fail || noconv);
  if (m != 0ull && (int)(threadIdx.x & 63) == __ffsll((long long)m) - 1)
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
  count_c2p(counter_slot(cnt), st, n / npe);
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
#pragma unroll
    for (int v = 0; v < NV; ++v) out[v] = 0.0;
  }
  count_wave(&counter_slot(cnt)->bad_input, !ok);
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
// NV * NT doubles, sflag NT ints and svote one int per wave (for this call only).
// Must be reached by all threads of the block; returns false, after one barrier,
// when no node of the block is flagged.
template <int DIM, int P, int NTB>
__device__ __forceinline__ bool physicality_block_t(double* Un, bool act, int tid, int el, int node,
                                                  const Tables& t, const PhysParams& q, Counters* cnt,
                                                  double* sbuf, int* sflag, int* svote) {
  using G = Geo<DIM, P>;
  constexpr int NV = G::NV, NPE = G::NPE, NT = NTB, N1 = G::N1;
  const bool bad = act && !admissible<DIM>(Un, q);
  if (!block_any<(NT + 63) / 64>(bad, svote)) return false;
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
  }
  const bool lead = act && eflag && node == 0;
  count_wave(&cnt->flagged, lead);
  count_wave(&cnt->smoothed, lead && avg_ok);
  count_wave(&cnt->bad_average, lead && !avg_ok);
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
  return true;
}

// Ordering of LDS data exchanged among the lanes of one wave: a wave's LDS accesses
// execute in program order, so the compiler only has to keep that order.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The operator on the elements of one wave, for layouts in which no element spans two
// waves: the steps and the arithmetic order of physicality_block_t, with wave-scope
// ordering in place of its workgroup barriers.  sbuf holds NV * NTB doubles and sflag
// NTB ints; slot is this lane's slot in them, base the slot of its element's node 0.
// Returns whether any node of the wave was flagged (uniform across the wave).
template <int DIM, int P, int NTB>
__device__ __forceinline__ bool physicality_wave(double* Un, bool act, int slot, int base, int node, const Tables& t,
                                                 const PhysParams& q, Counters* cnt, double* sbuf, int* sflag) {
  using G = Geo<DIM, P>;
  constexpr int NV = G::NV, NPE = G::NPE, NT = NTB, N1 = G::N1;
  const bool bad = act && !admissible<DIM>(Un, q);
  if (__ballot(bad) == 0ull) return false;
  double wn = t.w[node_coord<N1>(node, 0)];
  if (DIM > 1) wn *= t.w[node_coord<N1>(node, 1)];
  if (DIM > 2) wn *= t.w[node_coord<N1>(node, 2)];
#pragma unroll
  for (int v = 0; v < NV; ++v) sbuf[v * NT + slot] = wn * Un[v];
  sflag[slot] = bad ? 1 : 0;
  wave_sync();
  bool eflag = false;
  if (act)
    for (int n = 0; n < NPE; ++n) eflag |= (sflag[base + n] != 0);
  double Ub[NV];
  bool avg_ok = false;
  double s = 1.0;
  if (act && eflag) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      double acc = 0.0;
      for (int n = 0; n < NPE; ++n) acc += sbuf[v * NT + base + n];
      Ub[v] = acc * t.inv_wsum;
    }
    avg_ok = admissible<DIM>(Ub, q);
    if (avg_ok) s = node_factor<DIM>(Un, Ub, q);
  }
  const bool lead = act && eflag && node == 0;
  count_wave(&cnt->flagged, lead);
  count_wave(&cnt->smoothed, lead && avg_ok);
  count_wave(&cnt->bad_average, lead && !avg_ok);
  wave_sync();
  sbuf[slot] = s;
  wave_sync();
  if (act && eflag && avg_ok) {
    double smin = 1.0;
    for (int n = 0; n < NPE; ++n) smin = fmin(smin, sbuf[base + n]);
#pragma unroll
    for (int v = 0; v < NV; ++v) Un[v] = smin * Un[v] + (1.0 - smin) * Ub[v];
  }
  return true;
}

// The operator on a workgroup whose lanes hold consecutive elements (lane = element *
// NPE + node): per wave when NPE divides 64 (no element spans two waves), else with
// workgroup barriers.  Must be reached by all threads of the block.  Returns whether a
// node was flagged in this lane's wave (per-wave form) or block.
template <int DIM, int P, int NTB>
__device__ __forceinline__ bool physicality_t(double* Un, bool act, int tid, int el, int node, const Tables& t,
                                              const PhysParams& q, Counters* cnt, double* sbuf, int* sflag,
                                              int* svote) {
  if constexpr (64 % Geo<DIM, P>::NPE == 0)
    return physicality_wave<DIM, P, NTB>(Un, act, tid, tid - node, node, t, q, cnt, sbuf, sflag);
  else
    return physicality_block_t<DIM, P, NTB>(Un, act, tid, el, node, t, q, cnt, sbuf, sflag, svote);
}

template <int DIM, int P>
__global__ __launch_bounds__((Geo<DIM, P>::NT)) void k_enforce(double* __restrict__ U, MeshArgs m, Tables t,
                                                             PhysParams q, Counters* cnt) {
  using G = Geo<DIM, P>;
  constexpr int NV = G::NV, NPE = G::NPE, NT = G::NT, EPB = G::EPB;
  __shared__ double sbuf[NV * NT];
  __shared__ int sflag[NT];
  __shared__ int svote[(NT + 63) / 64];
  const int tid = threadIdx.x;
  const int el = tid / NPE, node = tid % NPE;
  const long long e = (long long)blockIdx.x * EPB + el;
  const bool act = e < m.nelem;
  const long long g = e * NPE + node;
  double u[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) u[v] = act ? U[v * m.ntot + g] : 1.0;
  physicality_t<DIM, P, NT>(u, act, tid, el, node, t, q, counter_slot(cnt), sbuf, sflag, svote);
  if (act) {
#pragma unroll
    for (int v = 0; v < NV; ++v) U[v * m.ntot + g] = u[v];
  }
}

// ------------------------------------------------------------ element kernel
// MODE_RHS reads the primitives of the nodes from HBM (a recovery launch wrote them);
// MODE_RHS_FUSED reads U and recovers its own nodes and the halo elements across the
// tile's boundary faces itself (one launch, no primitive buffer); MODE_STAGE is one
// SSP-RK stage.
// MODE_STAGE_LIM is the stage ahead of the slope limiter: the RK combination (no
// operator, no folding), the element averages of the result and its primitives.
enum { MODE_RHS = 0, MODE_STAGE = 1, MODE_RHS_FUSED = 2, MODE_STAGE_LIM = 3 };
// PREC_FP32: the volume and lift contractions in FP32 on the vector ALUs; PREC_FP32_MFMA:
// the same with the volume sweeps on the matrix cores (2D, p = 3 only)
enum { PREC_FP64 = 0, PREC_FP32 = 1, PREC_FP32_MFMA = 2 };
typedef float mfma_f32x4 __attribute__((ext_vector_type(4)));

// Tile of elements handled by one workgroup of k_element: TX x TY x TZ elements,
// one node per lane.  Faces inside the tile are evaluated once and shared by the
// two elements through LDS; only the tile's boundary faces are evaluated again by
// the neighbouring tile.
template <int DIM, int P>
struct TileGeo {
  using G = Geo<DIM, P>;
  static constexpr int N1 = G::N1, NPE = G::NPE, NV = G::NV, NFP = G::NFP;
  static constexpr int TX = DIM == 1 ? G::EPB
                          : DIM == 2 ? (P == 0 ? 16 : P == 1 ? 8 : P == 2 ? 7 : 4)
                                     : (P == 0 ? 8 : P == 1 ? 4 : P == 2 ? 3 : 2);
  static constexpr int TY = DIM == 1 ? 1 : DIM == 2 ? (P == 0 ? 16 : P == 1 ? 8 : 4)
                                                    : (P == 0 ? 8 : P == 1 ? 4 : P == 2 ? 3 : 2);
  static constexpr int TZ = DIM < 3 ? 1 : (P == 0 ? 4 : P == 1 ? 2 : 1);
  static constexpr int EPB = TX * TY * TZ;
  static constexpr int NT = EPB * NPE;
  static constexpr int NFX = (TX + 1) * TY * TZ;
  static constexpr int NFY = DIM > 1 ? TX * (TY + 1) * TZ : 0;
  static constexpr int NFZ = DIM > 2 ? TX * TY * (TZ + 1) : 0;
  static constexpr int FOFF1 = NFX * NFP;
  static constexpr int FOFF2 = FOFF1 + NFY * NFP;
  static constexpr int FPB = FOFF2 + NFZ * NFP;  // face points per tile
  static_assert(NT <= 256, "tile larger than a workgroup");
  // halo of the fused right-hand side: the elements across the tile's lowest and highest
  // active faces along each direction, C_d of them per side (the tile's cross-section)
  static constexpr int C0 = TY * TZ, C1 = DIM > 1 ? TX * TZ : 0, C2 = DIM > 2 ? TX * TY : 0;
  static constexpr int NHE = 2 * (C0 + C1 + C2);
  // the fused right-hand side is built where the halo adds at most one recovery per lane
  static constexpr bool kFusedRhs = NHE * NPE <= NT;
};

// index of the face point (direction d, face coordinate f along d, the other two local
// element coordinates, point pt) in the tile's face-point list
template <int DIM, int P>
__device__ __forceinline__ int tile_face_index(int d, int f, const int* l, int pt) {
  using T = TileGeo<DIM, P>;
  int fi;
  if (d == 0) fi = (l[2] * T::TY + l[1]) * (T::TX + 1) + f;
  else if (d == 1) fi = (l[2] * (T::TY + 1) + f) * T::TX + l[0];
  else fi = (f * T::TY + l[1]) * T::TX + l[0];
  const int off = d == 0 ? 0 : (d == 1 ? T::FOFF1 : T::FOFF2);
  return off + fi * T::NFP + pt;
}

template <typename X>
__device__ __forceinline__ X sel3(int d, X a, X b, X c) { return d == 0 ? a : (d == 1 ? b : c); }

// One point of the tile's face-point list, with the addressing of the two elements
// that share its face (the face lies between local elements f-1 and f along d).
// Scalar selects rather than small arrays indexed by the per-lane direction, which
// the compiler would otherwise place in scratch memory.
template <int DIM, int P>
struct TileFacePoint {
  int d, f, pt;
  int fidx;                 // index in the tile's face-point list (tile_face_index)
  int loc0, lstride;        // tile-local element of the face's row at coordinate 0 along d; stride along d
  long long gbase, gstride; // the same in global element numbering
  int od, nnd, per;         // tile origin, mesh extent and periodicity along d
  bool left_local, right_local;

  // point fp of the face-point list (tile_face_index order)
  __device__ __forceinline__ TileFacePoint(int fp, const int* o, const MeshArgs& m) {
    using T = TileGeo<DIM, P>;
    int dd, fi, l0, l1, l2, ff;
    if (fp < T::FOFF1) { dd = 0; fi = fp; }
    else if (DIM > 1 && fp < T::FOFF2) { dd = 1; fi = fp - T::FOFF1; }
    else { dd = 2; fi = fp - T::FOFF2; }
    const int face = fi / T::NFP;
    const int p = fi - face * T::NFP;
    if (dd == 0) {
      ff = face % (T::TX + 1); l1 = (face / (T::TX + 1)) % T::TY; l2 = face / ((T::TX + 1) * T::TY); l0 = 0;
    } else if (dd == 1) {
      l0 = face % T::TX; ff = (face / T::TX) % (T::TY + 1); l2 = face / (T::TX * (T::TY + 1)); l1 = 0;
    } else {
      l0 = face % T::TX; l1 = (face / T::TX) % T::TY; ff = face / (T::TX * T::TY); l2 = 0;
    }
    init(dd, ff, l0, l1, l2, p, o, m);
    fidx = fp;
  }

  // Point taken by slot k of the face phase.  Slots run over the points of the tile's
  // own boundary faces first (f = 0 or f = T_d: one side belongs to a neighbouring
  // tile and is read from HBM), then over the inner ones (both sides in LDS), so a
  // wave meets (nearly) one kind of point and runs one load path per side.
  __device__ __forceinline__ static TileFacePoint from_slot(int k, const int* o, const MeshArgs& m) {
    using T = TileGeo<DIM, P>;
    constexpr int NFP = T::NFP, TX = T::TX, TY = T::TY, TZ = T::TZ;
    constexpr int C0 = TY * TZ, C1 = TX * TZ, C2 = TX * TY;  // faces per tile layer normal to x, y, z
    constexpr int B0 = 2 * C0 * NFP, B1 = DIM > 1 ? 2 * C1 * NFP : 0, B2 = DIM > 2 ? 2 * C2 * NFP : 0;
    constexpr int NB = B0 + B1 + B2;  // boundary points
    constexpr int I0 = (TX - 1) * C0 * NFP, I1 = DIM > 1 ? (TY - 1) * C1 * NFP : 0;
    constexpr int I2 = DIM > 2 ? (TZ - 1) * C2 * NFP : 0;
    static_assert(NB + I0 + I1 + I2 == T::FPB, "every face point has one slot");
    constexpr int N0 = TX > 1 ? TX - 1 : 1, N1 = TY > 1 ? TY - 1 : 1, N2 = TZ > 1 ? TZ - 1 : 1;
    int dd, r, ff, cross;
    if (k < NB) {
      if (DIM == 1 || k < B0) { dd = 0; r = k; }
      else if (DIM == 2 || k < B0 + B1) { dd = 1; r = k - B0; }
      else { dd = 2; r = k - B0 - B1; }
      const int p = r % NFP;
      r /= NFP;
      const int cd = sel3(dd, C0, C1, C2);
      const bool hi = r >= cd;
      cross = hi ? r - cd : r;
      ff = hi ? sel3(dd, TX, TY, TZ) : 0;
      r = p;
    } else {
      r = k - NB;
      if (DIM == 1 || r < I0) { dd = 0; }
      else if (DIM == 2 || r < I0 + I1) { dd = 1; r -= I0; }
      else { dd = 2; r -= I0 + I1; }
      const int p = r % NFP;
      r /= NFP;
      // r = cross (T_d - 1) + f - 1
      cross = sel3(dd, r / N0, r / N1, r / N2);
      ff = 1 + r - cross * sel3(dd, N0, N1, N2);
      r = p;
    }
    // coordinates of the face's cross-section (the one along d is 0)
    const int l0 = dd == 0 ? 0 : cross % TX;
    const int l1 = dd == 0 ? cross % TY : (dd == 1 ? 0 : cross / TX);
    const int l2 = dd == 0 ? cross / TY : (dd == 1 ? cross / TX : 0);
    TileFacePoint fc;
    fc.init(dd, ff, l0, l1, l2, r, o, m);
    const int l[3] = {l0, l1, l2};
    fc.fidx = tile_face_index<DIM, P>(dd, ff, l, r);
    return fc;
  }

  __device__ __forceinline__ TileFacePoint() {}

  __device__ __forceinline__ void init(int dd, int ff, int l0, int l1, int l2, int p, const int* o,
                                       const MeshArgs& m) {
    using T = TileGeo<DIM, P>;
    d = dd;
    f = ff;
    pt = p;
    // the coordinate along d is 0 here and every tile origin lies inside the mesh
    const bool inside = (o[0] + l0 < m.nex) && (o[1] + l1 < m.ney) && (o[2] + l2 < m.nez);
    od = sel3(d, o[0], o[1], o[2]);
    nnd = sel3(d, m.nex, m.ney, m.nez);
    per = sel3(d, m.periodic[0], m.periodic[1], m.periodic[2]);
    lstride = sel3(d, 1, T::TX, T::TX * T::TY);
    loc0 = (l2 * T::TY + l1) * T::TX + l0;
    gstride = sel3<long long>(d, 1, m.nex, (long long)m.nex * m.ney);
    gbase = ((long long)(o[2] + l2) * m.ney + (o[1] + l1)) * m.nex + (o[0] + l0) - (long long)od * gstride;
    const int gl = od + f - 1, gr = od + f;
    left_local = inside && f >= 1 && gl < nnd;
    right_local = inside && f <= sel3(d, T::TX, T::TY, T::TZ) - 1 && gr < nnd;
  }
  __device__ __forceinline__ int left_elem() const { return loc0 + (f - 1) * lstride; }
  __device__ __forceinline__ int right_elem() const { return loc0 + f * lstride; }
  // global element left / right of the face after the periodic wrap, -1 at an outflow boundary
  __device__ __forceinline__ long long left_global() const {
    int g = od + f - 1;
    if (g < 0) {
      if (!per) return -1;
      g += nnd;
    }
    return gbase + g * gstride;
  }
  __device__ __forceinline__ long long right_global() const {
    int g = od + f;
    if (g >= nnd) {
      if (!per) return -1;
      g -= nnd;
    }
    return gbase + g * gstride;
  }
};

// XCD-aware tile order: workgroups are dispatched round-robin over the 8 XCDs
// (hardware block b runs on XCD b % 8), so hardware block b is mapped to logical
// tile start(x) + b / 8, where XCD x owns the contiguous range of nb/8 (+1 for the
// first nb % 8 XCDs) tiles starting at start(x).  Neighbouring tiles, which read
// each other's halo primitives, then share one XCD's L2.  With rev the range is
// walked backwards: consecutive stage launches alternate direction, so a stage
// starts on the tiles whose outputs the previous one wrote last, still in that
// XCD's L2.  A bijection for any nb.
__device__ __forceinline__ int xcd_tile(int b, int nb, int rev = 0) {
  const int q = nb >> 3, r = nb & 7;
  const int x = b & 7, k = b >> 3;
  const int cnt = q + (x < r ? 1 : 0);
  return x * q + min(x, r) + (rev ? cnt - 1 - k : k);
}

// Halo element hs of a tile (TileGeo::NHE of them): direction d, side (0: across the
// lowest active face along d, 1: across the highest), position c in the tile's
// cross-section.  Returns its global element after the periodic wrap, or -1 where
// there is none (a non-periodic mesh end, or a cross-section position outside the mesh).
template <int DIM, int P>
__device__ __forceinline__ long long halo_element(int hs, const int* o, const MeshArgs& m) {
  using T = TileGeo<DIM, P>;
  int d, r;
  if (hs < 2 * T::C0) { d = 0; r = hs; }
  else if (DIM == 2 || hs < 2 * (T::C0 + T::C1)) { d = 1; r = hs - 2 * T::C0; }
  else { d = 2; r = hs - 2 * (T::C0 + T::C1); }
  const int cd = sel3(d, T::C0, T::C1, T::C2);
  const int side = r >= cd ? 1 : 0;
  const int c = r - side * cd;
  int l[3];
  if (d == 0) { l[0] = 0; l[1] = c % T::TY; l[2] = c / T::TY; }
  else if (d == 1) { l[0] = c % T::TX; l[1] = 0; l[2] = c / T::TX; }
  else { l[0] = c % T::TX; l[1] = c / T::TX; l[2] = 0; }
  const int n[3] = {m.nex, m.ney, m.nez};
  int g[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) g[k] = o[k] + l[k];
  // the cross-section position must lie in the mesh
#pragma unroll
  for (int k = 0; k < 3; ++k)
    if (k != d && g[k] >= n[k]) return -1;
  const int td = sel3(d, T::TX, T::TY, T::TZ);
  const int od = sel3(d, o[0], o[1], o[2]);
  const int nd = sel3(d, n[0], n[1], n[2]);
  const int nact = min(td, nd - od);  // active elements of the tile along d
  int gd = side ? od + nact : od - 1;
  if (gd < 0 || gd >= nd) {
    if (!sel3(d, m.periodic[0], m.periodic[1], m.periodic[2])) return -1;
    gd = gd < 0 ? gd + nd : gd - nd;
  }
  if (d == 0) g[0] = gd; else if (d == 1) g[1] = gd; else g[2] = gd;
  return ((long long)g[2] * m.ney + g[1]) * m.nex + g[0];
}

// Halo slot of the element across face point fc when that element is not in the tile:
// side 1 for a face whose left element is in the tile (the highest active face), else 0.
template <int DIM, int P>
__device__ __forceinline__ int halo_slot(int d, bool a_left, int loc0) {
  using T = TileGeo<DIM, P>;
  int c;
  if (d == 0) c = loc0 / T::TX;
  else if (d == 1) c = (loc0 / (T::TX * T::TY)) * T::TX + loc0 % T::TX;
  else c = loc0;
  const int off = d == 0 ? 0 : (d == 1 ? 2 * T::C0 : 2 * (T::C0 + T::C1));
  const int cd = sel3(d, T::C0, T::C1, T::C2);
  return off + (a_left ? cd : 0) + c;
}

enum { BC_OUTFLOW = 1, BC_REFLECT = 2, BC_FIXED = 3 };

// Exterior state at a boundary face of direction d from the interior trace Wi: outflow
// (the trace), a reflecting wall (its mirror image, u_d negated) or a fixed state.
// `upper` selects the end (the interior element lies below the face).
template <int DIM>
__device__ __forceinline__ void exterior_state(const MeshArgs& m, int d, bool upper, const double* Wi,
                                               double* We) {
  constexpr int NV = DIM + 2;
  const int kind = upper ? sel3(d, m.bchi[0], m.bchi[1], m.bchi[2]) : sel3(d, m.bclo[0], m.bclo[1], m.bclo[2]);
#pragma unroll
  for (int v = 0; v < NV; ++v) We[v] = Wi[v];
  if (kind == BC_REFLECT) comp_add<DIM>(We + 1, d, -2.0 * comp<DIM>(We + 1, d));
  if (kind == BC_FIXED) {
    const double* w = m.bw[d][upper ? 1 : 0];
    We[0] = w[0];
#pragma unroll
    for (int j = 0; j < DIM; ++j) We[1 + j] = w[1 + j];
    We[NV - 1] = w[4];
  }
}

// Primitive trace at one point of an element face normal to d, interpolated along the
// element's line of nodes through that point (Sec. 2.4 traces, reading R12 for the
// fallback).  The weights are l_b(+1) taken over the nodes n0, n0 + step, ...,
// n0 + P step: on the element's + face n0 is the line's first node and step its
// stride, on its - face n0 is the last node and step the negated stride, since
// l_b(-1) = l_{P-b}(+1) on the symmetric Gauss-Legendre nodes.  When rho or P
// interpolates to <= 0 the primitives of the node nearest the face
// (n0 + P step) are used instead; returns whether that happened.
template <int NV, int NT, int P>
__device__ __forceinline__ bool trace_lds(const double* sW, int n0, int step, const Tables& t, double* Wt) {
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    double acc = 0.0;
#pragma unroll
    for (int b = 0; b <= P; ++b) acc += t.lp[b] * sW[v * NT + n0 + b * step];
    Wt[v] = acc;
  }
  if (!(Wt[0] > 0.0) || !(Wt[NV - 1] > 0.0)) {
#pragma unroll
    for (int v = 0; v < NV; ++v) Wt[v] = sW[v * NT + n0 + P * step];
    return true;
  }
  return false;
}

// The same from the state in HBM: src points at node n0 of component 0.
template <int NV, int P>
__device__ __forceinline__ bool trace_glb(const double* src, long long ntot, int step, const Tables& t,
                                          double* Wt) {
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    double acc = 0.0;
#pragma unroll
    for (int b = 0; b <= P; ++b) acc += t.lp[b] * src[v * ntot + b * step];
    Wt[v] = acc;
  }
  if (!(Wt[0] > 0.0) || !(Wt[NV - 1] > 0.0)) {
#pragma unroll
    for (int v = 0; v < NV; ++v) Wt[v] = src[v * ntot + P * step];
    return true;
  }
  return false;
}

// Materialise a value in registers at this point of the program: its computation
// cannot be sunk below it (an empty asm that reads and writes the register).
__device__ __forceinline__ void pin_reg(double& x) { asm volatile("" : "+v"(x)); }
__device__ __forceinline__ void pin_reg(float& x) { asm volatile("" : "+v"(x)); }

// Waves per SIMD the element kernel is compiled for: the 2D p >= 2 kernels sit a
// few VGPRs above the 96 that 5 waves allow, and bounded to 96 they spill at most
// four registers; elsewhere the compiler's allocation stands (a bound spills
// heavily, or LDS limits the occupancy anyway).
template <int DIM, int P>
constexpr int elem_min_waves() { return (DIM == 2 && P >= 2) ? 5 : 1; }

template <int DIM, int P, int EOS, int PREC, int MODE, int FLUX>
__global__ __launch_bounds__((TileGeo<DIM, P>::NT), (elem_min_waves<DIM, P>())) void k_element(ElemArgs a) {
  using T = TileGeo<DIM, P>;
  constexpr int N1 = T::N1, NPE = T::NPE, NV = T::NV, NT = T::NT, EPB = T::EPB;
  constexpr int NFP = T::NFP, FPB = T::FPB, TX = T::TX, TY = T::TY, TZ = T::TZ;
  // sW and sF hold one value per node and variable, elements ES apart: one unused
  // slot after each element when NPE is even, so that the lanes reading the same
  // node of neighbouring elements fall in different LDS banks
  constexpr int ES = NPE % 2 == 0 ? NPE + 1 : NPE, NTP = EPB * ES;
  __shared__ double sW[NV * NTP];
  __shared__ double sF[NV * NTP];
  __shared__ double sFh[NV * FPB];
  __shared__ double sFref[(PREC != PREC_FP64) ? DIM * NV * EPB * NFP : 1];
  static_assert(PREC != PREC_FP32_MFMA || (DIM == 2 && P == 3), "MFMA sweeps are built for 2D p = 3");
  constexpr bool kStage = MODE == MODE_STAGE || MODE == MODE_STAGE_LIM;
  __shared__ int sflag[(MODE == MODE_STAGE) ? NT : 1];
  __shared__ int svote[(NT + 63) / 64];
  // fused right-hand side: the primitives of the halo elements, recovered in the tile
  constexpr bool kFused = MODE == MODE_RHS_FUSED;
  static_assert(!kFused || T::kFusedRhs, "fused right-hand side needs a halo of at most one node per lane");
  constexpr int NHP = T::NHE * ES;
  __shared__ double sWh[kFused ? NV * NHP : 1];

  const MeshArgs& m = a.m;
  const Tables& t = a.t;
  const PhysParams& q = a.q;
  const long long ntot = m.ntot;
  const int tid = threadIdx.x;
  const int el = tid / NPE, node = tid % NPE;
  // tile origin
  const int ntx = (m.nex + TX - 1) / TX, nty = (m.ney + TY - 1) / TY, ntz = (m.nez + TZ - 1) / TZ;
  const int tile = xcd_tile(blockIdx.x, ntx * nty * ntz, a.rev);
  const int o[3] = {(tile % ntx) * TX, ((tile / ntx) % nty) * TY, (tile / (ntx * nty)) * TZ};
  const int lc[3] = {el % TX, (el / TX) % TY, el / (TX * TY)};
  const bool act = (o[0] + lc[0] < m.nex) && (o[1] + lc[1] < m.ney) && (o[2] + lc[2] < m.nez);
  const long long e = act ? ((long long)(o[2] + lc[2]) * m.ney + (o[1] + lc[1])) * m.nex + (o[0] + lc[0]) : 0;
  const long long g = e * NPE + node;

  double W[NV];
  if constexpr (kFused) {
    // recover this node's primitives and those of one halo node (at most), both loads first
    constexpr int NHN = T::NHE * NPE;
    const int hs = tid / NPE;  // halo element of this lane's halo node (tid < NHN)
    const long long hg = tid < NHN ? halo_element<DIM, P>(hs, o, m) : -1;
    double u[NV], uh[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) u[v] = act ? a.Uk[v * ntot + g] : 0.0;
#pragma unroll
    for (int v = 0; v < NV; ++v) uh[v] = hg >= 0 ? a.Uk[v * ntot + hg * NPE + node] : 0.0;
    if (act) {
      const int st = con2prim<EOS, DIM>(u, W, q);
      count_c2p(counter_slot(a.cnt), st, e);
    } else {
#pragma unroll
      for (int v = 0; v < NV; ++v) W[v] = (v == 0 || v == NV - 1) ? 1.0 : 0.0;
    }
    if (hg >= 0) {
      // counted by the tile that owns the element, not here
      double wh[NV];
      (void)con2prim<EOS, DIM>(uh, wh, q);
#pragma unroll
      for (int v = 0; v < NV; ++v) sWh[v * NHP + hs * ES + node] = wh[v];
    }
  } else {
#pragma unroll
    for (int v = 0; v < NV; ++v) W[v] = act ? a.W[v * ntot + g] : (v == 0 || v == NV - 1 ? 1.0 : 0.0);
  }
  const int ln = el * ES + node;  // this node's slot in sW and sF
#pragma unroll
  for (int v = 0; v < NV; ++v) sW[v * NTP + ln] = W[v];

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
    element_sync<NPE>();  // the previous direction's reads of sF are done
#pragma unroll
    for (int v = 0; v < NV; ++v) sF[v * NTP + ln] = F[v];
    element_sync<NPE>();
    const int id = node_coord<N1>(node, d);
    const int pt = face_pt<DIM, N1>(node, d);
    if constexpr (PREC == PREC_FP64) {
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        double acc = 0.0;
#pragma unroll
        for (int aa = 0; aa < N1; ++aa) acc += t.dhat[id][aa] * sF[v * NTP + el * ES + line_node<DIM, N1>(d, pt, aa)];
        R[v] += m.two_dx[d] * acc;
      }
    } else if constexpr (PREC == PREC_FP32_MFMA) {
      // The same deviations contracted on the matrix cores: v_mfma_f32_4x4x1f32 forms 16
      // independent 4x4 outer products per wave and instruction, block b from lanes
      // 4b..4b+3, row r from lane 4b+r (operand A), column c from lane 4b+c (operand B),
      // the 4x4 result in lane 4b+c, one row per accumulator register.  With one node per
      // lane (lane = 16 e + 4 j + i in a wave's four elements, 2D p = 3) a block is a line
      // of nodes: rows are the 4 conserved variables (NV = 4), columns the 4 output nodes
      // along the line, K runs over the 4 nodes of the line in four instructions.  Along x
      // the line is the lane's own j and the result lands in the lane's own node; along y
      // the block's line is the lane's i, the result lands in the transposed lane (16 e +
      // 4 i + j) and one lane permute per variable brings it home.
      const int lane = tid & 63;
      const int qq = lane & 3, jl = (lane >> 2) & 3;
      const int eb = el * ES;
      const int n0 = d == 0 ? jl * 4 : jl;  // the block line's first node
      const double ref = sF[qq * NTP + eb + n0];
      mfma_f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int aa = 0; aa < 4; ++aa) {
        const int na = d == 0 ? jl * 4 + aa : aa * 4 + jl;
        const float A = (float)(sF[qq * NTP + eb + na] - ref);
        acc = __builtin_amdgcn_mfma_f32_4x4x1f32(A, t.dhat_f[qq][aa], acc, 0, 0, 0);
      }
      const int src = d == 0 ? lane : ((lane & ~15) | (qq << 2) | jl);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const float r = d == 0 ? acc[v] : __shfl(acc[v], src, 64);
        Rf[v] += (float)m.two_dx[d] * r;
        if (id == 0) sFref[((d * NV + v) * EPB + el) * NFP + pt] = F[v];
      }
    } else {
      // deviations from the line's first node, so only the variation along d enters FP32
      const int n0 = el * ES + line_node<DIM, N1>(d, pt, 0);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const double ref = sF[v * NTP + n0];
        float acc = 0.0f;
#pragma unroll
        for (int aa = 0; aa < N1; ++aa)
          acc += t.dhat_f[id][aa] * (float)(sF[v * NTP + el * ES + line_node<DIM, N1>(d, pt, aa)] - ref);
        Rf[v] += (float)m.two_dx[d] * acc;
        if (id == 0) sFref[((d * NV + v) * EPB + el) * NFP + pt] = F[v];
      }
    }
  }
  // end the contraction here: left to itself the compiler sinks these FMAs to the
  // lift and keeps all the loaded fluxes live through the face phase (~70 VGPRs)
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    if constexpr (PREC == PREC_FP64) pin_reg(R[v]);
    else pin_reg(Rf[v]);
  }
  __syncthreads();
  // rhs mode: the volume result waits in sF (free from here on) through the face phase,
  // which lowers the register peak to 6 waves per SIMD for 2D p = 3 (measured 3% faster;
  // the stage kernel gains nothing from it)
  constexpr bool kParkR = (MODE == MODE_RHS || MODE == MODE_RHS_FUSED) && PREC == PREC_FP64;
  if constexpr (kParkR) {
#pragma unroll
    for (int v = 0; v < NV; ++v) sF[v * NTP + ln] = R[v];
  }

  // ---- faces of the tile: primitive traces (FP64), exterior states, HLL flux per face point.
  // Side A of a face point is an element in this tile (the left one when it is), side B
  // the other one: in this tile (LDS), in a neighbouring tile (HBM), or absent at an
  // outflow boundary, where the exterior state equals the interior trace.
  unsigned nfb = 0;  // trace fallbacks seen by this lane
  for (int k = tid; k < FPB; k += NT) {
    const TileFacePoint<DIM, P> fc = TileFacePoint<DIM, P>::from_slot(k, o, m);
    if (!fc.left_local && !fc.right_local) continue;
    const int d = fc.d;
    const int line0 = line_node<DIM, N1>(d, fc.pt, 0);
    const int stride = sel3(d, 1, N1, N1 * N1);
    const bool a_left = fc.left_local;
    // + face of the left element: forward along the line; - face of the right: backward
    const int fwd0 = line0, bwd0 = line0 + P * stride;
    double WA[NV], WB[NV];
    {
      const int ob = (a_left ? fc.left_elem() : fc.right_elem()) * ES;
      nfb += trace_lds<NV, NTP, P>(sW, ob + (a_left ? fwd0 : bwd0), a_left ? stride : -stride, t, WA);
    }
    if (a_left && fc.right_local) {
      nfb += trace_lds<NV, NTP, P>(sW, fc.right_elem() * ES + bwd0, -stride, t, WB);
    } else {
      const long long ge = a_left ? fc.right_global() : fc.left_global();
      if (ge >= 0) {
        if constexpr (kFused) {
          const int hb = halo_slot<DIM, P>(d, a_left, fc.loc0) * ES;
          nfb += trace_lds<NV, NHP, P>(sWh, hb + (a_left ? bwd0 : fwd0), a_left ? -stride : stride, t, WB);
        } else {
          nfb += trace_glb<NV, P>(a.W + ge * NPE + (a_left ? bwd0 : fwd0), ntot, a_left ? -stride : stride, t, WB);
        }
      } else {
        // no neighbour: a boundary face (side A's element is below it at the upper end)
        exterior_state<DIM>(m, d, a_left, WA, WB);
      }
    }
    double WL[NV], WR[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      WL[v] = a_left ? WA[v] : WB[v];
      WR[v] = a_left ? WB[v] : WA[v];
    }
    double Fh[NV];
    if constexpr (FLUX == FLUX_HLLC)
      hllc_flux<EOS, DIM>(WL, WR, d, q, Fh);
    else
      hll_flux<EOS, DIM>(WL, WR, d, q, Fh);
#pragma unroll
    for (int v = 0; v < NV; ++v) sFh[v * FPB + fc.fidx] = Fh[v];
  }
  // lift weights (2/dx_d)(1/w_i) l_i(+-1) of this node, fetched (per-lane table loads)
  // and formed before the barrier so that their latency overlaps the wait
  double cpl[DIM], cml[DIM];
  if constexpr (PREC == PREC_FP64) {
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const int id = node_coord<N1>(node, d);
      const double sc = m.two_dx[d] * t.iw[id];
      cpl[d] = sc * t.lp[id];
      cml[d] = sc * t.lm[id];
      pin_reg(cpl[d]);
      pin_reg(cml[d]);
    }
  }
  // the epilogue's state loads, issued before the barrier (inactive lanes read element 0)
  double Ukv[NV], U0v[NV];
  const bool need_u0 = kStage && (a.ca != 0.0 || a.za != 0.0);
  if constexpr (kStage) {
#pragma unroll
    for (int v = 0; v < NV; ++v) Ukv[v] = a.Uk[v * ntot + g];
#pragma unroll
    for (int v = 0; v < NV; ++v) U0v[v] = 0.0;
    if (need_u0) {
#pragma unroll
      for (int v = 0; v < NV; ++v) U0v[v] = a.Un[v * ntot + g];
    }
  }
  // trace fallbacks: one atomic per wave that saw any (all lanes are active here)
  static_assert(2 * ((FPB + NT - 1) / NT) < 16, "per-lane fallback count fits wave_sum16");
  {
    const unsigned long long w = wave_sum16(nfb);
    if (w != 0ull && (tid & 63) == 0) atomicAdd(&counter_slot(a.cnt)->trace_fallback, w);
  }
  __syncthreads();

  // ---- lift: S_i = -sum_d (2/dx_d)(1/w_{i_d}) [l_{i_d}(+1) Fhat^+ - l_{i_d}(-1) Fhat^-]
  if constexpr (kParkR) {
#pragma unroll
    for (int v = 0; v < NV; ++v) R[v] = sF[v * NTP + ln];
  }
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    const int id = node_coord<N1>(node, d);
    const int pt = face_pt<DIM, N1>(node, d);
    const int im = tile_face_index<DIM, P>(d, lc[d], lc, pt);
    const int ip = tile_face_index<DIM, P>(d, lc[d] + 1, lc, pt);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      if constexpr (PREC == PREC_FP64) {
        R[v] -= cpl[d] * sFh[v * FPB + ip] - cml[d] * sFh[v * FPB + im];
      } else {
        const double ref = sFref[((d * NV + v) * EPB + el) * NFP + pt];
        const float fpv = (float)(sFh[v * FPB + ip] - ref);
        const float fmv = (float)(sFh[v * FPB + im] - ref);
        Rf[v] -= (float)m.two_dx[d] * t.iw_f[id] * (t.lp_f[id] * fpv - t.lm_f[id] * fmv);
      }
    }
  }
  if constexpr (PREC != PREC_FP64) {
#pragma unroll
    for (int v = 0; v < NV; ++v) R[v] = (double)Rf[v];
  }

  // ---- epilogue
  if constexpr (MODE == MODE_RHS || MODE == MODE_RHS_FUSED) {
    if (act) {
#pragma unroll
      for (int v = 0; v < NV; ++v) a.out[v * ntot + g] = R[v];
    }
  } else {
    double Un[NV], U0[NV];  // U^(k+1), U^n
#pragma unroll
    for (int v = 0; v < NV; ++v) U0[v] = act ? U0v[v] : 0.0;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const double uk = act ? Ukv[v] : 1.0;
      Un[v] = a.ca * U0[v] + a.cb * (uk + a.dt * R[v]);
    }
    if constexpr (MODE == MODE_STAGE_LIM) {
      // the unlimited stage and its element averages (quadrature sum in node order);
      // sF was last read in the volume phase, before the face phase's closing barrier
      if (act) {
#pragma unroll
        for (int v = 0; v < NV; ++v) a.out[v * ntot + g] = Un[v];
      }
      double wn = t.w[node_coord<N1>(node, 0)];
      if (DIM > 1) wn *= t.w[node_coord<N1>(node, 1)];
      if (DIM > 2) wn *= t.w[node_coord<N1>(node, 2)];
#pragma unroll
      for (int v = 0; v < NV; ++v) sF[v * NTP + ln] = wn * Un[v];
      __syncthreads();
      if (act) {
        for (int v = node; v < NV; v += NPE) {
          double acc = 0.0;
          for (int n = 0; n < NPE; ++n) acc += sF[v * NTP + el * ES + n];
          a.avg[(long long)v * m.nelem + e] = acc * t.inv_wsum;
        }
      }
      // the next stage's primitives of every node, Newton started from this stage's
      // input (the limiter launch recovers again only the nodes it changes); not
      // counted here: a node whose recovery fails is marked with a NaN density, and the
      // limiter launch recovers and counts it
      if (act && a.Wout) {
        double Wn[NV], Wp[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) Wp[v] = sW[v * NTP + ln];
        const int st = con2prim<EOS, DIM>(Un, Wn, q, Wp, false);
        if (st != C2P_OK) Wn[0] = __builtin_nan("");
#pragma unroll
        for (int v = 0; v < NV; ++v) a.Wout[v * ntot + g] = Wn[v];
      }
      return;
    }
    if (a.Pout && act) {
#pragma unroll
      for (int v = 0; v < NV; ++v) a.Pout[v * ntot + g] = Un[v];
    }
    // true when the operator ran on this lane's wave (or tile); otherwise every node
    // passed its admissibility test and the recovery need not repeat it
    bool changed = true;
    if (a.phys) {
      // sF was last read in the volume phase, before the face phase's closing barrier
      // (the FP32 vector-sweep form keeps the workgroup form and its single flag write:
      // with the per-wave form that kernel spills past its register bound, 10% slower)
      if constexpr (PREC == PREC_FP32)
        changed = physicality_block_t<DIM, P, NT>(Un, act, tid, el, node, t, q, counter_slot(a.cnt), sF, sflag, svote);
      else
        changed = physicality_t<DIM, P, NT>(Un, act, tid, el, node, t, q, counter_slot(a.cnt), sF, sflag, svote);
      if (a.opflag && changed && (PREC == PREC_FP32 ? tid == 0 : (tid & 63) == 0)) *a.opflag = 1u;
    }
    if (act) {
      if (a.za != 0.0) {
#pragma unroll
        for (int v = 0; v < NV; ++v) a.out[v * ntot + g] = a.za * U0[v] + a.zb * Un[v];
      } else {
#pragma unroll
        for (int v = 0; v < NV; ++v) a.out[v * ntot + g] = Un[v];
      }
      if (a.Wout) {
        double Wn[NV];
        double Wp[NV];  // this node's primitives at the start of the stage (Newton start)
#pragma unroll
        for (int v = 0; v < NV; ++v) Wp[v] = sW[v * NTP + ln];
        const int st = con2prim<EOS, DIM>(Un, Wn, q, Wp, !changed);
        count_c2p(counter_slot(a.cnt), st, e);
#pragma unroll
        for (int v = 0; v < NV; ++v) a.Wout[v * ntot + g] = Wn[v];
      }
    }
  }
}

}  // namespace dgsrhd
