// Device-side SRHD physics for the gfx950 kernels: equations of state (Sec. 2.2),
// primitive/conserved relations and fluxes (Sec. 2.1), wavespeeds and the HLL
// numerical flux (Sec. 2.4), admissibility (Sec. 2.5, Eq. physicality) and the
// four conserved-to-primitive solvers of Sec. 3.  Everything is FP64 and lives
// in registers; one node (or one face point) per lane.
//
// Variables: primitive W = (rho, u_1..u_DIM, P) with u = gamma v the spatial
// 4-velocity; conserved U = (D, S_1..S_DIM, tau) with S the momentum density and
// tau = E - D c^2.
#pragma once
#include <hip/hip_runtime.h>

namespace dgsrhd {

enum { EOS_IDEAL = 0, EOS_TM = 1 };
enum { C2P_NEWTON = 0, C2P_QUARTIC = 1, C2P_CUBIC = 2, C2P_BRENT = 3 };
enum { C2P_OK = 0, C2P_INADMISSIBLE = 1, C2P_NOCONV = 2, C2P_BADP = 3 };
enum { FLUX_HLL = 0, FLUX_HLLC = 1 };

// Floor state written for a failed recovery: rho = 1e-10, u = 0, P = 1e-10 c^2.
constexpr double kRhoFloor = 1e-10;
constexpr double kPFloor = 1e-10;

struct PhysParams {
  double c, c2, c4, inv_c, inv_c2;
  double gam;    // adiabatic index Gamma (ideal EOS)
  double gm1;    // Gamma - 1
  double alpha;  // Gamma / (Gamma - 1)
  double eps;    // relative margin of the physicality operator
  int c2p;       // recovery solver
  int c2p_iters; // > 0: the fixed-iteration solvers of the recovery study (Sec. 3.3): exactly
                 // this many Newton steps from w = 1/2 (ideal EOS, no convergence test) or
                 // at most this many Brent steps (TM EOS)
};

// ---------------------------------------------------------------- EOS (Sec. 2.2)
// h - c^2 as a function of Theta = P / rho.  Taub-Matthews:
// h = 5/2 Theta + 3/2 sqrt(Theta^2 + 4/9 c^4); the excess over c^2 is
// 5/2 Theta + 3/2 Theta^2 / (sqrt(Theta^2 + 4/9 c^4) + 2/3 c^2), free of cancellation.
template <int EOS>
__host__ __device__ __forceinline__ double h_excess(double th, const PhysParams& q) {
  if constexpr (EOS == EOS_IDEAL) {
    return q.alpha * th;
  } else {
    const double s = sqrt(th * th + (4.0 / 9.0) * q.c4);
    return 2.5 * th + 1.5 * th * th / (s + (2.0 / 3.0) * q.c2);
  }
}

// 1 / sqrt(x): the device's reciprocal square root (one refined v_rsq), the plain
// quotient on the host
__host__ __device__ __forceinline__ double inv_sqrt(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return rsqrt(x);
#else
  return 1.0 / sqrt(x);
#endif
}

// sqrt(x) for x >= 0 as x * (1 / sqrt(x)) through the reciprocal square root: fewer
// instructions than the correctly rounded root, within a few ulp.  Exact 0 at x = 0;
// NaN for x < 0 or NaN, as sqrt.
__host__ __device__ __forceinline__ double sqrt_pos(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return x == 0.0 ? 0.0 : x * rsqrt(x);
#else
  return sqrt(x);
#endif
}

// 1 / x to about 2^-44 relative: the device's reciprocal with one Newton refinement
// (a quotient to that accuracy is enough for a Newton step that is not the last);
// the plain quotient on the host
__host__ __device__ __forceinline__ double rcp_refined(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  const double r = __builtin_amdgcn_rcp(x);
  return fma(fma(-x, r, 1.0), r, r);
#else
  return 1.0 / x;
#endif
}

// Component d of a DIM-vector stored from v[0], for a direction known only at run
// time: a chain of selects over values.  An indexed access would move the array to
// scratch memory, and so would the optimiser's folding of a select of two loads into
// one indexed load, which the empty asm (device pass only) hides the loads from.
__host__ __device__ __forceinline__ double opaque(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  asm("" : "+v"(x));
#endif
  return x;
}
template <int DIM>
__host__ __device__ __forceinline__ double comp(const double* v, int d) {
  double x = opaque(v[0]);
#pragma unroll
  for (int j = 1; j < DIM; ++j) x = (d == j) ? opaque(v[j]) : x;
  return x;
}
template <int DIM>
__host__ __device__ __forceinline__ void comp_add(double* v, int d, double x) {
#pragma unroll
  for (int j = 0; j < DIM; ++j)
    if (d == j) v[j] += x;
}

// ------------------------------------------------- state relations (Sec. 2.1)
// Everything a face or node needs from a primitive state: conserved variables
// (Eq. primitive_to_conserved) and the pieces shared by fluxes and wavespeeds.
template <int EOS, int DIM>
struct StateEval {
  double U[DIM + 2];
  double g2, ig;  // gamma^2, 1/gamma
  double P;
  double th, he;  // Theta, h - c^2
  double sq;      // Taub-Matthews: sqrt(Theta^2 + 4/9 c^4)
  double isq;     // Taub-Matthews: 1 / sq
  double r;       // 1 / (rho (gamma + 1))
};

template <int EOS, int DIM>
__host__ __device__ __forceinline__ void eval_state(const double* W, const PhysParams& q, StateEval<EOS, DIM>& s) {
  const double rho = W[0];
  const double P = W[DIM + 1];
  double usq = 0.0;
#pragma unroll
  for (int j = 0; j < DIM; ++j) usq += W[1 + j] * W[1 + j];
  const double g2 = 1.0 + usq * q.inv_c2;
  const double ig = inv_sqrt(g2);
  const double g = g2 * ig;
  // one reciprocal for Theta = P / rho and for 1 / (gamma + 1) in tau
  const double r = 1.0 / (rho * (g + 1.0));
  const double th = P * (g + 1.0) * r;
  double he;
  if constexpr (EOS == EOS_IDEAL) {
    he = q.alpha * th;
    s.sq = 0.0;
    s.isq = 0.0;
  } else {
    const double x = th * th + (4.0 / 9.0) * q.c4;  // > 0
    s.isq = inv_sqrt(x);
    s.sq = x * s.isq;
    // th^2 / (sq + 2/3 c^2) equals sq - 2/3 c^2; the difference costs no division and,
    // for Theta >= c^2 / 3, loses at most a factor 18 to cancellation (a few 1e-16 of he)
    const double a = (2.0 / 3.0) * q.c2;
    if (th >= 0.5 * a) {
      he = 2.5 * th + 1.5 * (s.sq - a);
    } else {
      he = 2.5 * th + 1.5 * th * th / (s.sq + a);
    }
  }
  const double D = g * rho;
  const double gH = g * rho * (q.c2 + he) * q.inv_c2;  // gamma rho h / c^2
  s.U[0] = D;
#pragma unroll
  for (int j = 0; j < DIM; ++j) s.U[1 + j] = gH * W[1 + j];
  // tau = gamma^2 rho h - P - D c^2 = D |u|^2/(gamma+1) + gamma^2 rho (h - c^2) - P
  s.U[DIM + 1] = D * usq * (rho * r) + g2 * rho * he - P;
  s.g2 = g2;
  s.ig = ig;
  s.P = P;
  s.th = th;
  s.he = he;
  s.r = r;
}

// Physical flux along direction d in (D, S, tau) variables (Eq. srhd_flux with the
// energy row minus c^2 times the mass row): (D v_d, S v_d + P e_d, (tau + P) v_d).
template <int EOS, int DIM>
__host__ __device__ __forceinline__ void flux_dir(const double* W, const StateEval<EOS, DIM>& s, int d, double* F) {
  const double vd = comp<DIM>(W + 1, d) * s.ig;
#pragma unroll
  for (int k = 0; k < DIM + 2; ++k) F[k] = s.U[k] * vd;
#pragma unroll
  for (int j = 0; j < DIM; ++j)
    if (j == d) F[1 + j] += s.P;
  F[DIM + 1] += s.P * vd;
}

// Extreme signal speeds along d (Sec. 2.4):
// lambda_pm = (v_d pm sqrt(sigma (c^2 - v_d^2 + c^2 sigma)))/(1 + sigma),
// sigma = c_s^2 / (gamma^2 (c^2 - c_s^2)).  With c_s^2 = c^2 N / M from the EOS
// (ideal: N = Gamma Theta, M = c^2 + alpha Theta; Taub-Matthews: N = 3 Theta^2 +
// 5 Theta s, M = 12 Theta^2 + 2 c^4 + 12 Theta s) and K = M - N, multiplying through
// by gamma^2 K gives the same speeds with one division:
// lambda_pm = (v_d gamma^2 K pm sqrt(N (gamma^2 K (c^2 - v_d^2) + c^2 N))) / (gamma^2 K + N).
// K is formed without cancellation: c^2 + (alpha - Gamma) Theta (alpha >= Gamma for
// Gamma <= 2), resp. 9 Theta^2 + 7 Theta s + 2 c^4.
template <int EOS, int DIM>
__host__ __device__ __forceinline__ void wavespeeds_nd(const double* W, const StateEval<EOS, DIM>& s, int d,
                                                      const PhysParams& q, double& nm, double& np, double& den) {
  double N, K;
  if constexpr (EOS == EOS_IDEAL) {
    N = q.gam * s.th;
    K = q.c2 + (q.alpha - q.gam) * s.th;
  } else {
    const double th = s.th;
    N = th * (3.0 * th + 5.0 * s.sq);
    K = th * (9.0 * th + 7.0 * s.sq) + 2.0 * q.c4;
  }
  const double vd = comp<DIM>(W + 1, d) * s.ig;
  const double gK = s.g2 * K;
  const double root = sqrt_pos(N * (gK * (q.c2 - vd * vd) + q.c2 * N));
  den = gK + N;  // > 0
  nm = vd * gK - root;
  np = vd * gK + root;
}

template <int EOS, int DIM>
__host__ __device__ __forceinline__ void wavespeeds(const double* W, const StateEval<EOS, DIM>& s, int d,
                                                   const PhysParams& q, double& lm, double& lp) {
  double nm, np, den;
  wavespeeds_nd<EOS, DIM>(W, s, d, q, nm, np, den);
  const double inv = 1.0 / den;
  lm = nm * inv;
  lp = np * inv;
}

// HLL numerical flux along d between left and right primitive states
// (lambda_L = min of the two lambda_-, lambda_R = max of the two lambda_+).
template <int EOS, int DIM>
__host__ __device__ __forceinline__ void hll_flux(const double* WL, const double* WR, int d, const PhysParams& q,
                                         double* Fh) {
  constexpr int NV = DIM + 2;
  StateEval<EOS, DIM> sL, sR;
  eval_state<EOS, DIM>(WL, q, sL);
  eval_state<EOS, DIM>(WR, q, sR);
  double FL[NV], FR[NV];
  flux_dir<EOS, DIM>(WL, sL, d, FL);
  flux_dir<EOS, DIM>(WR, sR, d, FR);
  // the speeds as fractions n / den (den > 0), compared and combined without dividing:
  // lambda_L = nA / dA = min of the lambda_-, lambda_R = nB / dB = max of the lambda_+
  double nmL, npL, dnL, nmR, npR, dnR;
  wavespeeds_nd<EOS, DIM>(WL, sL, d, q, nmL, npL, dnL);
  wavespeeds_nd<EOS, DIM>(WR, sR, d, q, nmR, npR, dnR);
  const bool lminL = nmL * dnR <= nmR * dnL;
  const double nA = lminL ? nmL : nmR, dA = lminL ? dnL : dnR;
  const bool lmaxL = npL * dnR >= npR * dnL;
  const double nB = lmaxL ? npL : npR, dB = lmaxL ? dnL : dnR;
  if (nA >= 0.0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) Fh[k] = FL[k];
  } else if (nB <= 0.0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) Fh[k] = FR[k];
  } else {
    // (l_R F_L - l_L F_R + l_L l_R (U_R - U_L)) / (l_R - l_L), numerator and
    // denominator multiplied by dA dB
    const double cL = nB * dA, cR = nA * dB, cU = nA * nB;
    const double inv = 1.0 / (cL - cR);
#pragma unroll
    for (int k = 0; k < NV; ++k) Fh[k] = (cL * FL[k] - cR * FR[k] + cU * (sR.U[k] - sL.U[k])) * inv;
  }
}

// HLLC numerical flux along d (the paper's second solver, Sec. 2.4, after Mignone &
// Bodo 2005): the HLL speeds lambda_L, lambda_R bound a fan with one contact of speed
// lambda* and pressure p*.  With the HLL state and flux of D, S_d and tau
// (E = tau + D c^2, F_E = F_tau + c^2 F_D), lambda* is the root inside the fan of
//   F^hll_E lambda*^2 - c^2 (E^hll + F^hll_Sd) lambda* + c^4 S^hll_d = 0,
// taken as 2 c^2 S^hll_d / (b + sqrt(b^2 - 4 F^hll_E S^hll_d)), b = E^hll + F^hll_Sd, and
// p* = F^hll_Sd - lambda* F^hll_E / c^2.  The star state on side K is
// U*_K = (lambda_K U_K - F_K + p* (0, e_d, lambda*)) / (lambda_K - lambda*) and the flux
// F_K + lambda_K (U*_K - U_K): F_L, F*_L, F*_R or F_R by the signs of lambda_L,
// lambda*, lambda_R.
//
// Evaluated with two divisions: the outer speeds stay fractions n / den (den > 0) as in
// hll_flux, scaled by a power of two to den ~ 1; the HLL state and flux are kept
// multiplied by Delta = (lambda_R - lambda_L) den_L den_R > 0, which leaves lambda*
// unchanged (the quadratic is homogeneous in them) and scales p* by Delta; and with
// lambda_K = n / den,
//   F*_K = F_K + n (lambda* U_K - F_K + p* (0, e_d, lambda*)) / (n - lambda* den).
template <int EOS, int DIM>
__host__ __device__ __forceinline__ void hllc_flux(const double* WL, const double* WR, int d, const PhysParams& q,
                                          double* Fh) {
  constexpr int NV = DIM + 2;
  StateEval<EOS, DIM> sL, sR;
  eval_state<EOS, DIM>(WL, q, sL);
  eval_state<EOS, DIM>(WR, q, sR);
  double FL[NV], FR[NV];
  flux_dir<EOS, DIM>(WL, sL, d, FL);
  flux_dir<EOS, DIM>(WR, sR, d, FR);
  double nmL, npL, dnL, nmR, npR, dnR;
  wavespeeds_nd<EOS, DIM>(WL, sL, d, q, nmL, npL, dnL);
  wavespeeds_nd<EOS, DIM>(WR, sR, d, q, nmR, npR, dnR);
  // lambda_L = nA / dA (the lesser lambda_-), lambda_R = nB / dB (the greater lambda_+)
  const bool lminL = nmL * dnR <= nmR * dnL;
  double nA = lminL ? nmL : nmR, dA = lminL ? dnL : dnR;
  const bool lmaxL = npL * dnR >= npR * dnL;
  double nB = lmaxL ? npL : npR, dB = lmaxL ? dnL : dnR;
  if (nA >= 0.0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) Fh[k] = FL[k];
    return;
  }
  // the four scaled by one power of two to denominators near 1 (exact: the speeds and
  // every result below are unchanged), so that the products below stay near the size of
  // the states instead of growing with c^4 gamma^4 (Taub-Matthews, SI units)
  int ex;
  (void)frexp(fmax(dA, dB), &ex);
  nA = ldexp(nA, -ex);
  dA = ldexp(dA, -ex);
  nB = ldexp(nB, -ex);
  dB = ldexp(dB, -ex);
  // Delta times the HLL state and flux of the rows the contact needs (D, S_d, tau)
  const double cA = nA * dB, cB = nB * dA, cAB = dA * dB, cU = nA * nB;
  const double Dl = cB - cA;
  const double ULs = comp<DIM>(sL.U + 1, d), URs = comp<DIM>(sR.U + 1, d);
  const double FLs = comp<DIM>(FL + 1, d), FRs = comp<DIM>(FR + 1, d);
  const double UhD = cB * sR.U[0] - cA * sL.U[0] + cAB * (FL[0] - FR[0]);
  const double UhS = cB * URs - cA * ULs + cAB * (FLs - FRs);
  const double UhT = cB * sR.U[NV - 1] - cA * sL.U[NV - 1] + cAB * (FL[NV - 1] - FR[NV - 1]);
  const double FhD = cB * FL[0] - cA * FR[0] + cU * (sR.U[0] - sL.U[0]);
  const double FhS = cB * FLs - cA * FRs + cU * (URs - ULs);
  const double FhT = cB * FL[NV - 1] - cA * FR[NV - 1] + cU * (sR.U[NV - 1] - sL.U[NV - 1]);
  const double Eh = UhT + q.c2 * UhD, FEh = FhT + q.c2 * FhD;
  const double b = Eh + FhS;
  const double disc = fmax(b * b - 4.0 * FEh * UhS, 0.0);
  const double lam = 2.0 * q.c2 * UhS / (b + sqrt(disc));
  const double ps = FhS - lam * FEh * q.inv_c2;  // Delta p*
  const bool left = lam >= 0.0;
  if (!left && !(nB > 0.0)) {
#pragma unroll
    for (int k = 0; k < NV; ++k) Fh[k] = FR[k];
    return;
  }
  const double n = left ? nA : nB, dn = left ? dA : dB;
  const double r = n / (Dl * (n - lam * dn));
  const double nr = r * Dl;  // n / (n - lambda* den)
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const double U = left ? sL.U[k] : sR.U[k];
    const double F = left ? FL[k] : FR[k];
    double extra = 0.0;
    if (k == NV - 1) extra = ps * lam;
#pragma unroll
    for (int j = 0; j < DIM; ++j)
      if (k == 1 + j && j == d) extra = ps;
    Fh[k] = F + nr * (lam * U - F) + r * extra;
  }
}

// --------------------------------------------------- admissibility (Sec. 2.5)
// q(U) = E/c^2 - sqrt(D^2 + |S|^2/c^2) in tau form: tau/c^2 - (|S|^2/c^2)/(D + sqrt(D^2 + |S|^2/c^2)).
// With D > 0 the denominator is positive, so q > 0 is tested as
// (tau/c^2) (D + sqrt(D^2 + s2)) > s2, s2 = |S|^2/c^2, without the division.
__host__ __device__ __forceinline__ bool admissible_ts(double D, double tau, double s2, const PhysParams& q) {
  return (D > 0.0) && (tau * q.inv_c2 * (D + sqrt_pos(D * D + s2)) > s2);
}

template <int DIM>
__host__ __device__ __forceinline__ bool admissible(const double* U, const PhysParams& q) {
  double s2 = 0.0;
#pragma unroll
  for (int j = 0; j < DIM; ++j) s2 += U[1 + j] * U[1 + j];
  return admissible_ts(U[0], U[DIM + 1], s2 * q.inv_c2, q);
}

// ------------------------------------------------ recovery (Sec. 3)
__host__ __device__ __forceinline__ double cube_root(double x) { return cbrt(x); }

// cos(acos(x) / 3) for x in [-1, 1], i.e. the largest root t of 4 t^3 - 3 t = x
// (the trigonometric form of a cubic's largest real root).  For x > -0.9 a
// degree-4 least-squares fit of that function (error <= 3.3e-3) refined by three
// Newton steps on 4 t^3 - 3 t = x, whose derivative stays above 1.6 there (within
// 3 ulp of the exact value); near x = -1, where the root becomes double, the
// library acos and cos.
__host__ __device__ __forceinline__ double cos_third_acos(double x) {
  if (x > -0.9) {
    double t = (((-0.0366375023370486 * x + 0.051729089070298197) * x - 0.041218899401455941) * x +
                0.15925314888101053) * x + 0.86575468322880189;
#pragma unroll
    for (int it = 0; it < 3; ++it) {
      const double t2 = t * t;
      t -= (t * (4.0 * t2 - 3.0) - x) / (12.0 * t2 - 3.0);
    }
    return t;
  }
  return cos(acos(x) * (1.0 / 3.0));
}

// TM cubic of Eq. (synge_cubic): W^3 + c1 W^2 + c2 W + c3 = 0, W = gamma^2 - 1.
__host__ __device__ __forceinline__ void tm_cubic_coeffs(double xi, double eta, double& c1, double& c2, double& c3) {
  const double x2 = xi * xi, e2 = eta * eta;
  const double dm = (eta - xi) * (eta + xi);
  const double i16 = 1.0 / (16.0 * dm * dm);
  const double k = 4.0 * (e2 + x2) - (x2 + 1.0);
  c1 = 8.0 * ((e2 + x2) * k - 14.0 * x2 * e2) * i16;
  c2 = (k * k - 57.0 * x2 * e2) * i16;
  c3 = -9.0 * x2 * e2 * i16;
}

// The same cubic multiplied through by 16 D^4 (eta^2 - xi^2)^2 and written in
// X = D xi = |S| / c, Y = D eta = E / c^2 and D: A W^3 + C1 W^2 + C2 W + C3 with
// A = 16 (Y^2 - X^2)^2 (no division).  Every coefficient is homogeneous of degree 8
// in (X, Y, D), so the three may be scaled by one power of two first.
__host__ __device__ __forceinline__ void tm_cubic_scaled(double X, double Y, double D, double& A, double& C1,
                                                         double& C2, double& C3) {
  const double x2 = X * X, e2 = Y * Y;
  const double dm = (Y - X) * (Y + X);
  A = 16.0 * dm * dm;
  const double k = 4.0 * (e2 + x2) - (x2 + D * D);
  C1 = 8.0 * ((e2 + x2) * k - 14.0 * x2 * e2);
  C2 = k * k - 57.0 * x2 * e2;
  C3 = -9.0 * x2 * e2;
}

// A start for Newton on the TM cubic A W^3 + C1 W^2 + C2 W + C3 (tm_cubic_scaled): its
// largest root by the closed form of the monic cubic evaluated in FP32 (relative error
// ~1e-6 away from a double root; three FP64 Newton steps then reach rounding level, and
// the caller accepts the result only when the last step is that small).
// FP32 pieces of that start on the device: the hardware reciprocal, square root, log2
// and exp2 (about one ulp each; the FP64 Newton steps absorb it), the cube root as
// exp2(log2|y| / 3) with the sign of y.
#if defined(__HIP_DEVICE_COMPILE__)
__device__ __forceinline__ float start_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float start_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float start_cbrt(float y) {
  return copysignf(__builtin_amdgcn_exp2f(__builtin_amdgcn_logf(fabsf(y)) * (1.0f / 3.0f)), y);
}
#else
__host__ __forceinline__ float start_rcp(float x) { return 1.0f / x; }
__host__ __forceinline__ float start_sqrt(float x) { return sqrtf(x); }
__host__ __forceinline__ float start_cbrt(float y) { return cbrtf(y); }
#endif

__host__ __device__ __forceinline__ double tm_cubic_start_f32(double A, double C1, double C2, double C3) {
  const float ia = start_rcp((float)A);
  const float c1 = (float)C1 * ia, c2 = (float)C2 * ia, c3 = (float)C3 * ia;
  const float Q = (3.0f * c2 - c1 * c1) * (1.0f / 9.0f);
  const float R = (9.0f * c1 * c2 - 27.0f * c3 - 2.0f * c1 * c1 * c1) * (1.0f / 54.0f);
  const float dd = Q * Q * Q + R * R;
  float W;
  if (dd < 0.0f) {
    const float sq = start_sqrt(-Q);
    const float x = fminf(1.0f, fmaxf(-1.0f, R * start_rcp(-Q * sq)));
    float t;
    if (x > -0.9f) {
      // cos(acos(x) / 3): the fit of cos_third_acos and two Newton steps on 4 t^3 - 3 t = x
      t = (((-0.0366375f * x + 0.0517291f) * x - 0.0412189f) * x + 0.159253f) * x + 0.865755f;
#pragma unroll
      for (int it = 0; it < 2; ++it) {
        const float t2 = t * t;
        t -= (t * (4.0f * t2 - 3.0f) - x) * start_rcp(12.0f * t2 - 3.0f);
      }
    } else {
      t = cosf(acosf(x) * (1.0f / 3.0f));
    }
    W = 2.0f * sq * t - c1 * (1.0f / 3.0f);
  } else {
    const float sd = start_sqrt(dd);
    W = -c1 * (1.0f / 3.0f) + start_cbrt(R + sd) + start_cbrt(R - sd);
  }
  return (double)W;
}

// Brent's bracketed root finder (R. P. Brent, Algorithms for Minimization without
// Derivatives, 1973: inverse quadratic interpolation / secant with a bisection
// safeguard) on the TM cubic over [lo, hi]; returns false at the cap of maxit steps.
__host__ __device__ __forceinline__ bool tm_brent_root(double c1, double c2, double c3, double lo, double hi, double& root,
                                                      int maxit = 100) {
  auto f = [&](double W) { return ((W + c1) * W + c2) * W + c3; };
  double a = lo, b = hi, fa = f(a), fb = f(b);
  double c = a, fc = fa, d = b - a, e = d;
  const double eps = 2.220446049250313e-16;
  for (int it = 0; it < maxit; ++it) {
    if ((fb > 0.0) == (fc > 0.0)) {
      c = a; fc = fa; d = b - a; e = d;
    }
    if (fabs(fc) < fabs(fb)) {
      a = b; b = c; c = a; fa = fb; fb = fc; fc = fa;
    }
    const double tol1 = 2.0 * eps * fabs(b);
    const double xm = 0.5 * (c - b);
    if (fabs(xm) <= tol1 || fb == 0.0) {
      root = b;
      return true;
    }
    if (fabs(e) >= tol1 && fabs(fa) > fabs(fb)) {
      double p, qq;
      const double s = fb / fa;
      if (a == c) {
        p = 2.0 * xm * s;
        qq = 1.0 - s;
      } else {
        const double t = fa / fc, r = fb / fc;
        p = s * (2.0 * xm * t * (t - r) - (b - a) * (r - 1.0));
        qq = (t - 1.0) * (r - 1.0) * (s - 1.0);
      }
      if (p > 0.0) qq = -qq;
      p = fabs(p);
      if (2.0 * p < fmin(3.0 * xm * qq - fabs(tol1 * qq), fabs(e * qq))) {
        e = d;
        d = p / qq;
      } else {
        d = xm; e = d;
      }
    } else {
      d = xm; e = d;
    }
    a = b; fa = fb;
    b += (fabs(d) > tol1) ? d : (xm > 0.0 ? tol1 : -tol1);
    fb = f(b);
  }
  root = b;
  return false;
}

// Conserved -> primitive at one node with the configured solver.  Returns a C2P_*
// status; on failure writes the floor state.  Also returns the pieces the
// implicit-function-theorem adjoint needs through the primitive output only.
// Wprev, when given, is the node's primitive state of the previous SSP-RK stage: with
// the TM EOS and C2P_NEWTON it starts three Newton steps on the cubic (without Wprev the
// closed-form root evaluated in FP32 starts them), accepted when the last step is below
// 1e-9 W and the iterate lies on the branch of the largest root (f' > 0 beyond the
// inflection point); otherwise the analytic root with one Newton polish.  Both give
// the same root to rounding.  With
// the ideal EOS and C2P_NEWTON it is the start of the Newton iteration on the quartic
// (any start in (0, 1) converges to its one root there; the stop rule is unchanged).
// known_admissible: the caller has evaluated admissible<DIM>(U) (the same expression)
// and it held, so the test is skipped.
template <int EOS, int DIM>
__host__ __device__ __forceinline__ int con2prim(const double* U, double* W, const PhysParams& q,
                                                 const double* Wprev = nullptr, bool known_admissible = false) {
  constexpr int NV = DIM + 2;
  const double D = U[0];
  const double tau = U[NV - 1];
  double s2 = 0.0;
#pragma unroll
  for (int j = 0; j < DIM; ++j) s2 += U[1 + j] * U[1 + j];
  const bool ok = known_admissible || admissible_ts(D, tau, s2 * q.inv_c2, q);
  int status = C2P_OK;
  double rho = kRhoFloor, P = kPFloor * q.c2, gb = 0.0, Smag = 0.0;
  double iS = 0.0;  // 1 / |S| (0 at rest)
  if (!ok) {
    status = C2P_INADMISSIBLE;
  } else {
    iS = s2 > 0.0 ? inv_sqrt(s2) : 0.0;
    Smag = s2 * iS;
    int method = q.c2p;
    if constexpr (EOS == EOS_IDEAL) {
      const double iD = 1.0 / D;
      const double xi = Smag * iD * q.inv_c;
      const double t = tau * iD * q.inv_c2;  // eta - 1
      const double eta = 1.0 + t;
      const double al = q.alpha;
      double w = 0.0;
      if (method == C2P_QUARTIC) {
        // analytic quartic in beta through its resolvent cubic (readings: leading
        // beta^4 with a3 on beta^3; R with 9 i1 i2; trigonometric branch via atan2)
        const double G = q.gam, g1 = q.gm1;
        const double den = g1 * g1 * (xi * xi + 1.0);
        const double a3 = -2.0 * G * g1 * xi * eta / den;
        const double a2 = (G * G * eta * eta + 2.0 * g1 * xi * xi - g1 * g1) / den;
        const double a1 = -2.0 * G * xi * eta / den;
        const double a0 = xi * xi / den;
        const double i1 = -a2, i2 = a3 * a1 - 4.0 * a0, i3 = 4.0 * a2 * a0 - a1 * a1 - a3 * a3 * a0;
        const double R = (9.0 * i1 * i2 - 27.0 * i3 - 2.0 * i1 * i1 * i1) / 54.0;
        const double Sq = (3.0 * i2 - i1 * i1) / 9.0;
        const double T = R * R + Sq * Sq * Sq;
        double x;
        if (T < 0.0) {
          x = 2.0 * sqrt(-Sq) * cos(atan2(sqrt(-T), R) / 3.0) - i1 / 3.0;
        } else {
          const double sT = sqrt(T);
          x = cube_root(R + sT) + cube_root(R - sT) - i1 / 3.0;
        }
        const double Bq = 0.5 * (a3 + sqrt(a3 * a3 - 4.0 * a2 + 4.0 * x));
        const double Cq = 0.5 * (x - sqrt(x * x - 4.0 * a0));
        double beta = 0.5 * (-Bq + sqrt(Bq * Bq - 4.0 * Cq));
        if (!(xi > 0.0)) beta = 0.0;
        if (!isfinite(beta)) {
          status = C2P_NOCONV;
        } else {
          const double sq = sqrt((1.0 - beta) * (1.0 + beta));
          rho = D * sq;
          gb = beta / sq;
          P = q.gm1 * (tau - Smag * beta * q.c + D * q.c2 * beta * beta / (1.0 + sq));
        }
      } else {
        // Newton-Raphson on the quartic P(w) of Eq. (iterative_quartic)
        const double A = (al - 1.0) * xi;
        const double B = 2.0 * (al * t + al + 1.0);   // 2 (alpha eta + 1)
        const double C = 2.0 * (al + 1.0) * xi;
        const double Dd = 2.0 * (al * t + al - 1.0);  // 2 (alpha eta - 1)
        if (xi < 1e-4) {
          // small-xi series, Eq. (iterative_cubic_approximation)
          const double ame = 0.5 * Dd, ape = 0.5 * B;
          const double k1 = (al - 1.0) / (2.0 * ame);
          const double k3 = (al - 1.0) * (al - 1.0) / (8.0 * ame * ame * ame * ame) *
                            ((al + 3.0) * ape - 4.0 * (al + 1.0));
          w = k1 * xi + k3 * xi * xi * xi;
        } else {
          w = 0.0;
          if (Wprev != nullptr) {
            // start from the previous stage's root: w = |u| / (c (gamma + 1))
            double u2 = 0.0;
#pragma unroll
            for (int j = 0; j < DIM; ++j) u2 += Wprev[1 + j] * Wprev[1 + j];
            w = sqrt_pos(u2) * q.inv_c / (sqrt_pos(1.0 + u2 * q.inv_c2) + 1.0);
          }
          if (!(w > 0.0 && w < 1.0)) {
            const double b = xi / eta;
            w = b / (1.0 + sqrt(1.0 - b * b));
          }
          const bool fixed = q.c2p_iters > 0;
          // the recovery study's fixed-iteration solver starts from the middle of (0, 1)
          if (fixed) w = 0.5;
          const int cap = fixed ? q.c2p_iters : 30;
          bool conv = fixed;
          for (int it = 0; it < cap; ++it) {
            const double Pw = (((A * w - B) * w + C) * w - Dd) * w + A;
            const double dPw = ((4.0 * A * w - 3.0 * B) * w + 2.0 * C) * w - Dd;
            double wn = w - Pw / dPw;
            if (wn <= 0.0) wn = 0.5 * w;
            else if (wn >= 1.0) wn = 0.5 * (w + 1.0);
            const double step = fabs(wn - w);
            w = wn;
            if (!fixed && step <= 1e-13 * wn) { conv = true; break; }
          }
          if (!conv) status = C2P_NOCONV;
        }
        const double w2 = w * w;
        const double om = (1.0 - w) * (1.0 + w);
        const double r1 = 1.0 / (1.0 + w2);
        const double beta = 2.0 * w * r1;
        rho = D * om * r1;
        gb = 2.0 * w / om;
        P = q.gm1 * (tau - Smag * beta * q.c + D * q.c2 * 2.0 * w2 * r1);
      }
    } else {
      double Wc;
      bool done = false;
      if (method == C2P_NEWTON) {
        // Newton on the cubic scaled by 16 D^4 (eta^2 - xi^2)^2 (the same iterates as on
        // the monic one, without a division for the coefficients), its coefficients from
        // (X, Y, D) / 2^e with 2^e the binade of D; started from the previous stage's
        // root inside a stage, else from the closed-form root in FP32
        int e;
        (void)frexp(D, &e);
        double A, C1, C2, C3;
        tm_cubic_scaled(ldexp(Smag * q.inv_c, -e), ldexp(tau * q.inv_c2 + D, -e), ldexp(D, -e), A, C1, C2, C3);
        double Wn;
        if (Wprev != nullptr) {
          double u2 = 0.0;
#pragma unroll
          for (int j = 0; j < DIM; ++j) u2 += Wprev[1 + j] * Wprev[1 + j];
          Wn = u2 * q.inv_c2;  // gamma^2 - 1 of the previous stage
        } else {
          Wn = tm_cubic_start_f32(A, C1, C2, C3);
        }
        // (the first two steps with a refined reciprocal of f', the last with the quotient)
        double step = 0.0;
#pragma unroll
        for (int it = 0; it < 3; ++it) {
          const double f = ((A * Wn + C1) * Wn + C2) * Wn + C3;
          const double fp = (3.0 * A * Wn + 2.0 * C1) * Wn + C2;
          step = it < 2 ? f * rcp_refined(fp) : f / fp;
          Wn -= step;
        }
        const double fp = (3.0 * A * Wn + 2.0 * C1) * Wn + C2;
        if (fabs(step) <= 1e-9 * fabs(Wn) && A > 0.0 && fp > 0.0 && 3.0 * A * Wn + C1 > 0.0) {
          Wc = Wn;
          done = true;
        }
      }
      if (!done) {
        const double iD = 1.0 / D;
        const double xi = Smag * iD * q.inv_c;
        const double eta = 1.0 + tau * iD * q.inv_c2;
        double c1, c2, c3;
        tm_cubic_coeffs(xi, eta, c1, c2, c3);
        if (method == C2P_BRENT) {
          if (c3 == 0.0) {
            Wc = 0.0;
          } else {
            double hi = 200.0 * 200.0 - 1.0;
            for (int k = 0; k < 60 && (((hi + c1) * hi + c2) * hi + c3) < 0.0; ++k) hi *= 4.0;
            if (!tm_brent_root(c1, c2, c3, 0.0, hi, Wc, q.c2p_iters > 0 ? q.c2p_iters : 100) && q.c2p_iters == 0)
              status = C2P_NOCONV;
          }
        } else {
          // analytic (trigonometric / Cardano), then one Newton step on the cubic
          const double Q = (3.0 * c2 - c1 * c1) * (1.0 / 9.0);
          const double R = (9.0 * c1 * c2 - 27.0 * c3 - 2.0 * c1 * c1 * c1) * (1.0 / 54.0);
          const double dd = Q * Q * Q + R * R;
          if (dd < 0.0) {
            double arg = R * inv_sqrt(-Q * Q * Q);
            arg = fmin(1.0, fmax(-1.0, arg));
            Wc = 2.0 * sqrt(-Q) * cos_third_acos(arg) - c1 * (1.0 / 3.0);
          } else {
            const double sd = sqrt(dd);
            Wc = -c1 * (1.0 / 3.0) + cube_root(R + sd) + cube_root(R - sd);
          }
          const double f = ((Wc + c1) * Wc + c2) * Wc + c3;
          const double fp = (3.0 * Wc + 2.0 * c1) * Wc + c2;
          Wc = Wc - f / fp;
        }
      }
      Wc = fmax(Wc, 0.0);
      const double g2 = 1.0 + Wc;
      const double ig = inv_sqrt(g2);  // 1 / gamma
      const double gam = g2 * ig;
      gb = sqrt_pos(Wc);  // gamma beta
      const double beta = gb * ig;
      rho = D * ig;
      // P = (X^2 - (rho c^2)^2)/(3X), X = E - M.v, via X_ = X - rho c^2 =
      // tau - |S| beta c + D c^2 (gamma^2 - 1) / (gamma (gamma + 1)), carried as
      // N = X_ (gamma + 1) so that one division remains:
      // P = N (N + 2 rho c^2 (gamma + 1)) / (3 (gamma + 1) (N + rho c^2 (gamma + 1)))
      const double gp1 = gam + 1.0;
      const double N = (tau - Smag * beta * q.c) * gp1 + D * q.c2 * Wc * ig;
      const double rc2g = rho * q.c2 * gp1;
      P = N * (N + 2.0 * rc2g) / (3.0 * gp1 * (N + rc2g));
    }
    if (!(P > 0.0) || !isfinite(P) || !isfinite(rho)) {
      if (status == C2P_OK) status = C2P_BADP;
    }
  }
  // the floor state at rest, exactly (also when the momentum itself is not finite)
  const bool floor = (status != C2P_OK && status != C2P_NOCONV) ||
                     (status == C2P_NOCONV && (!(P > 0.0) || !isfinite(P) || !isfinite(rho) || !isfinite(gb)));
  if (floor) {
    rho = kRhoFloor;
    P = kPFloor * q.c2;
  }
  W[0] = rho;
  const double scale = gb * q.c * iS;
#pragma unroll
  for (int j = 0; j < DIM; ++j) W[1 + j] = floor ? 0.0 : scale * U[1 + j];
  W[NV - 1] = P;
  return status;
}

}  // namespace dgsrhd
