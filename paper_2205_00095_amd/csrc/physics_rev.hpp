// Reverse-mode (vector-Jacobian) counterparts of the device physics in
// physics.hpp, written by hand statement by statement against the forward
// code, plus the implicit-function-theorem adjoint of the recovery.
//
// Convention: every *_rev function takes the forward inputs, recomputes what it
// needs, and ADDS the input adjoints into the lam_* arguments.
#pragma once
#include "physics.hpp"

namespace dgsrhd {

// d(h - c^2)/dTheta
template <int EOS>
__host__ __device__ __forceinline__ double h_excess_d(double th, const PhysParams& q, double sq = -1.0) {
  if constexpr (EOS == EOS_IDEAL) {
    return q.alpha;
  } else {
    const double s = sq >= 0.0 ? sq : sqrt(th * th + (4.0 / 9.0) * q.c4);
    const double den = s + (2.0 / 3.0) * q.c2;
    // 5/2 Theta + 3/2 Theta^2 / den,   d den / dTheta = Theta / s
    return 2.5 + 1.5 * (2.0 * th * den - th * th * th / s) / (den * den);
  }
}

// Adjoint of eval_state: given adjoints of (U[0..NV), g2, ig, th, he) and of P
// (returned through lam_W[NV-1]), accumulate into lam_W.  st is the forward
// evaluation at W (its square roots and quotients are reused).
template <int EOS, int DIM>
__host__ __device__ __forceinline__ void eval_state_rev(const double* W, const StateEval<EOS, DIM>& st,
                                                        const PhysParams& q, const double* lam_U, double lam_g2,
                                                        double lam_ig, double lam_th, double lam_he, double* lam_W) {
  constexpr int NV = DIM + 2;
  const double rho = W[0];
  double usq = 0.0;
#pragma unroll
  for (int j = 0; j < DIM; ++j) usq += W[1 + j] * W[1 + j];
  const double g2 = st.g2;
  const double ig = st.ig;
  const double g = g2 * ig;
  const double th = st.th;
  const double he = st.he;
  const double D = st.U[0];
  const double hc = (q.c2 + he) * q.inv_c2;
  const double gH = g * rho * hc;
  const double igp1 = rho * st.r;  // 1 / (g + 1)
  // ig = 1/g
  double lam_g = -lam_ig * ig * ig;
  // tau = D usq/(g+1) + g2 rho he - P
  const double lt = lam_U[NV - 1];
  double lam_D = lam_U[0] + lt * usq * igp1;
  double lam_usq = lt * D * igp1;
  lam_g += -lt * D * usq * igp1 * igp1;
  lam_g2 += lt * rho * he;
  double lam_rho = lt * g2 * he;
  lam_he += lt * g2 * rho;
  double lam_P = -lt;
  // S_j = gH u_j
  double lam_gH = 0.0;
#pragma unroll
  for (int j = 0; j < DIM; ++j) {
    lam_gH += lam_U[1 + j] * W[1 + j];
    lam_W[1 + j] += lam_U[1 + j] * gH;
  }
  // gH = g rho (c^2 + he)/c^2
  lam_g += lam_gH * rho * hc;
  lam_rho += lam_gH * g * hc;
  lam_he += lam_gH * g * rho * q.inv_c2;
  // D = g rho
  lam_g += lam_D * rho;
  lam_rho += lam_D * g;
  // he = h_excess(th); Taub-Matthews: he = 5/2 th + 3/2 (sq - 2/3 c^2), d sq / d th = th / sq
  if constexpr (EOS == EOS_IDEAL) lam_th += lam_he * q.alpha;
  else lam_th += lam_he * (2.5 + 1.5 * th * st.isq);
  // th = P / rho
  const double irho = (g + 1.0) * st.r;  // 1 / rho
  lam_P += lam_th * irho;
  lam_rho += -lam_th * th * irho;
  // g = sqrt(g2)
  lam_g2 += lam_g * 0.5 * ig;
  // g2 = 1 + usq/c^2
  lam_usq += lam_g2 * q.inv_c2;
#pragma unroll
  for (int j = 0; j < DIM; ++j) lam_W[1 + j] += 2.0 * W[1 + j] * lam_usq;
  lam_W[0] += lam_rho;
  lam_W[NV - 1] += lam_P;
}

template <int EOS, int DIM>
__host__ __device__ __forceinline__ void eval_state_rev(const double* W, const PhysParams& q, const double* lam_U,
                                                        double lam_g2, double lam_ig, double lam_th, double lam_he,
                                                        double* lam_W) {
  StateEval<EOS, DIM> st;
  eval_state<EOS, DIM>(W, q, st);
  eval_state_rev<EOS, DIM>(W, st, q, lam_U, lam_g2, lam_ig, lam_th, lam_he, lam_W);
}

// The signal speeds of wavespeeds() with the intermediates their adjoint reuses:
// lambda_pm = (vd gK pm root) inv, gK = gamma^2 K, root = sqrt(N X),
// X = gK (c^2 - vd^2) + c^2 N, inv = 1 / (gK + N) (N, K as in wavespeeds_nd).
struct SpeedParts {
  double vd, N, K, gK, X, rr, root, inv, lm, lp;  // rr = 1 / root (0 when root = 0)
};

// Its inputs pass through opaque() so that the compiler recomputes these values where
// the adjoint needs them instead of keeping the forward's copies live in between.
template <int EOS, int DIM>
__host__ __device__ __forceinline__ void speed_parts(const double* W, const StateEval<EOS, DIM>& s, int d,
                                                     const PhysParams& q, SpeedParts& p) {
  const double th = opaque(s.th), g2 = opaque(s.g2);
  if constexpr (EOS == EOS_IDEAL) {
    p.N = q.gam * th;
    p.K = q.c2 + (q.alpha - q.gam) * th;
  } else {
    const double sq = opaque(s.sq);
    p.N = th * (3.0 * th + 5.0 * sq);
    p.K = th * (9.0 * th + 7.0 * sq) + 2.0 * q.c4;
  }
  p.vd = comp<DIM>(W + 1, d) * opaque(s.ig);
  p.gK = g2 * p.K;
  p.X = p.gK * (q.c2 - p.vd * p.vd) + q.c2 * p.N;
  const double nx = p.N * p.X;
  p.rr = nx > 0.0 ? inv_sqrt(nx) : 0.0;
  p.root = nx * p.rr;
  p.inv = 1.0 / (p.gK + p.N);
  p.lm = (p.vd * p.gK - p.root) * p.inv;
  p.lp = (p.vd * p.gK + p.root) * p.inv;
}

// Adjoint of (U, F^d, lambda_-, lambda_+) of one primitive state along d.
// lam_U, lam_F: adjoints of the conserved state and of the flux; lam_lm, lam_lp:
// adjoints of the two signal speeds (pass 0 when unused).
template <int EOS, int DIM>
__host__ __device__ __forceinline__ void state_flux_speed_rev(const double* W, const StateEval<EOS, DIM>& s,
                                                              const SpeedParts& sp, int d, const PhysParams& q,
                                                              const double* lam_U_in, const double* lam_F,
                                                              double lam_lm, double lam_lp, bool with_speeds,
                                                              double* lam_W) {
  constexpr int NV = DIM + 2;
  const double vd = sp.vd;
  double lam_U[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) lam_U[k] = lam_U_in[k];
  // flux: F_k = U_k vd ; F_{1+d} += P ; F_tau += P vd
  double lam_vd = 0.0;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    lam_U[k] += lam_F[k] * vd;
    lam_vd += lam_F[k] * s.U[k];
  }
  double lam_P = comp<DIM>(lam_F + 1, d) + lam_F[NV - 1] * vd;
  lam_vd += lam_F[NV - 1] * s.P;
  double lam_g2 = 0.0, lam_th = 0.0;
  if (with_speeds) {
    // lambda_pm = (vd gK pm root) inv
    const double lam_den = -(lam_lm * sp.lm + lam_lp * sp.lp) * sp.inv;  // inv = 1 / (gK + N)
    const double lam_vdgK = (lam_lm + lam_lp) * sp.inv;
    const double lam_root = (lam_lp - lam_lm) * sp.inv;
    lam_vd += lam_vdgK * sp.gK;
    double lam_gK = lam_vdgK * vd + lam_den;
    double lam_N = lam_den;
    if (sp.root > 0.0) {
      // root = sqrt(N X), X = gK (c^2 - vd^2) + c^2 N
      const double lam_NX = 0.5 * lam_root * sp.rr;
      lam_N += lam_NX * sp.X;
      const double lam_X = lam_NX * sp.N;
      lam_gK += lam_X * (q.c2 - vd * vd);
      lam_vd += -2.0 * vd * sp.gK * lam_X;
      lam_N += q.c2 * lam_X;
    }
    // gK = gamma^2 K
    lam_g2 += lam_gK * sp.K;
    const double lam_K = lam_gK * s.g2;
    // N, K as functions of Theta
    if constexpr (EOS == EOS_IDEAL) {
      lam_th += q.gam * lam_N + (q.alpha - q.gam) * lam_K;
    } else {
      const double th = s.th, ds = th * s.isq;  // d sq / d Theta
      lam_th += lam_N * (6.0 * th + 5.0 * s.sq + 5.0 * th * ds) + lam_K * (18.0 * th + 7.0 * s.sq + 7.0 * th * ds);
    }
  }
  // vd = u_d * ig
  comp_add<DIM>(lam_W + 1, d, lam_vd * s.ig);
  const double lam_ig = lam_vd * comp<DIM>(W + 1, d);
  lam_W[NV - 1] += lam_P;
  eval_state_rev<EOS, DIM>(W, s, q, lam_U, lam_g2, lam_ig, lam_th, 0.0, lam_W);
}

template <int EOS, int DIM>
__host__ __device__ __forceinline__ void state_flux_speed_rev(const double* W, int d, const PhysParams& q,
                                                              const double* lam_U_in, const double* lam_F,
                                                              double lam_lm, double lam_lp, bool with_speeds,
                                                              double* lam_W) {
  StateEval<EOS, DIM> s;
  eval_state<EOS, DIM>(W, q, s);
  SpeedParts sp;
  speed_parts<EOS, DIM>(W, s, d, q, sp);
  state_flux_speed_rev<EOS, DIM>(W, s, sp, d, q, lam_U_in, lam_F, lam_lm, lam_lp, with_speeds, lam_W);
}

// Adjoint of hll_flux(WL, WR, d): accumulates into lam_WL and lam_WR (the branch
// chosen on the speeds as quotients, as the forward's fractions choose it except at
// exact ties).
template <int EOS, int DIM>
__host__ __device__ __forceinline__ void hll_flux_rev(const double* WL, const double* WR, int d, const PhysParams& q,
                                             const double* lam_Fh, double* lam_WL, double* lam_WR,
                                             bool need_L = true, bool need_R = true) {
  constexpr int NV = DIM + 2;
  StateEval<EOS, DIM> sL, sR;
  eval_state<EOS, DIM>(WL, q, sL);
  eval_state<EOS, DIM>(WR, q, sR);
  double FL[NV], FR[NV];
  flux_dir<EOS, DIM>(WL, sL, d, FL);
  flux_dir<EOS, DIM>(WR, sR, d, FR);
  double lmL, lpL, lmR, lpR;
  wavespeeds<EOS, DIM>(WL, sL, d, q, lmL, lpL);
  wavespeeds<EOS, DIM>(WR, sR, d, q, lmR, lpR);
  const double aL = fmin(lmL, lmR);
  const double aR = fmax(lpL, lpR);
  double lam_FL[NV], lam_FR[NV], lam_UL[NV], lam_UR[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) lam_FL[k] = lam_FR[k] = lam_UL[k] = lam_UR[k] = 0.0;
  double lam_lmL = 0.0, lam_lpL = 0.0, lam_lmR = 0.0, lam_lpR = 0.0;
  bool speeds = false;
  if (aL >= 0.0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) lam_FL[k] = lam_Fh[k];
  } else if (aR <= 0.0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) lam_FR[k] = lam_Fh[k];
  } else {
    speeds = true;
    const double inv = 1.0 / (aR - aL);
    double lam_aL = 0.0, lam_aR = 0.0;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      const double dU = sR.U[k] - sL.U[k];
      const double Fh = (aR * FL[k] - aL * FR[k] + aL * aR * dU) * inv;
      lam_FL[k] = lam_Fh[k] * aR * inv;
      lam_FR[k] = -lam_Fh[k] * aL * inv;
      lam_UR[k] = lam_Fh[k] * aL * aR * inv;
      lam_UL[k] = -lam_UR[k];
      lam_aR += lam_Fh[k] * (FL[k] + aL * dU - Fh) * inv;
      lam_aL += lam_Fh[k] * (-FR[k] + aR * dU + Fh) * inv;
    }
    if (lmL <= lmR) lam_lmL = lam_aL; else lam_lmR = lam_aL;
    if (lpL >= lpR) lam_lpL = lam_aR; else lam_lpR = lam_aR;
  }
  // the speed intermediates are recomputed per side rather than kept live from above
  if (need_L) {
    SpeedParts p;
    speed_parts<EOS, DIM>(WL, sL, d, q, p);
    state_flux_speed_rev<EOS, DIM>(WL, sL, p, d, q, lam_UL, lam_FL, lam_lmL, lam_lpL, speeds, lam_WL);
  }
  if (need_R) {
    SpeedParts p;
    speed_parts<EOS, DIM>(WR, sR, d, q, p);
    state_flux_speed_rev<EOS, DIM>(WR, sR, p, d, q, lam_UR, lam_FR, lam_lmR, lam_lpR, speeds, lam_WR);
  }
}

// Adjoint of hllc_flux(WL, WR, d): accumulates into lam_WL and lam_WR.  The forward
// branch is retaken (chosen here on the speeds as quotients; the forward compares the
// same speeds as fractions, which can choose otherwise only at exact ties, where the
// flux is continuous); in the star branch the reverse runs through the star state of
// the upwind side, the contact speed and pressure, the HLL state and flux rows they
// use, and the outer speeds.
template <int EOS, int DIM>
__host__ __device__ __forceinline__ void hllc_flux_rev(const double* WL, const double* WR, int d,
                                              const PhysParams& q, const double* lam_Fh, double* lam_WL,
                                              double* lam_WR, bool need_L = true, bool need_R = true) {
  constexpr int NV = DIM + 2;
  StateEval<EOS, DIM> sL, sR;
  eval_state<EOS, DIM>(WL, q, sL);
  eval_state<EOS, DIM>(WR, q, sR);
  double FL[NV], FR[NV];
  flux_dir<EOS, DIM>(WL, sL, d, FL);
  flux_dir<EOS, DIM>(WR, sR, d, FR);
  double lmL, lpL, lmR, lpR;
  wavespeeds<EOS, DIM>(WL, sL, d, q, lmL, lpL);
  wavespeeds<EOS, DIM>(WR, sR, d, q, lmR, lpR);
  const double aL = fmin(lmL, lmR), aR = fmax(lpL, lpR);
  double lam_FL[NV], lam_FR[NV], lam_UL[NV], lam_UR[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) lam_FL[k] = lam_FR[k] = lam_UL[k] = lam_UR[k] = 0.0;
  double lam_lmL = 0.0, lam_lpL = 0.0, lam_lmR = 0.0, lam_lpR = 0.0;
  bool speeds = false;
  if (aL >= 0.0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) lam_FL[k] = lam_Fh[k];
  } else {
    // forward: HLL rows, contact speed and pressure
    const double ih = 1.0 / (aR - aL);
    const double ULs = comp<DIM>(sL.U + 1, d), URs = comp<DIM>(sR.U + 1, d);
    const double FLs = comp<DIM>(FL + 1, d), FRs = comp<DIM>(FR + 1, d);
    const double UhD = (aR * sR.U[0] - aL * sL.U[0] + FL[0] - FR[0]) * ih;
    const double UhS = (aR * URs - aL * ULs + FLs - FRs) * ih;
    const double UhT = (aR * sR.U[NV - 1] - aL * sL.U[NV - 1] + FL[NV - 1] - FR[NV - 1]) * ih;
    const double FhD = (aR * FL[0] - aL * FR[0] + aL * aR * (sR.U[0] - sL.U[0])) * ih;
    const double FhS = (aR * FLs - aL * FRs + aL * aR * (URs - ULs)) * ih;
    const double FhT = (aR * FL[NV - 1] - aL * FR[NV - 1] + aL * aR * (sR.U[NV - 1] - sL.U[NV - 1])) * ih;
    const double Eh = UhT + q.c2 * UhD, FEh = FhT + q.c2 * FhD;
    const double b = Eh + FhS;
    const double disc0 = b * b - 4.0 * FEh * UhS;
    const double disc = fmax(disc0, 0.0);
    const double sd = sqrt(disc);
    const double den = b + sd;
    const double lam = 2.0 * q.c2 * UhS / den;
    const double ps = FhS - lam * FEh * q.inv_c2;
    const bool left = lam >= 0.0;
    if (!left && !(aR > 0.0)) {
#pragma unroll
      for (int k = 0; k < NV; ++k) lam_FR[k] = lam_Fh[k];
    } else {
      speeds = true;
      const double a = left ? aL : aR;
      const double ia = 1.0 / (a - lam);
      double lam_a = 0.0, lam_ia = 0.0, lam_ps = 0.0, lam_lam = 0.0;
      double lam_Us_side[NV], lam_Fs_side[NV];
#pragma unroll
      for (int k = 0; k < NV; ++k) {
        const double U = left ? sL.U[k] : sR.U[k];
        const double F = left ? FL[k] : FR[k];
        double extra = 0.0;
        if (k == NV - 1) extra = ps * lam;
#pragma unroll
        for (int j = 0; j < DIM; ++j)
          if (k == 1 + j && j == d) extra = ps;
        const double num = a * U - F + extra;
        const double Us = num * ia;
        // Fout = F + a (Us - U)
        const double lf = lam_Fh[k];
        double lF = lf, lU = -lf * a;
        lam_a += lf * (Us - U);
        const double lam_num = lf * a * ia;
        lam_ia += lf * a * num;
        lam_a += lam_num * U;
        lU += lam_num * a;
        lF -= lam_num;
        if (k == NV - 1) {
          lam_ps += lam_num * lam;
          lam_lam += lam_num * ps;
        }
#pragma unroll
        for (int j = 0; j < DIM; ++j)
          if (k == 1 + j && j == d) lam_ps += lam_num;
        lam_Us_side[k] = lU;
        lam_Fs_side[k] = lF;
      }
      // ia = 1 / (a - lam)
      const double lam_diff = -lam_ia * ia * ia;
      lam_a += lam_diff;
      lam_lam -= lam_diff;
      // ps = FhS - lam FEh / c^2
      double lam_FhS = lam_ps;
      lam_lam += -lam_ps * FEh * q.inv_c2;
      double lam_FEh = -lam_ps * lam * q.inv_c2;
      // lam = 2 c^2 UhS / den,  den = b + sqrt(disc)
      double lam_UhS = lam_lam * 2.0 * q.c2 / den;
      const double lam_den = -lam_lam * lam / den;
      double lam_b = lam_den;
      if (disc0 > 0.0) {
        const double lam_disc = lam_den * 0.5 / sd;
        lam_b += 2.0 * b * lam_disc;
        lam_FEh += -4.0 * UhS * lam_disc;
        lam_UhS += -4.0 * FEh * lam_disc;
      }
      // b = Eh + FhS; Eh = UhT + c^2 UhD; FEh = FhT + c^2 FhD
      lam_FhS += lam_b;
      const double lam_UhT = lam_b, lam_UhD = q.c2 * lam_b;
      const double lam_FhT = lam_FEh, lam_FhD = q.c2 * lam_FEh;
      // HLL rows: Uh = (aR UR - aL UL + FL - FR) ih, Fh = (aR FL - aL FR + aL aR (UR - UL)) ih
      double lam_aL = 0.0, lam_aR = 0.0;
#pragma unroll
      for (int k = 0; k < NV; ++k) {
        double lUh = 0.0, lFh = 0.0;
        if (k == 0) { lUh = lam_UhD; lFh = lam_FhD; }
        if (k == NV - 1) { lUh = lam_UhT; lFh = lam_FhT; }
#pragma unroll
        for (int j = 0; j < DIM; ++j)
          if (k == 1 + j && j == d) { lUh = lam_UhS; lFh = lam_FhS; }
        const double dU = sR.U[k] - sL.U[k];
        const double Uh = (aR * sR.U[k] - aL * sL.U[k] + FL[k] - FR[k]) * ih;
        const double Fh = (aR * FL[k] - aL * FR[k] + aL * aR * dU) * ih;
        lam_UR[k] += lUh * aR * ih + lFh * aL * aR * ih;
        lam_UL[k] += -lUh * aL * ih - lFh * aL * aR * ih;
        lam_FL[k] += lUh * ih + lFh * aR * ih;
        lam_FR[k] += -lUh * ih - lFh * aL * ih;
        lam_aR += lUh * (sR.U[k] - Uh) * ih + lFh * (FL[k] + aL * dU - Fh) * ih;
        lam_aL += lUh * (Uh - sL.U[k]) * ih + lFh * (-FR[k] + aR * dU + Fh) * ih;
      }
      // the upwind side's own U and F, and its speed
#pragma unroll
      for (int k = 0; k < NV; ++k) {
        if (left) {
          lam_UL[k] += lam_Us_side[k];
          lam_FL[k] += lam_Fs_side[k];
        } else {
          lam_UR[k] += lam_Us_side[k];
          lam_FR[k] += lam_Fs_side[k];
        }
      }
      if (left) lam_aL += lam_a; else lam_aR += lam_a;
      if (lmL <= lmR) lam_lmL = lam_aL; else lam_lmR = lam_aL;
      if (lpL >= lpR) lam_lpL = lam_aR; else lam_lpR = lam_aR;
    }
  }
  if (need_L) {
    SpeedParts p;
    speed_parts<EOS, DIM>(WL, sL, d, q, p);
    state_flux_speed_rev<EOS, DIM>(WL, sL, p, d, q, lam_UL, lam_FL, lam_lmL, lam_lpL, speeds, lam_WL);
  }
  if (need_R) {
    SpeedParts p;
    speed_parts<EOS, DIM>(WR, sR, d, q, p);
    state_flux_speed_rev<EOS, DIM>(WR, sR, p, d, q, lam_UR, lam_FR, lam_lmR, lam_lpR, speeds, lam_WR);
  }
}

// J[r][c] = dU_r / dW_c at the primitive state W (Eq. primitive_to_conserved).
template <int EOS, int DIM>
__host__ __device__ __forceinline__ void prim_jacobian(const double* W, const PhysParams& q, double J[DIM + 2][DIM + 2]) {
  constexpr int NV = DIM + 2;
  const double rho = W[0], P = W[NV - 1];
  double usq = 0.0;
#pragma unroll
  for (int j = 0; j < DIM; ++j) usq += W[1 + j] * W[1 + j];
  const double g2 = 1.0 + usq * q.inv_c2;
  const double g = sqrt(g2);
  const double th = P / rho;
  const double he = h_excess<EOS>(th, q);
  const double hd = h_excess_d<EOS>(th, q);
  const double H = rho * (q.c2 + he);      // rho h
  const double Hr = q.c2 + he - hd * th;   // dH/drho at fixed P
  const double Hp = hd;                    // dH/dP at fixed rho
  // D = g rho
  J[0][0] = g;
#pragma unroll
  for (int k = 0; k < DIM; ++k) J[0][1 + k] = rho * W[1 + k] * q.inv_c2 / g;
  J[0][NV - 1] = 0.0;
  // S_j = g H u_j / c^2
#pragma unroll
  for (int j = 0; j < DIM; ++j) {
    J[1 + j][0] = g * Hr * W[1 + j] * q.inv_c2;
    J[1 + j][NV - 1] = g * Hp * W[1 + j] * q.inv_c2;
#pragma unroll
    for (int k = 0; k < DIM; ++k)
      J[1 + j][1 + k] = H * q.inv_c2 * ((j == k ? g : 0.0) + W[1 + j] * W[1 + k] * q.inv_c2 / g);
  }
  // tau = g^2 H - P - g rho c^2
  J[NV - 1][0] = g2 * Hr - g * q.c2;
  J[NV - 1][NV - 1] = g2 * Hp - 1.0;
#pragma unroll
  for (int k = 0; k < DIM; ++k) J[NV - 1][1 + k] = W[1 + k] * q.inv_c2 * (2.0 * H - rho * q.c2 / g);
}

// Solve A^T x = b for x (Gaussian elimination with partial pivoting on A^T).
template <int N>
__host__ __device__ __forceinline__ void solve_transposed(const double A[N][N], const double* b, double* x) {
  double M[N][N + 1];
#pragma unroll
  for (int r = 0; r < N; ++r) {
#pragma unroll
    for (int c = 0; c < N; ++c) M[r][c] = A[c][r];
    M[r][N] = b[r];
  }
#pragma unroll
  for (int k = 0; k < N; ++k) {
    int piv = k;
    double best = fabs(M[k][k]);
#pragma unroll
    for (int r = k + 1; r < N; ++r) {
      const double v = fabs(M[r][k]);
      if (v > best) { best = v; piv = r; }
    }
#pragma unroll
    for (int r = k + 1; r < N; ++r) {
      if (r == piv) {
#pragma unroll
        for (int c = 0; c <= N; ++c) {
          const double tmp = M[k][c];
          M[k][c] = M[r][c];
          M[r][c] = tmp;
        }
      }
    }
    const double inv = 1.0 / M[k][k];
#pragma unroll
    for (int r = k + 1; r < N; ++r) {
      const double f = M[r][k] * inv;
#pragma unroll
      for (int c = k; c <= N; ++c) M[r][c] -= f * M[k][c];
    }
  }
#pragma unroll
  for (int k = N - 1; k >= 0; --k) {
    double s = M[k][N];
#pragma unroll
    for (int c = k + 1; c < N; ++c) s -= M[k][c] * x[c];
    x[k] = s / M[k][k];
  }
}

// Recovery adjoint by the implicit-function theorem: W = W(U) solves U(W) = U, so
// lam_U = (dU/dW)^{-T} lam_W at the recovered W.  Failed recoveries (floor state)
// do not depend on U: lam_U = 0.
template <int EOS, int DIM>
__host__ __device__ __forceinline__ void con2prim_rev(const double* W, int status, const PhysParams& q, const double* lam_W,
                                             double* lam_U) {
  constexpr int NV = DIM + 2;
  if (status != C2P_OK && status != C2P_NOCONV) {
#pragma unroll
    for (int k = 0; k < NV; ++k) lam_U[k] = 0.0;
    return;
  }
  double J[NV][NV];
  prim_jacobian<EOS, DIM>(W, q, J);
  solve_transposed<NV>(J, lam_W, lam_U);
}

// ---------------------------------------------------------------- dual numbers
// Forward-mode value with N tangents, used to differentiate the physicality
// operator's node factor on its active branch (only for flagged elements).
template <int N>
struct Dual {
  double v;
  double t[N];
};

template <int N>
__host__ __device__ __forceinline__ Dual<N> dconst(double v) {
  Dual<N> r;
  r.v = v;
#pragma unroll
  for (int i = 0; i < N; ++i) r.t[i] = 0.0;
  return r;
}
template <int N>
__host__ __device__ __forceinline__ Dual<N> operator+(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r; r.v = a.v + b.v;
#pragma unroll
  for (int i = 0; i < N; ++i) r.t[i] = a.t[i] + b.t[i];
  return r;
}
template <int N>
__host__ __device__ __forceinline__ Dual<N> operator-(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r; r.v = a.v - b.v;
#pragma unroll
  for (int i = 0; i < N; ++i) r.t[i] = a.t[i] - b.t[i];
  return r;
}
template <int N>
__host__ __device__ __forceinline__ Dual<N> operator*(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r; r.v = a.v * b.v;
#pragma unroll
  for (int i = 0; i < N; ++i) r.t[i] = a.t[i] * b.v + a.v * b.t[i];
  return r;
}
template <int N>
__host__ __device__ __forceinline__ Dual<N> operator*(double a, const Dual<N>& b) {
  Dual<N> r; r.v = a * b.v;
#pragma unroll
  for (int i = 0; i < N; ++i) r.t[i] = a * b.t[i];
  return r;
}
template <int N>
__host__ __device__ __forceinline__ Dual<N> operator/(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r; r.v = a.v / b.v;
  const double ib = 1.0 / b.v;
#pragma unroll
  for (int i = 0; i < N; ++i) r.t[i] = (a.t[i] - r.v * b.t[i]) * ib;
  return r;
}
template <int N>
__host__ __device__ __forceinline__ Dual<N> dsqrt(const Dual<N>& a) {
  Dual<N> r; r.v = sqrt(a.v);
  const double f = (r.v > 0.0) ? 0.5 / r.v : 0.0;
#pragma unroll
  for (int i = 0; i < N; ++i) r.t[i] = a.t[i] * f;
  return r;
}

// The node factor s_i of the physicality operator (same arithmetic and branches
// as node_factor in kernels.hpp) in dual numbers over (U_i, U_bar).
template <int DIM, int N>
__host__ __device__ __forceinline__ Dual<N> node_factor_dual(const Dual<N>* Ui, const Dual<N>* Ub, const PhysParams& q) {
  constexpr int NV = DIM + 2;
  const double eps = q.eps;
  const Dual<N> Di = Ui[0], Ei = Ui[NV - 1] + q.c2 * Ui[0];
  const Dual<N> Db = Ub[0], Eb = Ub[NV - 1] + q.c2 * Ub[0];
  const Dual<N> one = dconst<N>(1.0);
  const Dual<N> sD = (Di.v >= eps * Db.v) ? one : ((1.0 - eps) * Db) / (Db - Di);
  const Dual<N> sE = (Ei.v >= eps * Eb.v) ? one : ((1.0 - eps) * Eb) / (Eb - Ei);
  const Dual<N> s1 = (sE.v < sD.v) ? sE : sD;
  Dual<N> U1[NV], dl[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    U1[v] = s1 * Ui[v] + (one - s1) * Ub[v];
    dl[v] = U1[v] - Ub[v];
  }
  const Dual<N> tb = q.inv_c2 * Ub[NV - 1];
  Dual<N> sb2 = dconst<N>(0.0), s12 = dconst<N>(0.0), ds2 = dconst<N>(0.0), sbds = dconst<N>(0.0);
#pragma unroll
  for (int j = 0; j < DIM; ++j) {
    const Dual<N> sb = q.inv_c * Ub[1 + j], s1j = q.inv_c * U1[1 + j], dsj = q.inv_c * dl[1 + j];
    sb2 = sb2 + sb * sb;
    s12 = s12 + s1j * s1j;
    ds2 = ds2 + dsj * dsj;
    sbds = sbds + sb * dsj;
  }
  const Dual<N> Qb = tb * (tb + 2.0 * Ub[0]) - sb2;
  const Dual<N> t1 = q.inv_c2 * U1[NV - 1];
  const Dual<N> Q1 = t1 * (t1 + 2.0 * U1[0]) - s12;
  if (!(Q1.v < eps * Qb.v)) return s1;
  const Dual<N> dt = q.inv_c2 * dl[NV - 1], dD = dl[0];
  const Dual<N> a = dt * (dt + 2.0 * dD) - ds2;
  const Dual<N> b = 2.0 * (tb * dt + tb * dD + Ub[0] * dt - sbds);
  const Dual<N> cp = (1.0 - eps) * Qb;
  Dual<N> disc = b * b - 4.0 * a * cp;
  if (disc.v < 0.0) disc = dconst<N>(0.0);
  const Dual<N> s2 = (2.0 * cp) / (dsqrt(disc) - b);
  return s1 * s2;
}

}  // namespace dgsrhd
