"""Cancellation ratio of the DG right-hand side, for the FP64 parity bars.

Every component of R = V + S is a sum of products of basis weights with nodal and
numerical fluxes.  Two FP64 evaluations of it that round differently (another
order of operations, fused multiply-adds, a few-ulp recovery) can differ by
about u * T, u = 2^-53, where T is the sum of the magnitudes of those terms:

  T_i = sum_d (2/dx_d) [ sum_a |dhat[i_d, a]| |F^d|_a
                         + (1/w_{i_d}) (|l_{i_d}(+1)| |Fhat^+| + |l_{i_d}(-1)| |Fhat^-|) ]

with |F^d| = (|D v_d|, |S v_d| + P e_d, (|tau| + P)|v_d|) the magnitudes of the
flux's own terms and |Fhat| the magnitude of the HLL combination
(|lambda_R| |F_L| + |lambda_L| |F_R| + |lambda_L lambda_R| (|U_L| + |U_R|)) / (lambda_R - lambda_L)
(or the upwind |F| outside the fan).  The cancellation ratio of component k is
kappa_k = max_i T_k,i / ||R_k||_inf: the normwise relative difference to expect
between two correct evaluations is a modest multiple of u kappa_k.

Built from the oracle's own flux, wavespeed and trace functions on absolute
values; no method arithmetic of its own beyond those magnitudes."""
from __future__ import annotations

import torch

from oracle import basis
from oracle import dg as odg
from oracle import srhd
from oracle.con2prim import con2prim

U_ROUND = 2.0 ** -53


def _flux_mag(W, d, st):
    U = srhd.prim_to_cons(W, st).abs()
    rho, u, P = W[0], W[1:-1], W[-1]
    vd = (u[d] / srhd.lorentz(u, st.c)).abs()
    F = U * vd
    F[1 + d] = F[1 + d] + P.abs()
    F[-1] = F[-1] + P.abs() * vd
    return F


def _hll_mag(WL, WR, d, st):
    UL, UR = srhd.prim_to_cons(WL, st).abs(), srhd.prim_to_cons(WR, st).abs()
    FL, FR = _flux_mag(WL, d, st), _flux_mag(WR, d, st)
    lmL, lpL = srhd.wavespeeds(WL, d, st)
    lmR, lpR = srhd.wavespeeds(WR, d, st)
    aL = torch.minimum(lmL, lmR)
    aR = torch.maximum(lpL, lpR)
    mid = (aR.abs() * FL + aL.abs() * FR + (aL * aR).abs() * (UR + UL)) / (aR - aL)
    return torch.where(aL >= 0, FL, torch.where(aR <= 0, FR, mid))


def rhs_term_magnitude(U, st):
    """T (same layout as U): the magnitude sum of the terms of every R component."""
    tb = basis.tables(st.p)
    W, _ = con2prim(U, st)
    adh = torch.as_tensor(abs(tb["dhat"]), dtype=torch.float64)
    T = torch.zeros_like(W)
    for d in range(st.dim):
        ax, ea = 6 - d, 3 - d
        F = _flux_mag(W, d, st)
        T = T + (2.0 / st.dx(d)) * torch.movedim(torch.tensordot(F, adh, dims=([ax], [1])), -1, ax)
        Wm, Wp, _ = odg.traces(W, d, st)
        WL, WR = odg.face_states(Wm, Wp, d, st)
        Fh = _hll_mag(WL, WR, d, st)
        n = W.shape[ea]
        Fplus = Fh.narrow(ea, 1, n).unsqueeze(ax)
        Fminus = Fh.narrow(ea, 0, n).unsqueeze(ax)
        shp = [1] * 7
        shp[ax] = st.p + 1
        cp = torch.as_tensor(abs(tb["lp"]) / tb["w"], dtype=torch.float64).reshape(shp)
        cm = torch.as_tensor(abs(tb["lm"]) / tb["w"], dtype=torch.float64).reshape(shp)
        T = T + (2.0 / st.dx(d)) * (cp * Fplus + cm * Fminus)
    return T


def rhs_cancellation(U, st, R=None):
    """kappa_k per conserved component (tensor of n_var values)."""
    if R is None:
        R = odg.rhs(U, st)
    T = rhs_term_magnitude(U, st).reshape(U.shape[0], -1).abs().max(1).values
    Rn = R.reshape(U.shape[0], -1).abs().max(1).values.clamp(min=1e-300)
    return T / Rn
