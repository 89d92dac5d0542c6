"""SRHD state relations (Sec. 2.1, 2.4, 2.5).  Test infrastructure.

Primitive state W = (rho, u_1..u_dim, P), u = gamma v the spatial part of the
4-velocity (Sec. 2.1).  Conserved state U = (D, S_1..S_dim, tau) with
S = M (the momentum density) and tau = E - D c^2 (the energy minus the rest
mass; a linear change of variables of the paper's (D, M, E)).

prim_to_cons   Eq. (primitive_to_conserved): D = gamma rho,
               M = gamma rho h u / c^2, E = gamma^2 rho h - P.
               tau is formed as D |u|^2/(gamma+1) + gamma^2 rho (h-c^2) - P,
               which equals gamma^2 rho h - P - D c^2 without cancellation.
flux           Eq. (srhd_flux) along direction d:
               (D v_d, S v_d + P e_d, (tau + P) v_d)  [energy row minus c^2
               times the mass row, for the tau variable].
wavespeeds     lambda_pm = (v_d pm sqrt(sigma (c^2 - v_d^2 + c^2 sigma)))/(1+sigma),
               sigma = c_s^2 / (gamma^2 (c^2 - c_s^2))  (Sec. 2.4).
hll            HLL flux with lambda_L = min of the two lambda_-, lambda_R = max
               of the two lambda_+ (Sec. 2.4); the three-branch HLL formula
               itself is the textbook one (the paper names the solver only).
hllc           HLLC flux (the paper's second solver, Sec. 2.4, after Mignone &
               Bodo 2005 and its multidimensional form): one contact of speed
               lambda* and pressure p* between the HLL speeds; the star states
               follow from the jump conditions across the outer waves and the
               contact conditions (normal velocity lambda*, pressure p*); lambda* is
               the root inside the HLL fan of the quadratic those conditions give
               in the HLL state and flux.
q_admiss       Eq. (physicality) with the plus sign of its second statement
               (Sec. 2.5): q = E/c^2 - sqrt(D^2 + |M|^2/c^2), written in tau
               form as tau/c^2 - (|S|^2/c^2)/(D + sqrt(D^2 + |S|^2/c^2)).

Pinned by tests/test_oracle_srhd.py: a Lorentz boost of the rest-frame
stress-energy tensor reproduces prim_to_cons; the lambda_pm equal the extreme
eigenvalues of dF/dU (Jacobian by autograd, eigenvalues by LAPACK) and reduce
to relativistic velocity addition when the transverse velocity vanishes;
HLL consistency F(W, W) = F(W) and upwinding; HLLC consistency, upwinding, the
contact conditions on both star states, and exact resolution of an isolated
contact (density and tangential-velocity jumps at equal pressure and normal
velocity), which HLL smears.
"""
from __future__ import annotations

import torch

from .eos import h_excess, sound_speed_sq
from .setup import HLLC


def lorentz(u, c: float):
    """gamma = sqrt(1 + |u|^2/c^2); u has the component axis first."""
    return torch.sqrt(1.0 + (u * u).sum(0) / (c * c))


def u_from_v(v, c: float):
    """4-velocity spatial part from the 3-velocity: u = v / sqrt(1 - |v|^2/c^2)."""
    g = 1.0 / torch.sqrt(1.0 - (v * v).sum(0) / (c * c))
    return g * v


def prim_to_cons(W, st):
    """W [nvar, ...] -> U [nvar, ...] (D, S, tau)."""
    c = st.c
    rho, u, P = W[0], W[1:-1], W[-1]
    g = lorentz(u, c)
    he = h_excess(P / rho, st.eos, st.gamma_ad, c)
    D = g * rho
    S = g * rho * (c * c + he) * u / (c * c)
    usq = (u * u).sum(0)
    tau = D * usq / (g + 1.0) + g * g * rho * he - P
    return torch.cat([D[None], S, tau[None]], 0)


def prim3_to_cons(rho, v, P, st):
    """(rho, 3-velocity, P) -> U; the input form used for initial data."""
    u = u_from_v(v, st.c)
    return prim_to_cons(torch.cat([rho[None], u, P[None]], 0), st)


def flux(W, d: int, st):
    """Physical flux F^d(W) in the (D, S, tau) variables."""
    U = prim_to_cons(W, st)
    rho, u, P = W[0], W[1:-1], W[-1]
    g = lorentz(u, st.c)
    vd = u[d] / g
    F = U * vd
    F = F.clone()
    F[1 + d] = F[1 + d] + P
    F[-1] = F[-1] + P * vd
    return F


def wavespeeds(W, d: int, st):
    c = st.c
    rho, u, P = W[0], W[1:-1], W[-1]
    cs2 = sound_speed_sq(P / rho, st.eos, st.gamma_ad, c)
    g2 = 1.0 + (u * u).sum(0) / (c * c)
    vd = u[d] / torch.sqrt(g2)
    sigma = cs2 / (g2 * (c * c - cs2))
    root = torch.sqrt(sigma * (c * c - vd * vd + c * c * sigma))
    return (vd - root) / (1.0 + sigma), (vd + root) / (1.0 + sigma)


def hll(WL, WR, d: int, st):
    UL, UR = prim_to_cons(WL, st), prim_to_cons(WR, st)
    FL, FR = flux(WL, d, st), flux(WR, d, st)
    lmL, lpL = wavespeeds(WL, d, st)
    lmR, lpR = wavespeeds(WR, d, st)
    aL = torch.minimum(lmL, lmR)
    aR = torch.maximum(lpL, lpR)
    mid = (aR * FL - aL * FR + aL * aR * (UR - UL)) / (aR - aL)
    return torch.where(aL >= 0, FL, torch.where(aR <= 0, FR, mid))


def hllc_star(WL, WR, d: int, st):
    """The pieces of the HLLC flux along d: outer speeds lamL, lamR (those of hll), the
    contact speed lam* and pressure p*, and the star states UsL, UsR (D, S, tau).

    With E = tau + D c^2 and, for side K, A_K = lam_K E_K - F_E,K and
    B_K = lam_K S_d,K - F_Sd,K (F_E = c^2 S_d the energy flux), the jump conditions
    across the K wave with the contact conditions (normal velocity lam*, pressure p*,
    c^2 S*_d = (E* + p*) lam*) give p* (c^2 - lam_K lam*) = A_K lam* - c^2 B_K for both
    K.  Eliminating p* leaves, in HLL averages,
        F^hll_E lam*^2 - c^2 (E^hll + F^hll_Sd) lam* + c^4 S^hll_d = 0,
    p* = F^hll_Sd - lam* F^hll_E / c^2,
    which for c = 1 is the quadratic of Mignone & Bodo (2005).  lam* is its root with
    the minus sign, written as 2 c^2 S^hll_d / (b + sqrt(b^2 - 4 F^hll_E S^hll_d)),
    b = E^hll + F^hll_Sd (no cancellation when F^hll_E is small).  The star states:
        U*_K = (lam_K U_K - F_K + p* (0, e_d, lam*)) / (lam_K - lam*)
    in (D, S, tau) (the tau row gets p* lam* like the energy row)."""
    c2 = st.c * st.c
    UL, UR = prim_to_cons(WL, st), prim_to_cons(WR, st)
    FL, FR = flux(WL, d, st), flux(WR, d, st)
    lmL, lpL = wavespeeds(WL, d, st)
    lmR, lpR = wavespeeds(WR, d, st)
    aL = torch.minimum(lmL, lmR)
    aR = torch.maximum(lpL, lpR)
    Uh = (aR * UR - aL * UL + FL - FR) / (aR - aL)              # HLL state
    Fh = (aR * FL - aL * FR + aL * aR * (UR - UL)) / (aR - aL)  # HLL flux
    ks = 1 + d                                                   # S_d row
    E_h = Uh[-1] + c2 * Uh[0]
    FE_h = Fh[-1] + c2 * Fh[0]
    b = E_h + Fh[ks]
    disc = torch.clamp(b * b - 4.0 * FE_h * Uh[ks], min=0.0)
    lam = 2.0 * c2 * Uh[ks] / (b + torch.sqrt(disc))
    ps = Fh[ks] - lam * FE_h / c2

    def star(U, F, a):
        extra = torch.zeros_like(U)
        extra[ks] = ps
        extra[-1] = ps * lam
        return (a * U - F + extra) / (a - lam)

    return aL, aR, lam, ps, star(UL, FL, aL), star(UR, FR, aR)


def hllc(WL, WR, d: int, st):
    """HLLC flux: F_L if lamL >= 0, F_L + lamL (U*_L - U_L) if lamL < 0 <= lam*,
    F_R + lamR (U*_R - U_R) if lam* < 0 < lamR, F_R if lamR <= 0."""
    UL, UR = prim_to_cons(WL, st), prim_to_cons(WR, st)
    FL, FR = flux(WL, d, st), flux(WR, d, st)
    aL, aR, lam, _, UsL, UsR = hllc_star(WL, WR, d, st)
    FsL = FL + aL * (UsL - UL)
    FsR = FR + aR * (UsR - UR)
    return torch.where(aL >= 0, FL, torch.where(lam >= 0, FsL, torch.where(aR > 0, FsR, FR)))


def face_flux(WL, WR, d: int, st):
    """The numerical flux the setup selects (HLL or HLLC)."""
    return hllc(WL, WR, d, st) if st.flux == HLLC else hll(WL, WR, d, st)


def q_admiss(U, st):
    c = st.c
    D, S, tau = U[0], U[1:-1], U[-1]
    s2 = (S * S).sum(0) / (c * c)
    return tau / (c * c) - s2 / (D + torch.sqrt(D * D + s2))


def admissible(U, st):
    return (U[0] > 0) & (q_admiss(U, st) > 0)
