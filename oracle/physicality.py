"""Physicality-enforcing operator (Sec. 2.5, the four-step procedure).  Test infrastructure.

Per element:
 1. flag the element if any node violates Eq. (physicality): D > 0 and q > 0;
 2. volume average U_bar = sum_i w_i U_i / sum_i w_i (tensor GL weights); if
    U_bar itself violates Eq. (physicality) the element is left unchanged and
    counted (reading: the paper says only that it cannot be made physical);
 3. per node i, two stages (Eqs. first_stage_positivity ... second_stage_solution):
    a. s_D, s_E: the largest s in [0,1] keeping D and E = tau + D c^2 positive
       along U_bar + s (U_i - U_bar);
    b. s1 = min(s_D, s_E),  U1 = s1 U_i + (1 - s1) U_bar;
    c. if U1 is admissible, s_i = s1;
    d. else s2 is the root in (0,1) of a s^2 + b s + c of Eq.
       (second_stage_coefficients) and s_i = s1 s2;
 4. s = min_i s_i and U_i <- s U_i + (1 - s) U_bar for every node.

Readings (the paper's strict inequalities have no largest solution, and its
printed coefficients are garbled):
  * the sign under the root of Eq. (physicality) is '+' (its second statement);
  * the b coefficient has no square on (M1 - M_bar);
  * a relative margin eps (1e-12): stage a targets D >= eps D_bar and
    E >= eps E_bar, stage c tests Q(U1) >= eps Q(U_bar), and stage d solves
    a s^2 + b s + (1 - eps) c = 0 with the stable root
    s2 = 2 (1-eps) c / (-b + sqrt(b^2 - 4 a (1-eps) c)), equal to the paper's
    (-b - sqrt(b^2 - 4ac))/(2a) for either sign of a;
  * Q(U) = (E/c^2)^2 - D^2 - |M|^2/c^2 and the coefficients are evaluated in
    tau form: with t = tau/c^2 and s = S/c, Q = t (t + 2D) - |s|^2,
    a = dt (dt + 2 dD) - |ds|^2, b = 2 (t_bar dt + t_bar dD + D_bar dt - s_bar.ds),
    c = Q(U_bar), where d* = U1 - U_bar.

Pinned by tests/test_oracle_physicality.py: bisection on s per node (brute
force) matches the closed form, averages are preserved, every node is
admissible afterwards, unflagged elements are untouched, idempotence.
"""
from __future__ import annotations

import torch

from .dg import elem_weights
from .srhd import admissible


def node_factor(Ui, Ub, st, eps):
    """s_i for the nodes Ui [nvar, n] of one element with average Ub [nvar]."""
    c2 = st.c * st.c
    Di, Ei = Ui[0], Ui[-1] + Ui[0] * c2
    Db, Eb = Ub[0], Ub[-1] + Ub[0] * c2
    one = torch.ones_like(Di)
    sD = torch.where(Di >= eps * Db, one, (1.0 - eps) * Db / (Db - Di))
    sE = torch.where(Ei >= eps * Eb, one, (1.0 - eps) * Eb / (Eb - Ei))
    s1 = torch.minimum(sD, sE)
    U1 = s1 * Ui + (1.0 - s1) * Ub[:, None]
    dl = U1 - Ub[:, None]

    def Q(t, D, s):
        return t * (t + 2.0 * D) - (s * s).sum(0)

    tb, sb = Ub[-1] / c2, Ub[1:-1] / st.c
    Qb = Q(tb, Ub[0], sb)
    Q1 = Q(U1[-1] / c2, U1[0], U1[1:-1] / st.c)
    dt, dD, ds = dl[-1] / c2, dl[0], dl[1:-1] / st.c
    a = dt * (dt + 2.0 * dD) - (ds * ds).sum(0)
    b = 2.0 * (tb * dt + tb * dD + Ub[0] * dt - (sb[:, None] * ds).sum(0))
    cp = (1.0 - eps) * Qb
    disc = torch.clamp(b * b - 4.0 * a * cp, min=0.0)
    s2 = 2.0 * cp / (-b + torch.sqrt(disc))
    need2 = Q1 < eps * Qb
    return torch.where(need2, s1 * s2, s1)


def enforce(U, st, stats=None):
    """Apply the operator to every element of U [nvar, nez, ney, nex, nk, nj, ni]."""
    eps = st.phys_eps
    adm = admissible(U, st)
    flagged = ~adm.flatten(3).all(-1)                  # [nez, ney, nex]
    if stats is not None:
        stats["flagged"] = stats.get("flagged", 0) + int(flagged.sum())
    if not bool(flagged.any()):
        return U
    w = elem_weights(st)
    Ubar = (U * w).sum((4, 5, 6)) / w.sum()             # [nvar, nez, ney, nex]
    out = U.clone()
    nv = U.shape[0]
    for idx in flagged.nonzero().tolist():
        ez, ey, ex = idx
        Ub = Ubar[:, ez, ey, ex]
        if not bool(admissible(Ub[:, None], st).all()):
            if stats is not None:
                stats["bad_average"] = stats.get("bad_average", 0) + 1
            continue
        Ui = U[:, ez, ey, ex].reshape(nv, -1)
        s = node_factor(Ui, Ub, st, eps).min()
        new = s * Ui + (1.0 - s) * Ub[:, None]
        out[:, ez, ey, ex] = new.reshape(U[:, ez, ey, ex].shape)
        if stats is not None:
            stats["smoothed"] = stats.get("smoothed", 0) + 1
    return out
