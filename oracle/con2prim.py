"""Conserved-to-primitive recovery, the four solvers of Sec. 3.  Test infrastructure.

Dimensionless variables (Sec. 3): xi = |M|/(D c), eta = E/(D c^2).  With the
stored tau = E - D c^2, eta = 1 + t where t = tau/(D c^2), and the combinations
alpha eta +- 1 are formed as alpha t + alpha +- 1.

ideal_newton   Sec. 3.1, iterative: Newton-Raphson on the quartic P(w) of
               Eq. (iterative_quartic), w in (0, 1), beta = 2w/(1+w^2)
               [Eq. (iterative_quartic_unknown)].  Readings: initial guess
               w0 = b/(1+sqrt(1-b^2)) with b = xi/eta (an upper bound of beta);
               stop when |dw| <= 1e-13 w, at most 30 iterations; an iterate that
               leaves (0,1) is pulled back halfway to the violated end; for
               xi < 1e-4 the cubic series of Eq. (iterative_cubic_approximation)
               is used instead.  Pressure from the tau form of
               P = (Gamma-1)(E - M.v - rho c^2):
               P = (Gamma-1)(tau - |S| beta c + D c^2 2w^2/(1+w^2)).
ideal_quartic  Sec. 3.1, analytic: the quartic in beta solved through its
               resolvent cubic.  Readings of garbled print: the quartic is
               beta^4 + a3 beta^3 + a2 beta^2 + a1 beta + a0;
               R = (9 i1 i2 - 27 i3 - 2 i1^3)/54; trigonometric branch
               x = 2 sqrt(-S) cos(atan2(sqrt(-T), R)/3) - i1/3.
               Pinned against the exact state on beta in [0.3, 0.99] (beta to
               2e-9, rho to 3e-8, P to 5e-8); below beta ~ 0.3 the chain loses
               digits to cancellation and its accuracy is only measured.
tm_cubic       Sec. 3.2, analytic: the cubic of Eq. (synge_cubic) in
               W = gamma^2 - 1 by the trigonometric (d < 0) or Cardano (d >= 0)
               formula, then one Newton step on the same cubic (reading: the
               closed form alone loses relative precision as |v| -> 0), W >= 0.
               P = ((E - M.v)^2 - (rho c^2)^2)/(3 (E - M.v)) (the printed form
               is in c = 1 units), evaluated as X_(X_ + 2 rho c^2)/(3 X) with
               X_ = X - rho c^2 = tau - |S| beta c + D c^2 W/(gamma(gamma+1)).
tm_brent       Sec. 3.2, iterative: Brent's method (scipy.optimize.brentq) on the
               same cubic, bracket W in [0, 200^2 - 1] expanded by 4x until it
               brackets.

Fixed iteration counts (Sec. 3.3, the recovery study: 6 and 12 Newton iterations,
25 and 50 for the TM iterative solver; Setup.c2p_iters > 0): ideal_newton runs
exactly that many Newton steps from w = 1/2 with no convergence test; the TM iterative solver runs Brent's method
as published (brent_steps below, Brent 1973, "zero" with tolerance 2 eps |b|) for at
most that many steps, because scipy's brentq does not expose its iterate after a
given number of steps.  brent_steps is pinned against scipy's brentq at
convergence, by the bracket it keeps at every step and by its step count bound.

Failure convention (reading; the paper does not specify one): if D <= 0 or
q <= 0 (Eq. physicality) or the recovered P <= 0, the node gets
rho = 1e-10, u = 0, P = 1e-10 c^2 and a nonzero status.

Pinned by tests/test_oracle_con2prim.py: round trip prim -> cons -> prim on the
well-conditioned domain, the paper's 25x25 (gamma, P) grid with c = 3e8,
residual of the quartic / cubic at the exact root computed from the
primitives, bisection on the defining equation, and the series vs Newton.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from .setup import BRENT, CUBIC, IDEAL, NEWTON, QUARTIC, TM
from .srhd import admissible

RHO_FLOOR = 1e-10
P_FLOOR = 1e-10

ST_OK, ST_INADMISSIBLE, ST_NOCONV, ST_BADP = 0, 1, 2, 3


def _prep(U, st):
    c = st.c
    ok = admissible(U, st)
    D = torch.where(ok, U[0], torch.ones_like(U[0]))
    S = torch.where(ok[None], U[1:-1], torch.zeros_like(U[1:-1]))
    tau = torch.where(ok, U[-1], torch.ones_like(U[-1]))
    s2 = (S * S).sum(0)
    pos = s2 > 0
    Smag = torch.sqrt(torch.where(pos, s2, torch.ones_like(s2)))
    Smag = torch.where(pos, Smag, torch.zeros_like(Smag))
    nhat = S / torch.where(pos, Smag, torch.ones_like(Smag))
    xi = Smag / (D * c)
    t = tau / (D * c * c)
    return ok, D, S, tau, Smag, nhat, xi, t


def _finish(ok, D, Smag, nhat, gam, gb, rho, P, st, status):
    c = st.c
    u = gb * c * nhat
    good = ok & (P > 0) & torch.isfinite(P) & torch.isfinite(rho)
    status = torch.where(ok & ~good, torch.full_like(status, ST_BADP), status)
    rho = torch.where(good, rho, torch.full_like(rho, RHO_FLOOR))
    P = torch.where(good, P, torch.full_like(P, P_FLOOR * c * c))
    u = torch.where(good[None], u, torch.zeros_like(u))
    return torch.cat([rho[None], u, P[None]], 0), status


def ideal_newton(U, st, tol=1e-13, max_iter=30, series_below=1e-4, w_start=None):
    c, G = st.c, st.gamma_ad
    ok, D, S, tau, Smag, nhat, xi, t = _prep(U, st)
    alpha = G / (G - 1.0)
    eta = 1.0 + t
    A = (alpha - 1.0) * xi
    B = 2.0 * (alpha * t + alpha + 1.0)      # 2 (alpha eta + 1)
    C = 2.0 * (alpha + 1.0) * xi
    Dd = 2.0 * (alpha * t + alpha - 1.0)     # 2 (alpha eta - 1)
    b = xi / eta
    w = b / (1.0 + torch.sqrt(1.0 - b * b))
    if w_start is not None:
        w = torch.full_like(w, w_start)
    small = xi < series_below
    active = ok & ~small
    for _ in range(max_iter):
        if not bool(active.any()):
            break
        Pw = (((A * w - B) * w + C) * w - Dd) * w + A
        dPw = ((4.0 * A * w - 3.0 * B) * w + 2.0 * C) * w - Dd
        wn = w - Pw / dPw
        wn = torch.where(wn <= 0, 0.5 * w, torch.where(wn >= 1, 0.5 * (w + 1.0), wn))
        step = (wn - w).abs()
        w = torch.where(active, wn, w)
        active = active & ~(step <= tol * wn)
    status = torch.where(ok, torch.zeros_like(xi, dtype=torch.int32),
                         torch.full_like(xi, ST_INADMISSIBLE, dtype=torch.int32))
    status = torch.where(active, torch.full_like(status, ST_NOCONV), status)
    # cubic series for small xi (Eq. iterative_cubic_approximation)
    ame = 0.5 * Dd                           # alpha eta - 1
    ape = 0.5 * B                            # alpha eta + 1
    k1 = (alpha - 1.0) / (2.0 * ame)
    k3 = (alpha - 1.0) ** 2 / (8.0 * ame ** 4) * ((alpha + 3.0) * ape - 4.0 * (alpha + 1.0))
    w = torch.where(small, k1 * xi + k3 * xi ** 3, w)
    w2 = w * w
    om = (1.0 - w) * (1.0 + w)
    beta = 2.0 * w / (1.0 + w2)
    gam = (1.0 + w2) / om
    gb = 2.0 * w / om
    rho = D / gam
    P = (G - 1.0) * (tau - Smag * beta * c + D * c * c * 2.0 * w2 / (1.0 + w2))
    return _finish(ok, D, Smag, nhat, gam, gb, rho, P, st, status)


def _cbrt(x):
    return torch.sign(x) * torch.abs(x) ** (1.0 / 3.0)


def ideal_quartic(U, st):
    c, G = st.c, st.gamma_ad
    ok, D, S, tau, Smag, nhat, xi, t = _prep(U, st)
    eta = 1.0 + t
    den = (G - 1.0) ** 2 * (xi * xi + 1.0)
    a3 = -2.0 * G * (G - 1.0) * xi * eta / den
    a2 = (G * G * eta * eta + 2.0 * (G - 1.0) * xi * xi - (G - 1.0) ** 2) / den
    a1 = -2.0 * G * xi * eta / den
    a0 = xi * xi / den
    i1 = -a2
    i2 = a3 * a1 - 4.0 * a0
    i3 = 4.0 * a2 * a0 - a1 * a1 - a3 * a3 * a0
    R = (9.0 * i1 * i2 - 27.0 * i3 - 2.0 * i1 ** 3) / 54.0
    Sq = (3.0 * i2 - i1 * i1) / 9.0
    T = R * R + Sq ** 3
    neg = T < 0
    Sn = torch.where(neg, Sq, -torch.ones_like(Sq))
    Tn = torch.where(neg, T, -torch.ones_like(T))
    x_trig = 2.0 * torch.sqrt(-Sn) * torch.cos(torch.atan2(torch.sqrt(-Tn), R) / 3.0) - i1 / 3.0
    Tp = torch.where(neg, torch.zeros_like(T), T)
    x_card = _cbrt(R + torch.sqrt(Tp)) + _cbrt(R - torch.sqrt(Tp)) - i1 / 3.0
    x = torch.where(neg, x_trig, x_card)
    Bq = 0.5 * (a3 + torch.sqrt(a3 * a3 - 4.0 * a2 + 4.0 * x))
    Cq = 0.5 * (x - torch.sqrt(x * x - 4.0 * a0))
    beta = 0.5 * (-Bq + torch.sqrt(Bq * Bq - 4.0 * Cq))
    beta = torch.where(xi > 0, beta, torch.zeros_like(beta))
    sq = torch.sqrt((1.0 - beta) * (1.0 + beta))
    gam = 1.0 / sq
    gb = beta / sq
    rho = D * sq
    P = (G - 1.0) * (tau - Smag * beta * c + D * c * c * beta * beta / (1.0 + sq))
    status = torch.where(ok, torch.zeros_like(xi, dtype=torch.int32),
                         torch.full_like(xi, ST_INADMISSIBLE, dtype=torch.int32))
    bad = ok & ~torch.isfinite(beta)
    status = torch.where(bad, torch.full_like(status, ST_NOCONV), status)
    return _finish(ok & ~bad, D, Smag, nhat, gam, gb, rho, P, st, status)


def _tm_coeffs(xi, eta):
    x2, e2 = xi * xi, eta * eta
    den = ((eta - xi) * (eta + xi)) ** 2
    k = 4.0 * (e2 + x2) - (x2 + 1.0)
    c1 = ((e2 + x2) * k - 14.0 * x2 * e2) / (2.0 * den)
    c2 = (k * k - 57.0 * x2 * e2) / (16.0 * den)
    c3 = -9.0 * x2 * e2 / (16.0 * den)
    return c1, c2, c3


def _tm_recover(ok, D, tau, Smag, nhat, W, st, status):
    c = st.c
    Wc = torch.clamp(W, min=0.0)
    gam = torch.sqrt(1.0 + Wc)
    beta = torch.sqrt(Wc / (Wc + 1.0))
    gb = torch.sqrt(Wc)
    rho = D / gam
    Xm = tau - Smag * beta * c + D * c * c * Wc / (gam * (gam + 1.0))
    X = Xm + rho * c * c
    P = Xm * (Xm + 2.0 * rho * c * c) / (3.0 * X)
    return _finish(ok, D, Smag, nhat, gam, gb, rho, P, st, status)


def tm_cubic(U, st):
    ok, D, S, tau, Smag, nhat, xi, t = _prep(U, st)
    eta = 1.0 + t
    c1, c2, c3 = _tm_coeffs(xi, eta)
    Q = (3.0 * c2 - c1 * c1) / 9.0
    R = (9.0 * c1 * c2 - 27.0 * c3 - 2.0 * c1 ** 3) / 54.0
    d = Q ** 3 + R * R
    neg = d < 0
    Qn = torch.where(neg, Q, -torch.ones_like(Q))
    arg = torch.clamp(R / torch.sqrt(-Qn ** 3), -1.0, 1.0)
    W_trig = 2.0 * torch.sqrt(-Qn) * torch.cos(torch.acos(arg) / 3.0) - c1 / 3.0
    dp = torch.where(neg, torch.zeros_like(d), d)
    W_card = -c1 / 3.0 + _cbrt(R + torch.sqrt(dp)) + _cbrt(R - torch.sqrt(dp))
    W = torch.where(neg, W_trig, W_card)
    f = ((W + c1) * W + c2) * W + c3
    fp = (3.0 * W + 2.0 * c1) * W + c2
    W = W - f / fp
    status = torch.where(ok, torch.zeros_like(xi, dtype=torch.int32),
                         torch.full_like(xi, ST_INADMISSIBLE, dtype=torch.int32))
    return _tm_recover(ok, D, tau, Smag, nhat, W, st, status)


def tm_brent(U, st, xtol=1e-300, rtol=4.0 * np.finfo(float).eps):
    from scipy.optimize import brentq
    ok, D, S, tau, Smag, nhat, xi, t = _prep(U, st)
    eta = 1.0 + t
    c1, c2, c3 = _tm_coeffs(xi, eta)
    c1n, c2n, c3n = (v.detach().reshape(-1).numpy() for v in (c1, c2, c3))
    okn = ok.reshape(-1).numpy()
    Wn = np.zeros_like(c1n)
    for k in range(Wn.size):
        if not okn[k] or c3n[k] == 0.0:
            continue
        f = (lambda W, a=c1n[k], b=c2n[k], cc=c3n[k]: ((W + a) * W + b) * W + cc)
        hi = 200.0 ** 2 - 1.0
        while f(hi) < 0:
            hi *= 4.0
        Wn[k] = brentq(f, 0.0, hi, xtol=xtol, rtol=rtol, maxiter=200)
    W = torch.from_numpy(Wn).reshape(xi.shape)
    status = torch.where(ok, torch.zeros_like(xi, dtype=torch.int32),
                         torch.full_like(xi, ST_INADMISSIBLE, dtype=torch.int32))
    return _tm_recover(ok, D, tau, Smag, nhat, W, st, status)


def brent_steps(f, a, b, max_steps, history=None):
    """Brent's root finder (Brent 1973, the procedure "zero") on [a, b] with f(a) f(b) <= 0:
    at each step keep b the best iterate and c the other end of a bracket [b, c]; try
    inverse quadratic interpolation through (a, b, c) (the secant when a = c), accept the
    step only if it lands well inside the bracket and shrinks faster than the step before
    the last, else bisect.  Tolerance 2 eps |b|.  Returns b after convergence or after
    max_steps function evaluations; history, if a list, receives (b, c, f(b), f(c)) at
    every step."""
    eps = float(np.finfo(float).eps)
    fa, fb = f(a), f(b)
    c, fc = a, fa
    d = e = b - a
    for _ in range(max_steps):
        if (fb > 0) == (fc > 0):
            # the bracket is [a, b]: restart from the old iterate
            c, fc = a, fa
            d = e = b - a
        if abs(fc) < abs(fb):
            # b must be the end with the smaller residual
            a, fa = b, fb
            b, fb = c, fc
            c, fc = a, fa
        tol = 2.0 * eps * abs(b)
        m = 0.5 * (c - b)
        if history is not None:
            history.append((b, c, fb, fc))
        if abs(m) <= tol or fb == 0.0:
            return b
        if abs(e) >= tol and abs(fa) > abs(fb):
            s = fb / fa
            if a == c:
                p, q = 2.0 * m * s, 1.0 - s
            else:
                qa, r = fa / fc, fb / fc
                p = s * (2.0 * m * qa * (qa - r) - (b - a) * (r - 1.0))
                q = (qa - 1.0) * (r - 1.0) * (s - 1.0)
            if p > 0:
                q = -q
            p = abs(p)
            if 2.0 * p < min(3.0 * m * q - abs(tol * q), abs(e * q)):
                e, d = d, p / q
            else:
                d = e = m
        else:
            d = e = m
        a, fa = b, fb
        b += d if abs(d) > tol else (tol if m > 0 else -tol)
        fb = f(b)
    return b


def tm_brent_fixed(U, st, max_steps):
    """The TM iterative solver with at most max_steps Brent steps (the recovery study)."""
    ok, D, S, tau, Smag, nhat, xi, t = _prep(U, st)
    eta = 1.0 + t
    c1, c2, c3 = _tm_coeffs(xi, eta)
    c1n, c2n, c3n = (v.detach().reshape(-1).numpy() for v in (c1, c2, c3))
    okn = ok.reshape(-1).numpy()
    Wn = np.zeros_like(c1n)
    for k in range(Wn.size):
        if not okn[k] or c3n[k] == 0.0:
            continue
        f = (lambda W, a=c1n[k], b=c2n[k], cc=c3n[k]: ((W + a) * W + b) * W + cc)
        hi = 200.0 ** 2 - 1.0
        while f(hi) < 0:
            hi *= 4.0
        Wn[k] = brent_steps(f, 0.0, hi, max_steps)
    W = torch.from_numpy(Wn).reshape(xi.shape)
    status = torch.where(ok, torch.zeros_like(xi, dtype=torch.int32),
                         torch.full_like(xi, ST_INADMISSIBLE, dtype=torch.int32))
    return _tm_recover(ok, D, tau, Smag, nhat, W, st, status)


def con2prim(U, st, method=None):
    """U [nvar, ...] -> (W [nvar, ...], status int32 [...])."""
    m = st.c2p if method is None else method
    if m < 0:
        m = NEWTON if st.eos == IDEAL else CUBIC
    fixed = getattr(st, "c2p_iters", 0)
    if st.eos == IDEAL and m == NEWTON and fixed > 0:
        # exactly `fixed` Newton steps from w = 1/2 (a negative tolerance never stops the
        # iteration).  Reading: the paper's study does not give its start; the middle of
        # (0, 1), from which it says any start converges, reproduces the pattern it
        # describes (6 steps near machine precision below gamma 10, 12 for all gamma).
        W, status = ideal_newton(U, st, tol=-1.0, max_iter=fixed, w_start=0.5)
        return W, torch.where(status == ST_NOCONV, torch.zeros_like(status), status)
    if st.eos == TM and m == BRENT and fixed > 0:
        return tm_brent_fixed(U, st, fixed)
    if st.eos == IDEAL and m == NEWTON:
        return ideal_newton(U, st)
    if st.eos == IDEAL and m == QUARTIC:
        return ideal_quartic(U, st)
    if st.eos == TM and m in (CUBIC, NEWTON):
        # Newton on the TM cubic (Sec. 3) converges to the same root the analytic
        # formula gives; the defined result is that root
        return tm_cubic(U, st)
    if st.eos == TM and m == BRENT:
        return tm_brent(U, st)
    raise ValueError(f"solver {m} does not apply to eos {st.eos}")


def bisect_beta(U, st, iters=200):
    """Brute force: bisection on beta in [0, 1) of the defining relation.

    For a trial beta the primitives follow from D and |M| alone
    (rho = D sqrt(1-beta^2), rho h = |M| c / (gamma^2 beta) from
    M = gamma^2 rho h v / c^2), and the residual is E(beta) - E.  Used only by
    the tests, scalar Python, any EOS."""
    from .eos import enthalpy
    c = st.c
    Dv = float(U[0]); Sv = math.sqrt(float((U[1:-1] ** 2).sum())); tv = float(U[-1])
    E = tv + Dv * c * c

    def resid(beta):
        g = 1.0 / math.sqrt(1.0 - beta * beta)
        rho = Dv / g
        rhoh = Sv * c / (g * g * beta)
        # solve h(Theta) c^2-scaled relation rho h(P/rho) = rhoh for P by bisection
        lo, hi = 0.0, rhoh
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            val = rho * float(enthalpy(torch.tensor(mid / rho, dtype=torch.float64),
                                       st.eos, st.gamma_ad, c))
            if val < rhoh:
                lo = mid
            else:
                hi = mid
        P = 0.5 * (lo + hi)
        return g * g * rhoh - P - E

    lo, hi = 1e-300, 1.0 - 1e-16
    flo = resid(lo) if Sv > 0 else 0.0
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        fm = resid(mid)
        if (fm > 0) == (flo > 0):
            lo, flo = mid, fm
        else:
            hi = mid
    return 0.5 * (lo + hi)
