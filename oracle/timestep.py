"""Third-order SSP Runge-Kutta step (Sec. 2.3, the Shu-Osher form).  Test infrastructure.

U1   = Pi(U + dt L(U))
U2   = Pi(3/4 U + 1/4 (U1 + dt L(U1)))
U^+  = Pi(1/3 U + 2/3 (U2 + dt L(U2)))
with L the DG right-hand side and Pi the physicality-enforcing operator.
Reading: the paper does not place the operator; it is applied after every
stage, so each stage stays a convex combination of admissible forward-Euler
states.  The step is fixed: dt = 0.1/(2p+1) min_d dx_d / c.

With Setup.limiter the slope limiter (oracle/limiter.py) acts on every stage
output before the operator: Pi(Lim(.)).

Lower orders (the paper pairs basis orders 0, 1, 2 with RK1, SSPRK2, SSPRK3 in
its convergence and performance runs, Sec. 2.3 citing the Shu-Osher schemes):
RK1 is forward Euler, U^+ = Pi(U + dt L(U)); SSPRK2 is
U1 = Pi(U + dt L(U)), U^+ = Pi(1/2 U + 1/2 (U1 + dt L(U1))).

Pinned by tests/test_oracle_timestep.py: one step of each scheme on a linear
ODE equals the Taylor polynomial of its order; the observed order on a
nonlinear ODE; and the full scheme's convergence on the exact translated
density wave (p = 2 with SSPRK3; p = 0 with RK1 and p = 1 with SSPRK2).
"""
from __future__ import annotations

from . import dg, limiter, physicality


def ssprk3(U, dt, L, P=lambda v: v):
    U1 = P(U + dt * L(U))
    U2 = P(0.75 * U + 0.25 * (U1 + dt * L(U1)))
    return P(U / 3.0 + (2.0 / 3.0) * (U2 + dt * L(U2)))


def rk1(U, dt, L, P=lambda v: v):
    return P(U + dt * L(U))


def ssprk2(U, dt, L, P=lambda v: v):
    U1 = P(U + dt * L(U))
    return P(0.5 * U + 0.5 * (U1 + dt * L(U1)))


SCHEMES = {1: rk1, 2: ssprk2, 3: ssprk3}


def step(U, dt, st, phys=True, stats=None, order=3):
    L = lambda V: dg.rhs(V, st, stats)  # noqa: E731
    scheme = SCHEMES[order]
    lim = (lambda V: limiter.limit(V, st, stats)) if getattr(st, "limiter", 0) else (lambda V: V)
    if phys:
        return scheme(U, dt, L, lambda V: physicality.enforce(lim(V), st, stats))
    return scheme(U, dt, L, lim)


def run(U, dt, nsteps, st, phys=True, stats=None, order=3):
    for _ in range(nsteps):
        U = step(U, dt, st, phys, stats, order)
    return U
