"""Third-order SSP Runge-Kutta step (Sec. 2.3, the Shu-Osher form).  Test infrastructure.

U1   = Pi(U + dt L(U))
U2   = Pi(3/4 U + 1/4 (U1 + dt L(U1)))
U^+  = Pi(1/3 U + 2/3 (U2 + dt L(U2)))
with L the DG right-hand side and Pi the physicality-enforcing operator.
Reading: the paper does not place the operator; it is applied after every
stage, so each stage stays a convex combination of admissible forward-Euler
states.  The step is fixed: dt = 0.1/(2p+1) min_d dx_d / c.

Pinned by tests/test_oracle_timestep.py: third-order convergence in time on
a scalar ODE with a known solution, and (test_oracle_convergence.py) the
full scheme on the exact translated density wave.
"""
from __future__ import annotations

from . import dg, physicality


def ssprk3(U, dt, L, P=lambda v: v):
    U1 = P(U + dt * L(U))
    U2 = P(0.75 * U + 0.25 * (U1 + dt * L(U1)))
    return P(U / 3.0 + (2.0 / 3.0) * (U2 + dt * L(U2)))


def step(U, dt, st, phys=True, stats=None):
    L = lambda V: dg.rhs(V, st, stats)  # noqa: E731
    if phys:
        return ssprk3(U, dt, L, lambda V: physicality.enforce(V, st, stats))
    return ssprk3(U, dt, L)


def run(U, dt, nsteps, st, phys=True, stats=None):
    for _ in range(nsteps):
        U = step(U, dt, st, phys, stats)
    return U
