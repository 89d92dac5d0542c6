"""Exact reference values the shock tests compare with (no code shared with either
implementation): the Rankine-Hugoniot state behind a shock that stops a stream, and
the paper's wall problem read from its golden file."""
import math

from scipy.optimize import brentq


def jump_state(gam, v1, rho1, p1):
    """(velocity V < 0 of the left shock, rho2, P2 of the gas at rest behind it, D1) for
    a cold-to-warm stream v1 > 0 stopped by a wall (or its mirror stream)."""
    W1 = 1.0 / math.sqrt(1.0 - v1 * v1)
    h1 = 1.0 + gam / (gam - 1.0) * p1 / rho1
    D1, S1 = W1 * rho1, rho1 * h1 * W1 * W1 * v1
    E1 = rho1 * h1 * W1 * W1 - p1
    FD, FS, FE = D1 * v1, S1 * v1 + p1, (E1 + p1) * v1

    def state(V):  # mass and momentum jumps with v2 = 0
        return (D1 * V - FD) / V, FS - V * S1

    def energy(V):
        rho2, P2 = state(V)
        return E1 - FE / V - (rho2 + P2 / (gam - 1.0))

    V = brentq(energy, -0.999999, -1e-12, xtol=1e-15)
    return (V,) + state(V) + (D1,)


def paper_wall_problem():
    """The paper's fifth 1D Riemann problem (tests/golden/riemann_problems_1d.txt)."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "riemann_problems_1d.txt")
    with open(path) as fh:
        rows = [ln.split() for ln in fh if ln.strip() and not ln.startswith("#")]
    r = [float(v) for v in rows[4][1:]]
    assert int(rows[4][0]) == 5 and r[0:4] == r[4:8]  # uniform start
    return {"rho": r[0], "v": r[1], "P": r[3], "gam": r[8], "t": r[9]}
