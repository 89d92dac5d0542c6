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


# ---------------------------------------------------------------------------------
# Exact solution of the 1D special-relativistic Riemann problem without transverse
# velocity, ideal gas, c = 1 (the construction of Marti & Mueller: a rarefaction or a
# shock on each side of a contact; the star pressure is where the two sides' star
# velocities agree).  Rarefactions integrate the characteristic relation
# d(atanh v) = -+ dp / (rho h c_s) along the isentrope numerically; shocks use the
# Taub adiabat and the relativistic jump conditions, and the tests check the jump
# conditions on the result.

def _h(rho, p, gam):
    return 1.0 + gam / (gam - 1.0) * p / rho


def _cs(rho, p, gam):
    return math.sqrt(gam * p / (rho * _h(rho, p, gam)))


def _rarefaction_dphi(rho_a, p_a, p, gam):
    """integral from p_a to p of dp' / (rho h c_s) along the isentrope through (rho_a, p_a)."""
    from scipy.integrate import quad

    def f(q):
        r = rho_a * (q / p_a) ** (1.0 / gam)
        return 1.0 / (r * _h(r, q, gam) * _cs(r, q, gam))

    import warnings
    from scipy.integrate import IntegrationWarning
    with warnings.catch_warnings():  # short intervals near p_a report roundoff, harmlessly
        warnings.simplefilter("ignore", IntegrationWarning)
        return quad(f, p_a, p, epsabs=0.0, epsrel=1e-11, limit=200)[0]


def _shock(rho_a, v_a, p_a, p_b, gam, sign):
    """Post-shock (rho_b, v_b) and shock speed for pre-shock state a and pressure p_b > p_a;
    sign = -1 for the left-facing shock, +1 for the right-facing one."""
    h_a = _h(rho_a, p_a, gam)
    k = (gam - 1.0) / (gam * p_b)

    def taub(hb):  # h_b^2 - h_a^2 - (h_b/rho_b + h_a/rho_a)(p_b - p_a), rho_b from the EOS
        return hb * hb - h_a * h_a - (hb * (hb - 1.0) * k + h_a / rho_a) * (p_b - p_a)

    hi = 2.0
    while taub(hi) < 0.0:
        hi *= 2.0
    h_b = brentq(taub, 1.0 + 1e-15, hi, xtol=1e-15, rtol=1e-15)
    rho_b = gam * p_b / ((gam - 1.0) * (h_b - 1.0))
    j2 = -(p_b - p_a) / (h_b / rho_b - h_a / rho_a)
    W_a = 1.0 / math.sqrt(1.0 - v_a * v_a)
    D2 = rho_a * rho_a * W_a * W_a
    Vs = (D2 * v_a + sign * math.sqrt(j2) * math.sqrt(j2 + D2 * (1.0 - v_a * v_a))) / (D2 + j2)
    # post-shock velocity (Marti & Mueller's expression with the signed mass flux
    # j = sign |j|); the tests check the three jump conditions on the result
    j = sign * math.sqrt(j2)
    Ws = 1.0 / math.sqrt(1.0 - Vs * Vs)
    v_b = (h_a * W_a * v_a + Ws * (p_b - p_a) / j) / (h_a * W_a + (p_b - p_a) * (Ws * v_a / j + 1.0 / (rho_a * W_a)))
    m = W_a * rho_a * (v_a - Vs)
    return rho_b, v_b, Vs, m


def _side(state, p, gam, sign):
    """Star velocity and density reached from `state` at pressure p by the wave on that side."""
    rho_a, v_a, p_a = state
    if p > p_a:
        rho_b, v_b, _, _ = _shock(rho_a, v_a, p_a, p, gam, sign)
        return v_b, rho_b
    phi = math.atanh(v_a) + sign * _rarefaction_dphi(rho_a, p_a, p, gam)
    return math.tanh(phi), rho_a * (p / p_a) ** (1.0 / gam)


def riemann_exact(left, right, gam):
    """Star pressure and velocity and a sampler xi = x/t -> (rho, v, p) for the states
    left = (rho, v, p) and right."""
    def gap(p):
        return _side(left, p, gam, -1)[0] - _side(right, p, gam, +1)[0]

    lo, hi = 1e-14 * max(left[2], right[2]), 10.0 * max(left[2], right[2])
    while gap(hi) > 0.0:
        hi *= 10.0
    ps = brentq(gap, lo, hi, xtol=1e-300, rtol=1e-15)
    vs, rhoL_s = _side(left, ps, gam, -1)
    _, rhoR_s = _side(right, ps, gam, +1)

    def fan(state, xi, sign):
        """State inside the rarefaction fan of `state` where the characteristic speed
        (v + sign c_s)/(1 + sign v c_s) equals xi."""
        rho_a, v_a, p_a = state

        def f(p):
            v, rho = _side(state, p, gam, sign)
            c = _cs(rho, p, gam)
            return (v + sign * c) / (1.0 + sign * v * c) - xi

        p = brentq(f, min(ps, p_a), max(ps, p_a), xtol=1e-300, rtol=1e-14)
        v, rho = _side(state, p, gam, sign)
        return rho, v, p

    def speeds(state, rho_s, sign):
        rho_a, v_a, p_a = state
        if ps > p_a:
            Vs = _shock(rho_a, v_a, p_a, ps, gam, sign)[2]
            return Vs, Vs
        ca, cs_ = _cs(rho_a, p_a, gam), _cs(rho_s, ps, gam)
        head = (v_a + sign * ca) / (1.0 + sign * v_a * ca)
        tail = (vs + sign * cs_) / (1.0 + sign * vs * cs_)
        return head, tail

    lh, lt = speeds(left, rhoL_s, -1)
    rh, rt = speeds(right, rhoR_s, +1)

    def fan_table(state, sign, n=3000):
        """(xi, rho, v, p) on a dense pressure grid through the fan, for interpolation."""
        import numpy as np
        pg = np.geomspace(state[2], ps, n)
        rows = []
        for q in pg:
            v, rho = _side(state, q, gam, sign)
            c = _cs(rho, q, gam)
            rows.append(((v + sign * c) / (1.0 + sign * v * c), rho, v, q))
        tab = np.array(sorted(rows))
        return tab

    tables = {}

    def profile(xi):
        """Vectorised sample over an array of xi (fans interpolated from a dense table)."""
        import numpy as np
        xi = np.asarray(xi, dtype=float)
        out = np.empty((3,) + xi.shape)
        regions = [(xi < lh, left), ((xi >= lt) & (xi < vs), (rhoL_s, vs, ps)),
                   ((xi >= vs) & (xi < rt), (rhoR_s, vs, ps)), (xi >= rh, right)]
        for m, val in regions:
            for q in range(3):
                out[q][m] = val[q]
        for sign, state, a, b in ((-1, left, lh, lt), (+1, right, rt, rh)):
            m = (xi >= a) & (xi < b)
            if ps < state[2] and m.any():  # a rarefaction on this side
                if sign not in tables:
                    tables[sign] = fan_table(state, sign)
                tab = tables[sign]
                for q in range(3):
                    out[q][m] = np.interp(xi[m], tab[:, 0], tab[:, 1 + q])
        return out

    def sample(xi):
        """(rho, v, p) at one xi = x/t (fans solved pointwise)."""
        if xi < vs:
            if xi <= lh:
                return tuple(left)
            if xi >= lt:
                return rhoL_s, vs, ps
            return fan(left, xi, -1)
        if xi >= rh:
            return tuple(right)
        if xi <= rt:
            return rhoR_s, vs, ps
        return fan(right, xi, +1)

    return {"p_star": ps, "v_star": vs, "rho_L_star": rhoL_s, "rho_R_star": rhoR_s,
            "left_speeds": (lh, lt), "right_speeds": (rt, rh), "sample": sample, "profile": profile}


def riemann_problem(i):
    """(left, right, Gamma, t_final) of the paper's 1D Riemann problem i (golden file)."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "riemann_problems_1d.txt")
    with open(path) as fh:
        rows = {int(ln.split()[0]): [float(v) for v in ln.split()[1:]]
                for ln in fh if ln.strip() and not ln.startswith("#")}
    r = rows[i]
    return (r[0], r[1], r[3]), (r[4], r[5], r[7]), r[8], r[9], (r[2], r[6])
