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


# ---------------------------------------------------------------------------------
# The same with a transverse velocity v_t (Pons, Marti & Mueller 2000): across every
# wave but the contact h W v_t is constant; in a rarefaction
#   dv_x/dp = +- 1 / (rho h W^2 c_s sqrt(1 + g)),  g = v_t^2 (xi^2 - 1) / (1 - xi v_x)^2,
# xi the characteristic speed, integrated numerically.  The tests check the jump
# conditions of all four conserved components across the shocks and the self-similar
# equation F' = xi U' inside the fans.

def _char_speed(vx, vt, c, sign):
    v2 = vx * vx + vt * vt
    root = c * math.sqrt((1.0 - v2) * (1.0 - v2 * c * c - vx * vx * (1.0 - c * c)))
    return (vx * (1.0 - c * c) + sign * root) / (1.0 - v2 * c * c)


def _vt_of(A, h, vx):
    W = math.sqrt((1.0 + A * A / (h * h)) / (1.0 - vx * vx))
    return A / (h * W)


def _side_t(state, p, gam, sign):
    """(v_x, v_t, rho) reached from state = (rho, v_x, v_t, p) at pressure p."""
    rho_a, vx_a, vt_a, p_a = state
    h_a = _h(rho_a, p_a, gam)
    W_a = 1.0 / math.sqrt(1.0 - vx_a * vx_a - vt_a * vt_a)
    A = h_a * W_a * vt_a
    if p > p_a:  # shock
        k = (gam - 1.0) / (gam * p)

        def taub(hb):
            return hb * hb - h_a * h_a - (hb * (hb - 1.0) * k + h_a / rho_a) * (p - p_a)

        hi = 2.0
        while taub(hi) < 0.0:
            hi *= 2.0
        h_b = brentq(taub, 1.0 + 1e-15, hi, xtol=1e-15, rtol=1e-15)
        rho_b = gam * p / ((gam - 1.0) * (h_b - 1.0))
        j2 = -(p - p_a) / (h_b / rho_b - h_a / rho_a)
        D2 = rho_a * rho_a * W_a * W_a
        Vs = (D2 * vx_a + sign * math.sqrt(j2) * math.sqrt(j2 + D2 * (1.0 - vx_a * vx_a))) / (D2 + j2)
        j = sign * math.sqrt(j2)
        Ws = 1.0 / math.sqrt(1.0 - Vs * Vs)
        vx_b = (h_a * W_a * vx_a + Ws * (p - p_a) / j) / (h_a * W_a + (p - p_a) * (Ws * vx_a / j + 1.0 / (rho_a * W_a)))
        return vx_b, _vt_of(A, h_b, vx_b), rho_b
    from scipy.integrate import solve_ivp

    def rhs(q, y):
        vx = y[0]
        r = rho_a * (q / p_a) ** (1.0 / gam)
        h = _h(r, q, gam)
        c = _cs(r, q, gam)
        vt = _vt_of(A, h, vx)
        W2 = 1.0 / (1.0 - vx * vx - vt * vt)
        xi = _char_speed(vx, vt, c, sign)
        g = vt * vt * (xi * xi - 1.0) / (1.0 - xi * vx) ** 2
        return [sign * 1.0 / (r * h * W2 * c * math.sqrt(1.0 + g))]

    if p == p_a:
        return vx_a, vt_a, rho_a
    sol = solve_ivp(rhs, (p_a, p), [vx_a], rtol=1e-12, atol=1e-14, method="DOP853")
    vx = float(sol.y[0, -1])
    rho = rho_a * (p / p_a) ** (1.0 / gam)
    return vx, _vt_of(A, _h(rho, p, gam), vx), rho


def riemann_exact_t(left, right, gam):
    """Star states and a sampler xi -> (rho, v_x, v_t, p) for left/right = (rho, v_x, v_t, p).
    The left wave uses sign -1 (its characteristic xi_-), the right one +1."""
    def gap(p):
        try:
            return _side_t(left, p, gam, -1)[0] - _side_t(right, p, gam, +1)[0]
        except ValueError:  # a rarefaction towards vacuum leaves the physical range: gap > 0 there
            return 1.0

    lo, hi = 1e-6 * min(left[3], right[3]), 10.0 * max(left[3], right[3])
    while gap(hi) > 0.0:
        hi *= 10.0
    ps = brentq(gap, lo, hi, xtol=1e-300, rtol=1e-14)
    vxs, vtL, rhoL = _side_t(left, ps, gam, -1)
    _, vtR, rhoR = _side_t(right, ps, gam, +1)

    def wave_speeds(state, vt_s, rho_s, sign):
        rho_a, vx_a, vt_a, p_a = state
        if ps > p_a:
            h_a = _h(rho_a, p_a, gam)
            W_a = 1.0 / math.sqrt(1.0 - vx_a * vx_a - vt_a * vt_a)
            h_b = _h(rho_s, ps, gam)
            j2 = -(ps - p_a) / (h_b / rho_s - h_a / rho_a)
            D2 = rho_a * rho_a * W_a * W_a
            Vs = (D2 * vx_a + sign * math.sqrt(j2) * math.sqrt(j2 + D2 * (1.0 - vx_a * vx_a))) / (D2 + j2)
            return Vs, Vs
        return (_char_speed(vx_a, vt_a, _cs(rho_a, p_a, gam), sign),
                _char_speed(vxs, vt_s, _cs(rho_s, ps, gam), sign))

    lh, lt = wave_speeds(left, vtL, rhoL, -1)
    rh, rt = wave_speeds(right, vtR, rhoR, +1)
    tables = {}

    def fan_table(state, sign, n=1500):
        import numpy as np
        rows = []
        for q in np.geomspace(state[3], ps, n):
            vx, vt, rho = _side_t(state, q, gam, sign)
            rows.append((_char_speed(vx, vt, _cs(rho, q, gam), sign), rho, vx, vt, q))
        return np.array(sorted(rows))

    def profile(xi):
        import numpy as np
        xi = np.asarray(xi, dtype=float)
        out = np.empty((4,) + xi.shape)
        for m, val in [(xi < lh, left), ((xi >= lt) & (xi < vxs), (rhoL, vxs, vtL, ps)),
                       ((xi >= vxs) & (xi < rt), (rhoR, vxs, vtR, ps)), (xi >= rh, right)]:
            for q in range(4):
                out[q][m] = val[q]
        for sign, state, a, b in ((-1, left, lh, lt), (+1, right, rt, rh)):
            m = (xi >= a) & (xi < b)
            if ps < state[3] and m.any():
                if sign not in tables:
                    tables[sign] = fan_table(state, sign)
                tab = tables[sign]
                for q in range(4):
                    out[q][m] = np.interp(xi[m], tab[:, 0], tab[:, 1 + q])
        return out

    def sample(xi):
        """(rho, v_x, v_t, p) at one xi, fans solved pointwise (slow; for checks)."""
        for sign, state, a, b in ((-1, left, lh, lt), (+1, right, rt, rh)):
            if ps < state[3] and min(a, b) <= xi <= max(a, b):
                def f(q):
                    vx, vt, rho = _side_t(state, q, gam, sign)
                    return _char_speed(vx, vt, _cs(rho, q, gam), sign) - xi

                q = brentq(f, min(ps, state[3]), max(ps, state[3]), xtol=1e-300, rtol=1e-13)
                vx, vt, rho = _side_t(state, q, gam, sign)
                return rho, vx, vt, q
        return tuple(float(v) for v in profile(np.array([xi]))[:, 0])

    import numpy as np
    return {"p_star": ps, "vx_star": vxs, "left": (rhoL, vtL), "right": (rhoR, vtR),
            "left_speeds": (lh, lt), "right_speeds": (rt, rh), "profile": profile, "sample": sample}
