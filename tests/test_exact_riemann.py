"""Checks of the exact Riemann solution the shock tests use (tests/_exact.py), on the
paper's 1D Riemann problems without transverse velocity (Sec. 4; states from
tests/golden/riemann_problems_1d.txt), and the oracle's p = 0 scheme converging to it.

The exact solution is pinned by what defines it: the three relativistic jump
conditions across every shock, continuity of pressure and velocity across the
contact, and rarefaction fans whose edges move with the characteristic speeds of the
states they join."""
import math

import numpy as np
import pytest
import torch

from oracle import srhd, timestep
from oracle.setup import HLLC, IDEAL, OUTFLOW, Setup

from ._exact import riemann_exact, riemann_problem


def _cons_flux(rho, v, p, gam):
    h = 1.0 + gam / (gam - 1.0) * p / rho
    W = 1.0 / math.sqrt(1.0 - v * v)
    D, S, E = rho * W, rho * h * W * W * v, rho * h * W * W - p
    return np.array([D, S, E]), np.array([D * v, S * v + p, (E + p) * v])


@pytest.mark.parametrize("prob", [1, 2, 4])
def test_exact_solution_is_consistent(prob):
    L, R, gam, t, vy = riemann_problem(prob)
    assert vy == (0.0, 0.0)
    s = riemann_exact(L, R, gam)
    ps, vs = s["p_star"], s["v_star"]
    # shocks: [F] = V [U] for mass, momentum and energy
    for sign, state, rho_s, (a, b) in ((-1, L, s["rho_L_star"], s["left_speeds"]),
                                       (+1, R, s["rho_R_star"], s["right_speeds"])):
        if ps > state[2]:
            assert a == b
            U0, F0 = _cons_flux(*state, gam)
            U1, F1 = _cons_flux(rho_s, vs, ps, gam)
            res = np.abs((F1 - F0) - a * (U1 - U0)) / (np.abs(F1) + np.abs(F0) + np.abs(U1) + np.abs(U0))
            assert float(res.max()) < 1e-12, (prob, sign, res)
        else:  # rarefaction: head and tail at the characteristic speeds, isentropic star state
            head, tail = (a, b) if sign < 0 else (b, a)
            for (rho, v, p), speed in ((state, head), ((rho_s, vs, ps), tail)):
                c = math.sqrt(gam * p / (rho * (1.0 + gam / (gam - 1.0) * p / rho)))
                assert abs((v + sign * c) / (1.0 + sign * v * c) - speed) < 1e-12
            assert abs(ps / rho_s ** gam - state[2] / state[0] ** gam) <= 1e-12 * state[2] / state[0] ** gam
    # the sampled profile: the initial states outside the fan, p and v continuous at the contact
    xi = np.array([-0.999, vs - 1e-9, vs + 1e-9, 0.999])
    prof = s["profile"](xi)
    assert np.allclose(prof[:, 0], L) and np.allclose(prof[:, -1], R)
    assert abs(prof[1, 1] - prof[1, 2]) < 1e-12 and abs(prof[2, 1] - prof[2, 2]) < 1e-12 * ps


def _l1_D(prob, N):
    L, R, gam, t, _ = riemann_problem(prob)
    st = Setup(dim=1, p=0, n_elem=(N, 1, 1), bc=(OUTFLOW,) * 3, eos=IDEAL, gamma_ad=gam, flux=HLLC)
    x = (np.arange(N) + 0.5) / N
    sh = (1, 1, N, 1, 1, 1)
    pick = lambda a, b: torch.tensor(np.where(x < 0.5, a, b).reshape(sh))  # noqa: E731
    U = srhd.prim3_to_cons(pick(L[0], R[0]), pick(L[1], R[1])[None], pick(L[2], R[2]), st)
    dt = 0.1 / N
    n = int(round(t / dt))
    U = timestep.run(U, dt, n, st, order=1)
    sub = (np.arange(N)[:, None] + (np.arange(16)[None, :] + 0.5) / 16) / N
    rho, v, _ = riemann_exact(L, R, gam)["profile"]((sub - 0.5) / (n * dt))
    De = (rho / np.sqrt(1.0 - v * v)).mean(1)
    return float(np.abs(U[0].reshape(-1).numpy() - De).mean())


@pytest.mark.parametrize("prob,rate", [(1, 0.4), (4, 0.4)])
def test_oracle_first_order_converges_to_the_exact_solution(prob, rate):
    """p = 0 with HLLC and RK1: the L1 error of D falls with the mesh width (at the
    reduced rate discontinuities allow)."""
    e1, e2 = _l1_D(prob, 100), _l1_D(prob, 200)
    assert math.log2(e1 / e2) > rate, (e1, e2)


def _cons_flux_t(rho, vx, vt, p, gam):
    h = 1.0 + gam / (gam - 1.0) * p / rho
    W = 1.0 / math.sqrt(1.0 - vx * vx - vt * vt)
    D, Sx, St, E = rho * W, rho * h * W * W * vx, rho * h * W * W * vt, rho * h * W * W - p
    return np.array([D, Sx, St, E]), np.array([D * vx, Sx * vx + p, St * vx, (E + p) * vx])


@pytest.mark.parametrize("prob", [1, 3, 4])
def test_exact_solution_with_transverse_velocity_is_consistent(prob):
    """The general solution (transverse velocity allowed): it reproduces the solution
    without transverse velocity where there is none, its shocks satisfy the jump
    conditions of all four conserved components, and inside its fans the self-similar
    equation dF/dxi = xi dU/dxi holds (checked by central differences)."""
    from ._exact import riemann_exact_t
    L, R, gam, t, vy = riemann_problem(prob)
    left, right = (L[0], L[1], vy[0], L[2]), (R[0], R[1], vy[1], R[2])
    s = riemann_exact_t(left, right, gam)
    if vy == (0.0, 0.0):
        s0 = riemann_exact(L, R, gam)
        assert abs(s["p_star"] / s0["p_star"] - 1.0) < 1e-10 and abs(s["vx_star"] - s0["v_star"]) < 1e-10
    ps, vxs = s["p_star"], s["vx_star"]
    for sign, state, (rho_s, vt_s), (a, b) in ((-1, left, s["left"], s["left_speeds"]),
                                                (+1, right, s["right"], s["right_speeds"])):
        if ps > state[3]:  # shock
            U0, F0 = _cons_flux_t(*state, gam)
            U1, F1 = _cons_flux_t(rho_s, vxs, vt_s, ps, gam)
            res = np.abs((F1 - F0) - a * (U1 - U0)) / (np.abs(F1) + np.abs(F0) + np.abs(U1) + np.abs(U0) + 1e-300)
            assert float(res.max()) < 1e-10, (prob, sign, res)
        else:  # fan: F' = xi U' at interior points
            lo_, hi_ = min(a, b), max(a, b)
            for xi in np.linspace(lo_, hi_, 7)[2:-2]:
                e = 1e-4 * (hi_ - lo_)
                Um, Fm = _cons_flux_t(*s["sample"](xi - e), gam)
                Up, Fp = _cons_flux_t(*s["sample"](xi + e), gam)
                dU, dF = (Up - Um) / (2 * e), (Fp - Fm) / (2 * e)
                scale = np.abs(dF).max() + abs(xi) * np.abs(dU).max()
                assert float(np.abs(dF - xi * dU).max()) < 1e-6 * scale, (prob, xi, dF, xi * dU)


def test_transverse_rarefaction_is_self_similar():
    """A rarefaction carrying transverse velocity (the term the paper's problems do not
    exercise on their fan side): F' = xi U' inside it, and h W v_t constant across it."""
    from ._exact import riemann_exact_t
    gam = 5.0 / 3.0
    left, right = (1.0, 0.1, 0.5, 10.0), (1.0, 0.0, -0.3, 0.1)
    s = riemann_exact_t(left, right, gam)
    a, b = s["left_speeds"]
    assert s["p_star"] < left[3] and b > a
    h = lambda r, p: 1.0 + gam / (gam - 1.0) * p / r  # noqa: E731
    A0 = h(left[0], left[3]) * left[2] / math.sqrt(1.0 - left[1] ** 2 - left[2] ** 2)
    for xi in np.linspace(a, b, 7)[1:-1]:
        e = 1e-4 * (b - a)
        Um, Fm = _cons_flux_t(*s["sample"](xi - e), gam)
        Up, Fp = _cons_flux_t(*s["sample"](xi + e), gam)
        dU, dF = (Up - Um) / (2 * e), (Fp - Fm) / (2 * e)
        assert float(np.abs(dF - xi * dU).max()) < 1e-6 * (np.abs(dF).max() + abs(xi) * np.abs(dU).max())
        rho, vx, vt, p = s["sample"](xi)
        assert abs(h(rho, p) * vt / math.sqrt(1.0 - vx * vx - vt * vt) / A0 - 1.0) < 1e-9
