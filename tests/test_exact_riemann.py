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
