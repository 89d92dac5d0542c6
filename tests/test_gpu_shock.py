"""Shock capturing on the GPU against the exact jump conditions: two cold streams
colliding head-on at 0.9c (ideal gas Gamma = 4/3) stop at the symmetry plane - a
wall by symmetry, as in the paper's reflecting-wall Riemann test (Sec. 4) - behind
two shocks moving outwards.  The plateau state and the shock speed follow from the
Rankine-Hugoniot conditions of the three conservation laws with the ideal-gas EOS,
solved here directly (a definition, shared with neither implementation).  First-order
basis (p = 0, RK1): no limiter is needed, as in the paper's p = 0 shock runs."""
import math

import numpy as np
import pytest
import torch
from scipy.optimize import brentq

from paper_2205_00095_amd import workloads as wl

pytestmark = pytest.mark.gpu

GAM, V1, RHO1, P1 = 4.0 / 3.0, 0.9, 1.0, 1e-4  # c = 1


def _jump_state():
    """(shock velocity V < 0 of the left shock, rho2, P2) of the gas at rest behind it."""
    W1 = 1.0 / math.sqrt(1.0 - V1 * V1)
    h1 = 1.0 + GAM / (GAM - 1.0) * P1 / RHO1
    D1, S1 = W1 * RHO1, RHO1 * h1 * W1 * W1 * V1
    E1 = RHO1 * h1 * W1 * W1 - P1
    FD, FS, FE = D1 * V1, S1 * V1 + P1, (E1 + P1) * V1

    def state(V):  # mass and momentum jumps with v2 = 0
        return (D1 * V - FD) / V, FS - V * S1

    def energy(V):
        rho2, P2 = state(V)
        return E1 - FE / V - (rho2 + P2 / (GAM - 1.0))

    V = brentq(energy, -0.999999, -1e-9, xtol=1e-15)
    return (V,) + state(V), D1


@pytest.mark.parametrize("flux,rho_tol", [(wl.FLUX_HLL, 1e-2), (wl.FLUX_HLLC, 1e-3)])
def test_colliding_streams_match_the_jump_conditions(flux, rho_tol):
    from paper_2205_00095_amd.solver import Solver
    (V, rho2, P2), D1 = _jump_state()
    N, t = 400, 0.3
    cfg = wl.make_config("wave1d", n_elem=(N, 1, 1), p=0, bc=(wl.OUTFLOW,) * 3, gamma_ad=GAM)
    cfg["flux"] = flux
    print(f"case colliding streams N={N} flux {flux}: exact V {V:.6f} rho2 {rho2:.6f} P2 {P2:.6f}", flush=True)
    shape = wl.field_shape(cfg)
    x = (np.arange(N) + 0.5) / N
    rho = np.full(shape, RHO1)
    v = np.where(x < 0.5, V1, -V1).reshape((1,) + shape)
    P = np.full(shape, P1)
    s = Solver(cfg)
    U = s.set_state(torch.from_numpy(wl.pack_primitives(rho, v, P)).cuda())
    dt = 0.1 / N
    n = int(round(t / dt))
    s.run(U, dt, n, order=1)
    W = s.con2prim(U).cpu().reshape(3, -1).numpy()
    D = U[0].cpu().reshape(-1).numpy()
    d = s.diagnostics()
    assert d["c2p_fail"] == 0
    xs = 0.5 + V * n * dt
    L = 0.5 - xs
    plateau = (x > xs + 0.2 * L) & (x < 0.5 - 0.2 * L)
    rho_p, P_p = W[0][plateau].mean(), W[2][plateau].mean()
    shock = x[np.where((x < 0.5) & (D > 0.5 * (D1 + rho2)))[0].min()]
    print(f"plateau rho {rho_p:.6f} P {P_p:.6f}; shock at {shock:.5f} (exact {xs:.5f})", flush=True)
    assert abs(rho_p / rho2 - 1.0) <= rho_tol
    assert abs(P_p / P2 - 1.0) <= 1e-3
    assert abs(shock - xs) <= 2.0 / N
    # mirror symmetry about the collision plane
    assert np.allclose(D, D[::-1], rtol=1e-9, atol=0.0)
