"""Pin of the oracle's shock capturing on the paper's reflecting-wall Riemann problem
(Sec. 4, its fifth 1D problem; state from tests/golden/riemann_problems_1d.txt), run as
two mirror streams meeting at x = 1 of [0, 2] with first-order basis (p = 0, RK1): the
stopped gas behind the reflected shock has the density and pressure the
Rankine-Hugoniot conditions give, and the shock sits where their shock speed puts it."""
import numpy as np
import pytest
import torch

from oracle import srhd, timestep
from oracle.con2prim import con2prim
from oracle.setup import HLL, HLLC, IDEAL, OUTFLOW, Setup

from ._exact import jump_state as _jump_state
from ._exact import paper_wall_problem as _paper_wall_problem


@pytest.mark.parametrize("flux,rho_tol", [(HLL, 1e-2), (HLLC, 1e-3)])
def test_paper_wall_problem_matches_the_jump_conditions(flux, rho_tol):
    c = _paper_wall_problem()
    V, rho2, P2, D1 = _jump_state(c["gam"], c["v"], c["rho"], c["P"])
    N = 100
    st = Setup(dim=1, p=0, n_elem=(N, 1, 1), lo=(0.0, 0.0, 0.0), hi=(2.0, 1.0, 1.0), bc=(OUTFLOW,) * 3,
               eos=IDEAL, gamma_ad=c["gam"], flux=flux)
    x = 2.0 * (np.arange(N) + 0.5) / N
    sh = (1, 1, N, 1, 1, 1)
    U = srhd.prim3_to_cons(torch.full(sh, c["rho"]), torch.tensor(np.where(x < 1.0, c["v"], -c["v"]).reshape((1,) + sh)),
                           torch.full(sh, c["P"]), st)
    dt = 0.1 * 2.0 / N
    n = int(round(c["t"] / dt))
    stats = {}
    U = timestep.run(U, dt, n, st, order=1, stats=stats)
    assert stats.get("c2p_fail", 0) == 0
    W, _ = con2prim(U, st)
    rho, P, D = W[0].reshape(-1).numpy(), W[-1].reshape(-1).numpy(), U[0].reshape(-1).numpy()
    xs = 1.0 + V * n * dt
    L = 1.0 - xs
    plateau = (x > xs + 0.2 * L) & (x < 1.0 - 0.2 * L)
    assert abs(rho[plateau].mean() / rho2 - 1.0) <= rho_tol
    assert abs(P[plateau].mean() / P2 - 1.0) <= 1e-3
    shock = x[np.where((x < 1.0) & (D > 0.5 * (D1 + rho2)))[0].min()]
    assert abs(shock - xs) <= 2.0 * 2.0 / N


@pytest.mark.parametrize("flux,rho_tol", [(HLL, 1e-2), (HLLC, 1e-3)])
def test_paper_wall_problem_as_specified(flux, rho_tol):
    """The same problem as the paper states it: [0, 1] with the inflow state fixed at
    x = 0 and a reflecting wall at x = 1."""
    from oracle.setup import DIRICHLET, REFLECT
    c = _paper_wall_problem()
    V, rho2, P2, D1 = _jump_state(c["gam"], c["v"], c["rho"], c["P"])
    N = 50
    st = Setup(dim=1, p=0, n_elem=(N, 1, 1), bc=(DIRICHLET, 0, 0), bc_hi=(REFLECT, 0, 0), eos=IDEAL,
               gamma_ad=c["gam"], flux=flux, bc_state={(0, 0): (c["rho"], c["v"], 0.0, 0.0, c["P"])})
    x = (np.arange(N) + 0.5) / N
    sh = (1, 1, N, 1, 1, 1)
    U = srhd.prim3_to_cons(torch.full(sh, c["rho"]), torch.full((1,) + sh, c["v"]), torch.full(sh, c["P"]), st)
    dt = 0.1 / N
    n = int(round(c["t"] / dt))
    stats = {}
    U = timestep.run(U, dt, n, st, order=1, stats=stats)
    assert stats.get("c2p_fail", 0) == 0
    W, _ = con2prim(U, st)
    rho, P, D = W[0].reshape(-1).numpy(), W[-1].reshape(-1).numpy(), U[0].reshape(-1).numpy()
    xs = 1.0 + V * n * dt
    L = 1.0 - xs
    plateau = (x > xs + 0.2 * L) & (x < 1.0 - 0.2 * L)
    assert abs(rho[plateau].mean() / rho2 - 1.0) <= rho_tol
    assert abs(P[plateau].mean() / P2 - 1.0) <= 1e-3
    shock = x[np.where(D > 0.5 * (D1 + rho2))[0].min()]
    assert abs(shock - xs) <= 2.0 / N
