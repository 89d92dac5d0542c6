"""Pin of the oracle's FP64 reverse-mode gradient (autograd) against central finite differences.

The gradient of J = int v_y^2 dA after n SSP-RK3 steps with respect to the
per-node initial v_y perturbation, on a small Kelvin-Helmholtz mesh."""
import numpy as np
import torch

from oracle import objective, srhd, timestep
from oracle.setup import Setup
from paper_2205_00095_amd import workloads as wl


def _J(delta, cfg, st, nsteps):
    rho, v, P = (torch.tensor(a) for a in wl.initial_primitives(cfg))
    v = v.clone()
    v[1] = v[1] + delta
    U = srhd.prim3_to_cons(rho, v, P, st).reshape((st.nvar,) + wl.field_shape(cfg))
    U = timestep.run(U, cfg["dt"] * 20, nsteps, st)   # large step: visible dynamics in few steps
    return objective.vy2_integral(U, st)


def test_autograd_gradient_matches_central_differences():
    cfg = wl.make_config("kh_ideal", n_elem=(4, 4, 1))
    st = Setup.from_config(cfg)
    delta0 = torch.tensor(wl.kh_perturbation(cfg))
    d = delta0.clone().requires_grad_(True)
    J = _J(d, cfg, st, 3)
    (g,) = torch.autograd.grad(J, d)
    dirs = torch.tensor(wl.random_directions(cfg, 3))
    for k in range(3):
        h = 1e-6
        Jp = float(_J(delta0 + h * dirs[k], cfg, st, 3))
        Jm = float(_J(delta0 - h * dirs[k], cfg, st, 3))
        fd = (Jp - Jm) / (2 * h)
        ad = float((g * dirs[k]).sum())
        assert abs(fd - ad) <= 1e-6 * abs(ad), (fd, ad)
    assert float(g.abs().max()) > 0
