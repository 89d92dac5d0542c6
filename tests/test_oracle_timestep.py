"""Pins of the oracle's SSP-RK3 (Sec. 2.3) and the full scheme's convergence (Sec. 4)."""
import math

import numpy as np
import pytest
import torch

from oracle import srhd, timestep
from oracle.setup import Setup
from paper_2205_00095_amd import workloads as wl


def test_linear_ode_step_is_third_order_taylor():
    """For L(y) = lam y one SSP-RK3 step multiplies by 1 + z + z^2/2 + z^3/6, z = lam dt."""
    for z in (0.1, -0.37, 1.3):
        y = timestep.ssprk3(torch.tensor([1.0]), z, lambda v: v)
        assert abs(float(y) - (1 + z + z * z / 2 + z ** 3 / 6)) < 1e-15


def test_linear_ode_step_lower_orders_taylor():
    """RK1 and SSPRK2 multiply by 1 + z and 1 + z + z^2/2 on L(y) = lam y."""
    for z in (0.1, -0.37, 1.3):
        y1 = timestep.rk1(torch.tensor([1.0]), z, lambda v: v)
        y2 = timestep.ssprk2(torch.tensor([1.0]), z, lambda v: v)
        assert abs(float(y1) - (1 + z)) < 1e-15
        assert abs(float(y2) - (1 + z + z * z / 2)) < 1e-15


@pytest.mark.parametrize("order,lo", [(1, 0.95), (2, 1.9)])
def test_nonlinear_ode_lower_orders(order, lo):
    def L(Y):
        return torch.stack([-Y[0] ** 2 + torch.cos(Y[1]), torch.ones_like(Y[1])])

    def solve(n):
        Y = torch.tensor([1.0, 0.0])
        for _ in range(n):
            Y = timestep.SCHEMES[order](Y, 1.0 / n, L)
        return float(Y[0])

    ref = solve_ref(L)
    e = [abs(solve(n) - ref) for n in (64, 128, 256)]
    orders = [math.log2(e[i] / e[i + 1]) for i in range(2)]
    assert min(orders) > lo, orders


def solve_ref(L, n=8192):
    Y = torch.tensor([1.0, 0.0])
    for _ in range(n):
        Y = timestep.ssprk3(Y, 1.0 / n, L)
    return float(Y[0])


def test_nonlinear_ode_order_three():
    """y' = -y^2 + cos t folded into an autonomous system; order from three step sizes."""
    def L(Y):
        return torch.stack([-Y[0] ** 2 + torch.cos(Y[1]), torch.ones_like(Y[1])])

    def solve(n):
        Y = torch.tensor([1.0, 0.0])
        for _ in range(n):
            Y = timestep.ssprk3(Y, 1.0 / n, L)
        return float(Y[0])

    ref = solve(4096)
    e = [abs(solve(n) - ref) for n in (16, 32, 64)]
    orders = [math.log2(e[i] / e[i + 1]) for i in range(2)]
    assert min(orders) > 2.8


def _l1_density_error(N, p=2, order=3):
    cfg = wl.make_config("wave1d", n_elem=(N, 1, 1), p=p)
    st = Setup.from_config(cfg)
    conv = lambda a: torch.tensor(a)  # noqa: E731
    U = srhd.prim3_to_cons(*(conv(a) for a in wl.initial_primitives(cfg)), st)
    U = U.reshape((3,) + wl.field_shape(cfg))
    tfinal = 0.03125
    n = int(round(tfinal / cfg["dt"]))
    U = timestep.run(U, cfg["dt"], n, st, order=order)
    Ue = srhd.prim3_to_cons(*(conv(a) for a in wl.wave1d_primitives(cfg, t=n * cfg["dt"])), st)
    from oracle import basis
    w = torch.tensor(basis.tables(cfg["p"])["w"])
    return float((0.5 * st.dx(0) * w * (U[0] - Ue.reshape(U.shape)[0]).abs()).sum())


@pytest.mark.slow
def test_density_wave_converges_at_order_p_plus_1():
    """p = 2, SSP-RK3, exact translated solution; expected order 3 (paper Table: 2.56-3.10)."""
    errs = {N: _l1_density_error(N) for N in (16, 32, 64)}
    o1 = math.log2(errs[16] / errs[32])
    o2 = math.log2(errs[32] / errs[64])
    assert o2 > 2.8 and o1 > 2.5, (errs, o1, o2)


@pytest.mark.parametrize("p,order,Ns,lo", [(0, 1, (64, 128, 256), 0.98), (1, 2, (32, 64, 128), 1.9)])
def test_density_wave_lower_orders(p, order, Ns, lo):
    """The paper's pairings (p = 0, RK1) and (p = 1, SSPRK2) converge at orders 1 and 2."""
    errs = [_l1_density_error(N, p, order) for N in Ns]
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert min(orders) > lo, (errs, orders)
