"""Pin of the oracle's full scheme on acoustic waves: a small-amplitude sound wave of
the equations linearised about rest (the paper's linear-wave tests, Sec. 4) returns
to its initial state after one period; the error converges at order p + 1 with the
paper's basis/integrator pairings.  The density-wave pin (uniform v and P) does not
exercise the pressure-velocity coupling this one does."""
import math

import pytest
import torch

from oracle import basis, srhd, timestep
from oracle.setup import Setup
from paper_2205_00095_amd import workloads as wl


def _period_error(N, p, order, dim=1):
    cfg = wl.make_config("sound", dim=dim, p=p, n_elem=tuple([N] * dim + [1] * (3 - dim)))
    st = Setup.from_config(cfg)
    conv = lambda a: torch.tensor(a)  # noqa: E731
    U0 = srhd.prim3_to_cons(*(conv(a) for a in wl.initial_primitives(cfg)), st)
    U0 = U0.reshape((st.nvar,) + wl.field_shape(cfg))
    T = wl.sound_period(cfg)
    n = int(math.ceil(T / cfg["dt"]))
    U = timestep.run(U0, T / n, n, st, order=order)
    w = torch.tensor(basis.tables(p)["w"])
    wt = w
    for _ in range(dim - 1):
        wt = wt[..., None] * w
    return float(((U[0] - U0[0]).abs() * wt).sum()) / (2 * N) ** dim


@pytest.mark.parametrize("p,order,Ns,lo", [(1, 2, (16, 32), 1.9), (2, 3, (8, 16), 2.8)])
def test_sound_wave_converges_at_order_p_plus_1(p, order, Ns, lo):
    e = [_period_error(N, p, order) for N in Ns]
    rate = math.log2(e[0] / e[1])
    assert rate > lo, (e, rate)


def test_sound_wave_eigenvector_is_a_linear_mode():
    """The generator's perturbation satisfies the linearised equations: the RHS of the
    oracle at t = 0 equals -d/dt of the exact linear solution (central difference in t)
    to discretisation accuracy on a fine 1D mesh."""
    from oracle import dg
    cfg = wl.make_config("sound", dim=1, p=3, n_elem=(32, 1, 1))
    st = Setup.from_config(cfg)
    conv = lambda a: torch.tensor(a)  # noqa: E731
    U = lambda t: srhd.prim3_to_cons(*(conv(a) for a in wl.sound_primitives(cfg, t=t)), st).reshape(  # noqa: E731
        (st.nvar,) + wl.field_shape(cfg))
    h = 1e-3
    dUdt = (U(h) - U(-h)) / (2 * h)
    R = dg.rhs(U(0.0), st)
    rel = float((R - dUdt).abs().max() / dUdt.abs().max())
    assert rel < 1e-4, rel
