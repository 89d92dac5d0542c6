"""Pins of the oracle's Kelvin-Helmholtz diagnostic J = integral of v_y^2 dA (Sec. 4,
the spatial mean of v_y^2 without the 1/|Omega| factor) against closed-form integrals.

The collocated Gauss-Legendre rule with p+1 points per direction integrates
polynomials of degree 2p+1 exactly, so a velocity field that is a polynomial of
degree <= p per element gives J to rounding; a dropped or doubled Jacobian factor
(dx_d / 2 in any direction), a wrong weight or a v_y taken as u_y (the 4-velocity)
changes these values by O(1)."""
import numpy as np
import pytest
import torch

from oracle import srhd
from oracle.objective import vy2_integral
from oracle.setup import IDEAL, OUTFLOW, PERIODIC, TM, Setup


def _node_coords(st):
    """Physical node coordinates per direction, broadcast to the nodal field shape."""
    shape = st.shape()
    xi, _ = np.polynomial.legendre.leggauss(st.p + 1)
    out = []
    for d in range(3):
        if d >= st.dim:
            out.append(np.zeros(shape))
            continue
        n = st.n_elem[d]
        dx = (st.hi[d] - st.lo[d]) / n
        pos = st.lo[d] + (np.arange(n)[:, None] + 0.5 * (xi[None] + 1.0)) * dx
        b = [1] * 6
        b[2 - d], b[5 - d] = pos.shape
        out.append(np.broadcast_to(pos.reshape(b), shape))
    return out


def _state(st, vx, vy, vz=None, rho=None, P=None):
    shape = st.shape()
    rho = np.full(shape, 1.3) if rho is None else rho
    P = np.full(shape, 0.7) if P is None else P
    comps = [np.broadcast_to(vx, shape), np.broadcast_to(vy, shape)]
    if st.dim == 3:
        comps.append(np.broadcast_to(np.zeros(shape) if vz is None else vz, shape))
    v = np.stack(comps)
    return srhd.prim3_to_cons(torch.tensor(rho), torch.tensor(v), torch.tensor(P), st)


KH_DOMAIN = dict(lo=(0.0, -1.0, 0.0), hi=(1.0, 1.0, 1.0), bc=(PERIODIC, OUTFLOW, PERIODIC))


@pytest.mark.parametrize("p,n,eos", [(3, (6, 5, 1), TM), (2, (4, 7, 1), IDEAL), (0, (9, 4, 1), TM)])
def test_uniform_vy_gives_vy2_times_area(p, n, eos):
    """A uniform v_y (with a uniform v_x beside it) on the Kelvin-Helmholtz domain
    [0,1] x [-1,1]: J = v_y^2 x area = 2 v_y^2, at any order and mesh."""
    st = Setup(dim=2, p=p, n_elem=n, eos=eos, **KH_DOMAIN)
    shape = st.shape()
    vy = 0.37
    U = _state(st, np.full(shape, -0.41), np.full(shape, vy))
    J = float(vy2_integral(U, st))
    assert abs(J - 2.0 * vy * vy) <= 1e-14 * 2.0 * vy * vy


def test_uniform_vy_3d_box():
    """The same in 3D on [0,2] x [-1,0.5] x [0,0.25] (volume 0.75)."""
    st = Setup(dim=3, p=2, n_elem=(3, 4, 2), lo=(0.0, -1.0, 0.0), hi=(2.0, 0.5, 0.25), eos=IDEAL)
    shape = st.shape()
    vy = -0.52
    U = _state(st, np.full(shape, 0.2), np.full(shape, vy), np.full(shape, 0.3))
    J = float(vy2_integral(U, st))
    assert abs(J - 0.75 * vy * vy) <= 1e-14 * 0.75 * vy * vy


@pytest.mark.parametrize("p", [1, 2, 3])
def test_separable_polynomial_field(p):
    """v_y = (a + b x)(c + e y) on [0,1] x [-1,1]: v_y^2 has degree 2 <= 2p + 1 in each
    direction, so the quadrature is exact and
    J = (a^2 + a b + b^2 / 3) (2 c^2 + 2 e^2 / 3)."""
    st = Setup(dim=2, p=p, n_elem=(5, 3, 1), eos=TM, **KH_DOMAIN)
    x, y, _ = _node_coords(st)
    a, b, c, e = 0.1, 0.2, 1.0, 0.5
    vy = (a + b * x) * (c + e * y)
    U = _state(st, 0.1 * np.ones_like(x), vy, rho=1.0 + 0.5 * x * x, P=0.5 + 0.25 * (y + 1.0))
    J = float(vy2_integral(U, st))
    exact = (a * a + a * b + b * b / 3.0) * (2.0 * c * c + 2.0 * e * e / 3.0)
    assert abs(J - exact) <= 1e-13 * exact


def test_sine_squared_field():
    """v_y = A sin(2 pi x) on [0,1] x [-1,1]: J = A^2 (the mean of sin^2 is 1/2, area 2).
    The field is not a polynomial; at p = 3 on 24 elements the composite rule is
    accurate to ~1e-13."""
    st = Setup(dim=2, p=3, n_elem=(24, 2, 1), eos=IDEAL, **KH_DOMAIN)
    x, y, _ = _node_coords(st)
    A = 0.3
    U = _state(st, np.zeros_like(x), A * np.sin(2 * np.pi * x))
    J = float(vy2_integral(U, st))
    assert abs(J - A * A) <= 1e-11 * A * A
