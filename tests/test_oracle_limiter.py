"""Pins of the oracle's slope limiter (reading R29 of the minmod limiter the paper names
for its p >= 1 shock runs): conservation, exactness on linear data, the cut-back of a
jump, the minmod bounds of each limited slope, idempotence, and the total variation
of the element averages over a limited forward-Euler step of a Riemann problem."""
import numpy as np
import pytest
import torch

from oracle import basis, limiter, srhd
from oracle import dg as odg
from oracle import physicality as ophys
from oracle.setup import HLLC, IDEAL, OUTFLOW, PERIODIC, Setup


def _averages(U, st):
    w = odg.elem_weights(st)
    return (U * w).sum((4, 5, 6)) / w.sum()


def _node_x(st, d=0):
    """Physical coordinate along d of every node, shaped like one component."""
    xi = torch.tensor(basis.tables(st.p)["x"])
    n = st.n_elem[d]
    h = (st.hi[d] - st.lo[d]) / n
    e = torch.arange(n, dtype=torch.float64)
    x = st.lo[d] + (e[:, None] + 0.5 * (xi[None, :] + 1.0)) * h       # [n, q]
    shape = st.shape()
    if d == 0:
        return x.reshape(1, 1, n, 1, 1, -1).expand(shape).clone()
    return x.reshape(1, n, 1, 1, -1, 1).expand(shape).clone()


def _field(st, f):
    """Conserved-looking field [nvar, ...]: each component a multiple of f plus an offset."""
    comps = [2.0 + (k + 1) * f for k in range(st.nvar)]
    return torch.stack(comps)


@pytest.mark.parametrize("dim,p", [(1, 1), (1, 3), (2, 2), (2, 3)])
def test_slope_is_the_linear_legendre_coefficient(dim, p):
    """The slope the limiter reads is the coefficient of xi_d in the Legendre expansion of
    the element's interpolating polynomial (fitted here by numpy's Legendre Vandermonde)."""
    from numpy.polynomial import legendre as L
    rng = np.random.default_rng(3)
    st = Setup(dim=dim, p=p, n_elem=(3, 2 if dim == 2 else 1, 1))
    U = torch.from_numpy(rng.normal(size=(st.nvar,) + st.shape()))
    w = odg.elem_weights(st)
    x = basis.tables(p)["x"]
    for d in range(dim):
        s = limiter._slope(U, w, limiter._xi(st, d), d).numpy()
        for k in range(st.nvar):
            for ey in range(st.n_elem[1] if dim == 2 else 1):
                for ex in range(st.n_elem[0]):
                    u = U[k, 0, ey, ex, 0].numpy()              # [nj, ni]
                    if dim == 1:
                        a = L.legfit(x, u[0], p)
                        ref = a[1]
                    else:
                        X, Y = np.meshgrid(x, x)                # X varies along i, Y along j
                        V = L.legvander2d(X.ravel(), Y.ravel(), [p, p])
                        a = np.linalg.solve(V, u.ravel()).reshape(p + 1, p + 1)   # a[deg_x, deg_y]
                        ref = a[1, 0] if d == 0 else a[0, 1]
                    assert abs(s[k, 0, ey, ex] - ref) <= 1e-13 * (1 + abs(ref))


@pytest.mark.parametrize("dim,p", [(1, 1), (1, 2), (1, 3), (2, 1), (2, 2), (2, 3)])
def test_linear_data_is_left_unchanged_and_averages_kept(dim, p):
    """A globally linear field: every interior element's slope equals half the difference
    of the neighbouring averages, so nothing is limited away from the ends (outflow ends
    see themselves and are cut to constants, keeping their averages)."""
    st = Setup(dim=dim, p=p, n_elem=(9, 7 if dim == 2 else 1, 1), bc=(OUTFLOW, OUTFLOW, OUTFLOW))
    x = _node_x(st, 0)
    y = _node_x(st, 1) if dim == 2 else 0 * x
    U = _field(st, 0.3 * x - 0.7 * y)
    stats = {}
    V = limiter.limit(U, st, stats)
    assert torch.allclose(_averages(V, st), _averages(U, st), rtol=0, atol=1e-14)
    inner = (slice(None), slice(None), slice(1, -1) if dim == 2 else slice(None), slice(1, -1))
    assert torch.allclose(V[inner], U[inner], rtol=0, atol=1e-14)


def test_periodic_linear_modes_only_limited_at_the_wrap():
    st = Setup(dim=1, p=2, n_elem=(12, 1, 1), bc=(PERIODIC, PERIODIC, PERIODIC))
    U = _field(st, _node_x(st, 0))
    V = limiter.limit(U, st)
    # the wrap joins x = 1 to x = 0: only the two elements beside it change (elsewhere the
    # slope and the half-differences agree to rounding, whichever minmod picks)
    diff = (V - U).abs().amax((0, 1, 2, 4, 5, 6))
    assert float(diff[1:-1].max()) <= 1e-14 and float(diff[0]) > 0.01 and float(diff[-1]) > 0.01


@pytest.mark.parametrize("p", [1, 2, 3])
def test_a_jump_inside_an_element_is_scaled_to_the_neighbour_difference(p):
    """A step from 1 to 3 whose jump lies inside element 4 of 10: its slope (the linear
    Legendre coefficient, from numpy's fit) is steeper than the difference to either
    constant neighbour, so the element's deviation from its average is scaled by the
    least ratio bound / slope over the components; the constant elements stay."""
    from numpy.polynomial import legendre as L
    st = Setup(dim=1, p=p, n_elem=(10, 1, 1), bc=(OUTFLOW, OUTFLOW, OUTFLOW))
    x = _node_x(st, 0)
    f = torch.where(x < 0.45, torch.ones_like(x), 3.0 * torch.ones_like(x))
    U = _field(st, f)
    V = limiter.limit(U, st)
    avg = _averages(U, st)[:, 0, 0]
    xs = basis.tables(p)["x"]
    ratios = []
    for k in range(st.nvar):
        slope = L.legfit(xs, U[k, 0, 0, 4, 0, 0].numpy(), p)[1]
        bound = min(float(avg[k, 5] - avg[k, 4]), float(avg[k, 4] - avg[k, 3]))
        assert 0 < bound < slope
        ratios.append(bound / slope)
    th = min(ratios)
    for k in range(st.nvar):
        assert torch.allclose(V[k, 0, 0, 4], avg[k, 4] + th * (U[k, 0, 0, 4] - avg[k, 4]), rtol=0, atol=1e-13)
    assert torch.equal(V[:, :, :, :4], U[:, :, :, :4]) and torch.equal(V[:, :, :, 5:], U[:, :, :, 5:])


@pytest.mark.parametrize("p", [1, 2, 3])
def test_a_spike_inside_an_element_is_cut_to_a_constant(p):
    """A bump confined to element 4 with equal constants on both sides: the two
    half-differences of the averages have opposite signs, so minmod gives zero and the
    element becomes its own average."""
    st = Setup(dim=1, p=p, n_elem=(10, 1, 1), bc=(OUTFLOW, OUTFLOW, OUTFLOW))
    x = _node_x(st, 0)
    f = 1.0 + torch.where((x > 0.4) & (x < 0.44), torch.ones_like(x), torch.zeros_like(x))
    U = _field(st, f)
    V = limiter.limit(U, st)
    avg = _averages(U, st)
    assert torch.allclose(V[:, 0, 0, 4], avg[:, 0, 0, 4, None, None, None].expand_as(V[:, 0, 0, 4]), rtol=0, atol=1e-14)
    assert torch.equal(V[:, :, :, :4], U[:, :, :, :4]) and torch.equal(V[:, :, :, 5:], U[:, :, :, 5:])


@pytest.mark.parametrize("dim,p", [(1, 2), (2, 1), (2, 3), (3, 1)])
def test_limited_slopes_obey_the_minmod_bounds(dim, p):
    """On random data: each element moves towards its average by one factor theta in
    [0, 1] for all components; every limited slope keeps the sign of its own slope and
    no larger magnitude, and stays within the minmod bound of the neighbour differences
    (up to the rounding guard); averages kept; limiting twice changes nothing more."""
    rng = np.random.default_rng(8)
    n = (7, 6 if dim > 1 else 1, 5 if dim > 2 else 1)
    st = Setup(dim=dim, p=p, n_elem=n, bc=(PERIODIC,) * 3)
    U = torch.from_numpy(rng.normal(size=(st.nvar,) + st.shape())) * 0.3 + 3.0
    V = limiter.limit(U, st)
    avg = _averages(U, st)
    assert torch.allclose(_averages(V, st), avg, rtol=0, atol=1e-13)
    # one factor per element: V - avg = theta (U - avg)
    dU, dV = U - avg[..., None, None, None], V - avg[..., None, None, None]
    th = (dV * dU).sum((0, 4, 5, 6)) / (dU * dU).sum((0, 4, 5, 6))
    assert bool(((th >= -1e-14) & (th <= 1 + 1e-14)).all()) and float((th < 1 - 1e-12).float().mean()) > 0.3
    assert torch.allclose(dV, th[None, ..., None, None, None] * dU, rtol=0, atol=1e-13)
    w = odg.elem_weights(st)
    sig = limiter.scales(avg, st)
    for d in range(dim):
        xi = limiter._xi(st, d)
        s = limiter._slope(U, w, xi, d)
        sv = limiter._slope(V, w, xi, d)
        ea = 3 - d
        fwd = torch.roll(avg, -1, ea) - avg
        bwd = avg - torch.roll(avg, 1, ea)
        bound = limiter._minmod(s, fwd, bwd).abs()
        assert bool(((sv == 0) | (torch.sign(sv) == torch.sign(s))).all())
        assert bool((sv.abs() <= s.abs() * (1 + 1e-12)).all())
        assert bool((sv.abs() <= bound * (1 + 1e-12) + 2 * limiter.EPS * sig).all())
    W = limiter.limit(V, st)
    assert torch.allclose(W, V, rtol=0, atol=1e-13)


def test_limited_euler_step_does_not_increase_the_total_variation_of_averages():
    """The paper's Sod-like Riemann problem 4 at p = 1 on 60 cells: forward-Euler steps
    (CFL 0.1/3), each followed by the limiter and the physicality operator, do not
    increase the total variation of the averages of D beyond the rounding guard (the
    limited scheme is TVD in the means here), while without the limiter it grows."""
    from tests._exact import riemann_problem
    L, R, gam, _, _ = riemann_problem(4)
    st = Setup(dim=1, p=1, n_elem=(60, 1, 1), bc=(OUTFLOW,) * 3, gamma_ad=gam, eos=IDEAL, flux=HLLC)
    x = _node_x(st, 0)
    pick = lambda a, b: torch.where(x < 0.5, a, b)  # noqa: E731
    one = torch.ones_like(x)
    rho = pick(L[0] * one, R[0] * one)
    v = pick(L[1] * one, R[1] * one)[None]
    P = pick(L[2] * one, R[2] * one)
    U = srhd.prim3_to_cons(rho, v, P, st)
    U = limiter.limit(U, st)
    dt = 0.1 / 3 / 60

    def tv(V):
        a = _averages(V, st)[0].reshape(-1)
        return float((a[1:] - a[:-1]).abs().sum())
    tv0 = tv(U)
    Un, grew = U.clone(), False
    for _ in range(20):
        raw = U + dt * odg.rhs(U, st)
        U = ophys.enforce(limiter.limit(raw, st), st)
        # up to what the rounding guard lets through (measured <= 2e-10 per step)
        assert tv(U) <= tv0 * (1 + 1e-8)
        tv0 = tv(U)
        tvn = tv(Un)
        Un = ophys.enforce(Un + dt * odg.rhs(Un, st), st)
        grew = grew or tv(Un) > tvn * (1 + 1e-4)   # measured up to 6e-3 per step
    assert grew


@pytest.mark.parametrize("p", [1, 2])
def test_strong_blast_stays_admissible_with_the_limiter(p):
    """The paper's strong blast wave (problem 2, pressure ratio 1e5) at 50 cells: 60 limited
    steps with the physicality operator keep every element average admissible and every
    recovery successful (the componentwise form lost an average in the first step)."""
    from oracle import timestep
    from tests._exact import riemann_problem
    L, R, gam, _, _ = riemann_problem(2)
    st = Setup(dim=1, p=p, n_elem=(50, 1, 1), bc=(OUTFLOW,) * 3, gamma_ad=gam, eos=IDEAL, flux=HLLC, limiter=1)
    x = _node_x(st, 0)
    one = torch.ones_like(x)
    pick = lambda a, b: torch.where(x < 0.5, a * one, b * one)  # noqa: E731
    U = srhd.prim3_to_cons(pick(L[0], R[0]), pick(L[1], R[1])[None], pick(L[2], R[2]), st)
    stats = {}
    U = timestep.run(U, 0.1 / (2 * p + 1) / 50, 60, st, stats=stats, order=p + 1)
    assert stats.get("c2p_fail", 0) == 0 and stats.get("bad_average", 0) == 0
    assert stats["limited"] > 0
    assert bool(srhd.admissible(U, st).all())
