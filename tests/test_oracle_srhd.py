"""Pins of the oracle's state relations, wavespeeds and HLL flux (Sec. 2.1, 2.4, 2.5)."""
import numpy as np
import pytest
import torch

from oracle import srhd
from oracle.setup import IDEAL, TM, Setup
from oracle.eos import enthalpy


def _random_prims(rng, n, dim, gmax=8.0, c=1.0):
    g = rng.uniform(1.0, gmax, n)
    rho = 10 ** rng.uniform(-1, 1, n)
    P = rho * 10 ** rng.uniform(-1, 1, n) * c * c
    nv = rng.standard_normal((dim, n))
    nv /= np.linalg.norm(nv, axis=0)
    v = nv * c * np.sqrt(1 - 1 / g ** 2)
    return rho, v, P


@pytest.mark.parametrize("kind", [IDEAL, TM])
@pytest.mark.parametrize("c", [1.0, 7.0])
def test_prim_to_cons_is_a_lorentz_boost(kind, c):
    """D = rho U^0/c and (E, M c) = first row of Lambda T_rest Lambda^T (explicit boost matrix)."""
    st = Setup(dim=3, p=0, eos=kind, c=c)
    rng = np.random.default_rng(3)
    rho, v, P = _random_prims(rng, 30, 3, c=c)
    U = srhd.prim3_to_cons(torch.tensor(rho), torch.tensor(v), torch.tensor(P), st).numpy()
    for k in range(30):
        vk = v[:, k]
        b2 = vk @ vk / c ** 2
        g = 1 / np.sqrt(1 - b2)
        L = np.eye(4)
        L[0, 0] = g
        L[0, 1:] = L[1:, 0] = g * vk / c
        L[1:, 1:] += (g - 1) * np.outer(vk, vk) / (vk @ vk)
        h = float(enthalpy(torch.tensor(P[k] / rho[k]), kind, st.gamma_ad, c))
        Trest = np.diag([rho[k] * h - P[k], P[k], P[k], P[k]])
        T = L @ Trest @ L.T
        E = U[-1, k] + U[0, k] * c * c
        assert abs(U[0, k] - g * rho[k]) < 1e-14 * U[0, k]
        assert abs(E - T[0, 0]) < 1e-12 * T[0, 0]
        assert np.allclose(U[1:4, k] * c, T[0, 1:], rtol=1e-12, atol=1e-12 * T[0, 0])


@pytest.mark.parametrize("kind", [IDEAL, TM])
@pytest.mark.parametrize("dim", [2, 3])
def test_wavespeeds_are_extreme_eigenvalues(kind, dim):
    """lambda_pm = min/max eigenvalue of dF^d/dU = (dF/dW)(dU/dW)^-1 (Jacobians by autograd)."""
    st = Setup(dim=dim, p=0, eos=kind)
    rng = np.random.default_rng(11)
    rho, v, P = _random_prims(rng, 12, dim)
    for k in range(12):
        u = srhd.u_from_v(torch.tensor(v[:, k:k + 1]), 1.0)[:, 0]
        W = torch.cat([torch.tensor([rho[k]]), u, torch.tensor([P[k]])])
        for d in range(dim):
            dU = torch.autograd.functional.jacobian(lambda w: srhd.prim_to_cons(w[:, None], st)[:, 0], W)
            dF = torch.autograd.functional.jacobian(lambda w: srhd.flux(w[:, None], d, st)[:, 0], W)
            ev = np.linalg.eigvals((dF @ torch.linalg.inv(dU)).numpy())
            assert np.abs(ev.imag).max() < 1e-9
            lm, lp = srhd.wavespeeds(W[:, None], d, st)
            assert abs(ev.real.min() - float(lm)) < 1e-11
            assert abs(ev.real.max() - float(lp)) < 1e-11


@pytest.mark.parametrize("kind", [IDEAL, TM])
def test_wavespeeds_reduce_to_velocity_addition(kind):
    st = Setup(dim=1, p=0, eos=kind)
    from oracle.eos import sound_speed_sq
    for vx in (-0.9, -0.3, 0.0, 0.5, 0.99):
        rho, P = 1.3, 0.7
        u = srhd.u_from_v(torch.tensor([[vx]]), 1.0)
        W = torch.cat([torch.tensor([[rho]]), u, torch.tensor([[P]])])
        cs = float(torch.sqrt(sound_speed_sq(torch.tensor(P / rho), kind, st.gamma_ad, 1.0)))
        lm, lp = srhd.wavespeeds(W, 0, st)
        assert abs(float(lp) - (vx + cs) / (1 + vx * cs)) < 1e-14
        assert abs(float(lm) - (vx - cs) / (1 - vx * cs)) < 1e-14


@pytest.mark.parametrize("kind", [IDEAL, TM])
def test_hll_consistency_and_upwinding(kind):
    st = Setup(dim=2, p=0, eos=kind)
    rng = np.random.default_rng(5)
    rho, v, P = _random_prims(rng, 40, 2)
    u = srhd.u_from_v(torch.tensor(v), 1.0)
    W = torch.cat([torch.tensor(rho)[None], u, torch.tensor(P)[None]])
    for d in range(2):
        assert torch.allclose(srhd.hll(W, W, d, st), srhd.flux(W, d, st), rtol=1e-13, atol=1e-13)
    # supersonic to +x: both states move right faster than sound -> left flux
    vL = torch.tensor([[0.99], [0.0]])
    vR = torch.tensor([[0.98], [0.05]])
    WL = torch.cat([torch.tensor([[1.0]]), srhd.u_from_v(vL, 1.0), torch.tensor([[0.01]])])
    WR = torch.cat([torch.tensor([[0.5]]), srhd.u_from_v(vR, 1.0), torch.tensor([[0.02]])])
    assert torch.equal(srhd.hll(WL, WR, 0, st), srhd.flux(WL, 0, st))
    assert torch.equal(srhd.hll(WR, WL, 0, st), srhd.flux(WR, 0, st))


def test_q_tau_form_equals_paper_form():
    st = Setup(dim=3, p=0)
    rng = np.random.default_rng(9)
    U = torch.tensor(rng.uniform(0.5, 2.0, (5, 100)))
    U[1:4] -= 1.0
    c = st.c
    E = U[-1] + U[0] * c * c
    q_paper = E / c ** 2 - torch.sqrt(U[0] ** 2 + (U[1:4] ** 2).sum(0) / c ** 2)
    assert torch.allclose(srhd.q_admiss(U, st), q_paper, rtol=1e-12, atol=1e-14)


# ------------------------------------------------------------------ HLLC
def _prims_tensor(rho, v, P, c):
    u = srhd.u_from_v(torch.tensor(v), c)
    return torch.cat([torch.tensor(rho)[None], u, torch.tensor(P)[None]])


@pytest.mark.parametrize("kind", [IDEAL, TM])
@pytest.mark.parametrize("c", [1.0, 7.0])
def test_hllc_consistency_and_upwinding(kind, c):
    st = Setup(dim=2, p=0, eos=kind, c=c)
    rng = np.random.default_rng(15)
    W = _prims_tensor(*_random_prims(rng, 40, 2, c=c), c)
    for d in range(2):
        F = srhd.flux(W, d, st)
        assert torch.allclose(srhd.hllc(W, W, d, st), F, rtol=1e-12, atol=1e-12 * float(F.abs().max()))
    # supersonic to +x: every wave moves right -> the left flux, and vice versa
    WL = _prims_tensor(np.array([1.0]), np.array([[0.99], [0.0]]) * c, np.array([0.01]) * c * c, c)
    WR = _prims_tensor(np.array([0.5]), np.array([[0.98], [0.05]]) * c, np.array([0.02]) * c * c, c)
    assert torch.equal(srhd.hllc(WL, WR, 0, st), srhd.flux(WL, 0, st))
    WL2 = _prims_tensor(np.array([1.0]), -np.array([[0.99], [0.0]]) * c, np.array([0.01]) * c * c, c)
    WR2 = _prims_tensor(np.array([0.5]), -np.array([[0.98], [0.05]]) * c, np.array([0.02]) * c * c, c)
    assert torch.equal(srhd.hllc(WL2, WR2, 0, st), srhd.flux(WR2, 0, st))


@pytest.mark.parametrize("kind", [IDEAL, TM])
@pytest.mark.parametrize("c", [1.0, 7.0])
def test_hllc_star_states_satisfy_the_contact_conditions(kind, c):
    """For random state pairs: lamL < lam* < lamR, both star states move with the
    contact (c^2 S*_d = (E* + p*) lam*), the star fluxes from the outer jump conditions
    equal the contact flux lam* U* + p* (0, e_d, lam*), and the fan integral of the two
    star states equals that of the HLL state."""
    st = Setup(dim=3, p=0, eos=kind, c=c)
    rng = np.random.default_rng(16)
    n = 400
    WL = _prims_tensor(*_random_prims(rng, n, 3, gmax=5.0, c=c), c)
    WR = _prims_tensor(*_random_prims(rng, n, 3, gmax=5.0, c=c), c)
    c2 = c * c
    for d in range(3):
        aL, aR, lam, ps, UsL, UsR = srhd.hllc_star(WL, WR, d, st)
        # (p* itself may come out negative for pairs that separate fast, a known limit of
        # the solver: the strong-rarefaction case the exact solution fills with near vacuum)
        assert bool((aL < lam).all()) and bool((lam < aR).all())
        for K, (W, Us, a) in enumerate(((WL, UsL, aL), (WR, UsR, aR))):
            E = Us[-1] + c2 * Us[0]
            lhs, rhs = c2 * Us[1 + d], (E + ps) * lam
            # rounding of the star states grows with 1 / |lam_K - lam*|
            kappa = (a.abs() + lam.abs() + c) / (a - lam).abs()
            scale = ((E.abs() + ps.abs()) * c + c2 * Us[1 + d].abs()) * kappa
            assert float(((lhs - rhs).abs() / scale).max()) < 1e-12, (kind, d, K)
            U, F = srhd.prim_to_cons(W, st), srhd.flux(W, d, st)
            Fs = F + a * (Us - U)
            contact = lam * Us
            contact[1 + d] = contact[1 + d] + ps
            contact[-1] = contact[-1] + ps * lam
            fs = F.abs() + (a * U).abs() + (a * Us).abs()
            assert float(((Fs - contact).abs() / fs).max()) < 1e-12, (kind, d, K)
        UL, UR = srhd.prim_to_cons(WL, st), srhd.prim_to_cons(WR, st)
        FL, FR = srhd.flux(WL, d, st), srhd.flux(WR, d, st)
        Uhll = (aR * UR - aL * UL + FL - FR) / (aR - aL)
        fan = ((lam - aL) * UsL + (aR - lam) * UsR) / (aR - aL)
        sc = (aR * UR).abs() + (aL * UL).abs() + FL.abs() + FR.abs()
        assert float(((fan - Uhll).abs() * (aR - aL) / sc).max()) < 1e-12


@pytest.mark.parametrize("kind", [IDEAL, TM])
@pytest.mark.parametrize("c", [1.0, 7.0])
@pytest.mark.parametrize("vn", [-0.3, -0.1, 0.0, 0.35])
def test_hllc_resolves_an_isolated_contact(kind, c, vn):
    """Density and tangential-velocity jump at equal pressure and normal velocity: the
    exact solution is the contact moving at vn, whose upwind state is the flux at the
    face; HLLC returns it exactly (to rounding), HLL does not (it smears the contact)."""
    st = Setup(dim=3, p=0, eos=kind, c=c)
    P = np.array([0.8 * c * c])
    vL = np.array([[vn], [0.3], [-0.2]]) * c
    vR = np.array([[vn], [-0.5], [0.1]]) * c
    WL = _prims_tensor(np.array([1.0]), vL, P, c)
    WR = _prims_tensor(np.array([0.05]), vR, P, c)
    FL, FR = srhd.flux(WL, 0, st), srhd.flux(WR, 0, st)
    Fc = srhd.hllc(WL, WR, 0, st)
    scale = float(FL.abs().max() + FR.abs().max())
    if vn > 0:
        exact = FL
    elif vn < 0:
        exact = FR
    else:
        exact = torch.zeros_like(FL)
        exact[1] = float(P[0])
    assert float((Fc - exact).abs().max()) <= 1e-13 * scale, (Fc, exact)
    assert float((srhd.hll(WL, WR, 0, st) - exact).abs().max()) > 1e-3 * scale
    _, _, lam, ps, _, _ = srhd.hllc_star(WL, WR, 0, st)
    assert abs(float(lam) - vn * c) <= 1e-14 * c and abs(float(ps) - float(P[0])) <= 1e-13 * float(P[0])


@pytest.mark.parametrize("kind", [IDEAL, TM])
def test_hllc_mirror_symmetry(kind):
    """Reflecting x -> -x and swapping the sides flips the sign of every flux row but the
    normal momentum's."""
    st = Setup(dim=2, p=0, eos=kind)
    rng = np.random.default_rng(17)
    WL = _prims_tensor(*_random_prims(rng, 60, 2), 1.0)
    WR = _prims_tensor(*_random_prims(rng, 60, 2), 1.0)
    flip = torch.tensor([1.0, -1.0, 1.0, 1.0])[:, None]
    F = srhd.hllc(WL, WR, 0, st)
    G = srhd.hllc(WR * flip, WL * flip, 0, st)
    sign = torch.tensor([-1.0, 1.0, -1.0, -1.0])[:, None]
    assert torch.allclose(G, sign * F, rtol=1e-12, atol=1e-12 * float(F.abs().max()))
