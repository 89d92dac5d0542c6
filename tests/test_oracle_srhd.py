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
