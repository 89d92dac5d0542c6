"""Pins of the oracle's conserved-to-primitive solvers (Sec. 3)."""
import numpy as np
import pytest
import torch

from oracle import con2prim as cp
from oracle import srhd
from oracle.setup import BRENT, CUBIC, IDEAL, NEWTON, QUARTIC, TM, Setup
from paper_2205_00095_amd import workloads as wl


def _states(rng, n, gmax, thlo, thhi, c=1.0, dim=3):
    g = rng.uniform(1.0, gmax, n)
    rho = 10 ** rng.uniform(-3, 3, n)
    P = rho * c * c * 10 ** rng.uniform(np.log10(thlo), np.log10(thhi), n)
    nv = rng.standard_normal((dim, n))
    nv /= np.linalg.norm(nv, axis=0)
    v = nv * c * np.sqrt((1 - 1 / g) * (1 + 1 / g))
    return rho, v, P


def _roundtrip(eos, method, rho, v, P, c=1.0):
    st = Setup(dim=v.shape[0], p=0, eos=eos, c=c)
    rho_t, v_t, P_t = (torch.tensor(a) for a in (rho, v, P))
    U = srhd.prim3_to_cons(rho_t, v_t, P_t, st)
    W, status = cp.con2prim(U, st, method)
    u_true = srhd.u_from_v(v_t, c)
    return W, status, rho_t, u_true, P_t


@pytest.mark.parametrize("eos,method", [(IDEAL, NEWTON), (TM, CUBIC), (TM, BRENT)])
def test_roundtrip_well_conditioned(eos, method):
    """prim -> cons -> prim to 1e-12 relative on gamma <= 10, Theta/c^2 in [1e-2, 1e2]."""
    rng = np.random.default_rng(21)
    n = 300 if method != BRENT else 60
    rho, v, P = _states(rng, n, 10.0, 1e-2, 1e2)
    W, status, rho_t, u_t, P_t = _roundtrip(eos, method, rho, v, P)
    assert int((status != 0).sum()) == 0
    assert ((W[0] - rho_t).abs() / rho_t).max() < 1e-12
    assert ((W[-1] - P_t).abs() / P_t).max() < 1e-12
    umag = torch.sqrt((u_t ** 2).sum(0))
    assert (torch.sqrt(((W[1:-1] - u_t) ** 2).sum(0)) / umag).max() < 1e-12


def test_ideal_quartic_measured_accuracy():
    """Analytic quartic (parity unpinned beyond its accuracy): 1e-7 on beta in [0.5, 0.9]."""
    rng = np.random.default_rng(22)
    n = 200
    beta = rng.uniform(0.5, 0.9, n)
    g = 1 / np.sqrt(1 - beta ** 2)
    rho = 10 ** rng.uniform(-1, 1, n)
    P = rho * 10 ** rng.uniform(-1, 1, n)
    v = np.stack([beta, 0 * beta, 0 * beta])
    W, status, rho_t, u_t, P_t = _roundtrip(IDEAL, QUARTIC, rho, v, P)
    assert int((status != 0).sum()) == 0
    vrec = W[1] / torch.sqrt(1 + (W[1:-1] ** 2).sum(0))
    assert ((vrec - torch.tensor(beta)).abs() / torch.tensor(beta)).max() < 1e-7
    assert g.max() < 3


@pytest.mark.parametrize("eos,method,tol", [(IDEAL, NEWTON, 1e-14), (TM, CUBIC, 1e-14)])
def test_paper_accuracy_grid(eos, method, tol):
    """The paper's 25x25 grid: gamma in [1,100], P in [1e5,1e10] Pa, D = 1, c = 3e8;
    relative error of the recovered velocity (Sec. 3.3)."""
    c = 3.0e8
    G, PP = wl.c2p_grid(25, c=c)
    g, P = G.ravel(), PP.ravel()
    rho = 1.0 / g
    beta = np.sqrt((1 - 1 / g) * (1 + 1 / g))
    v = np.stack([beta * c, 0 * g, 0 * g])
    W, status, rho_t, u_t, P_t = _roundtrip(eos, method, rho, v, P, c=c)
    assert int((status != 0).sum()) == 0
    vrec = W[1] / torch.sqrt(1 + (W[1:-1] ** 2).sum(0) / c ** 2)
    nz = beta > 0
    err = ((vrec.numpy() - beta * c)[nz] / (beta * c)[nz])
    assert np.abs(err).max() < tol


def test_riccardi_quartic_vanishes_at_exact_w():
    """P(w) of Eq. (iterative_quartic) at w = beta/(1 + sqrt(1-beta^2)) from the primitives."""
    rng = np.random.default_rng(23)
    st = Setup(dim=3, p=0, eos=IDEAL)
    rho, v, P = _states(rng, 200, 50.0, 1e-3, 1e3)
    U = srhd.prim3_to_cons(torch.tensor(rho), torch.tensor(v), torch.tensor(P), st).numpy()
    D, S, tau = U[0], U[1:4], U[4]
    xi = np.linalg.norm(S, axis=0) / D
    eta = 1 + tau / D
    a = st.gamma_ad / (st.gamma_ad - 1)
    beta = np.linalg.norm(v, axis=0)
    w = beta / (1 + np.sqrt((1 - beta) * (1 + beta)))
    terms = [(a - 1) * xi * w ** 4, -2 * (a * eta + 1) * w ** 3, 2 * (a + 1) * xi * w ** 2,
             -2 * (a * eta - 1) * w, (a - 1) * xi]
    res = sum(terms) / np.max(np.abs(terms), axis=0)
    assert np.abs(res).max() < 1e-12


def test_ideal_quartic_in_beta_vanishes_at_exact_beta():
    rng = np.random.default_rng(24)
    st = Setup(dim=3, p=0, eos=IDEAL)
    G = st.gamma_ad
    rho, v, P = _states(rng, 200, 20.0, 1e-2, 1e2)
    U = srhd.prim3_to_cons(torch.tensor(rho), torch.tensor(v), torch.tensor(P), st).numpy()
    xi = np.linalg.norm(U[1:4], axis=0) / U[0]
    eta = 1 + U[4] / U[0]
    den = (G - 1) ** 2 * (xi ** 2 + 1)
    a3 = -2 * G * (G - 1) * xi * eta / den
    a2 = (G ** 2 * eta ** 2 + 2 * (G - 1) * xi ** 2 - (G - 1) ** 2) / den
    a1 = -2 * G * xi * eta / den
    a0 = xi ** 2 / den
    b = np.linalg.norm(v, axis=0)
    terms = [b ** 4, a3 * b ** 3, a2 * b ** 2, a1 * b, a0]
    assert np.abs(sum(terms) / np.max(np.abs(terms), axis=0)).max() < 1e-12


def test_tm_cubic_vanishes_at_exact_W():
    """Eq. (synge_cubic) at W = gamma^2 - 1 computed from the primitives."""
    rng = np.random.default_rng(25)
    st = Setup(dim=3, p=0, eos=TM)
    rho, v, P = _states(rng, 200, 30.0, 1e-3, 1e3)
    U = srhd.prim3_to_cons(torch.tensor(rho), torch.tensor(v), torch.tensor(P), st)
    xi = torch.sqrt((U[1:4] ** 2).sum(0)) / U[0]
    eta = 1 + U[4] / U[0]
    c1, c2, c3 = (t.numpy() for t in cp._tm_coeffs(xi, eta))
    b2 = (np.asarray(v) ** 2).sum(0)
    W = b2 / ((1 - np.sqrt(b2)) * (1 + np.sqrt(b2)))
    terms = [W ** 3, c1 * W ** 2, c2 * W, c3]
    assert np.abs(sum(terms) / np.max(np.abs(terms), axis=0)).max() < 1e-11


def test_small_xi_series_matches_newton():
    """The cubic series (Eq. iterative_cubic_approximation) agrees with Newton where both apply."""
    st = Setup(dim=1, p=0, eos=IDEAL)
    theta = np.repeat([0.01, 1.0, 30.0], 5)
    hhat = 1.0 + 4.0 * theta                      # h/c^2 for Gamma = 4/3
    beta = (np.array([0.01, 0.05, 0.2, 0.5, 0.7] * 3) * 1e-4 / hhat)[None]
    U = srhd.prim3_to_cons(torch.ones(15), torch.tensor(beta), torch.tensor(theta), st)
    xi = U[1] / U[0]
    assert float(xi.max()) < 1e-4
    Ws, _ = cp.ideal_newton(U, st)                    # series branch
    Wn, s = cp.ideal_newton(U, st, series_below=0.0)  # forced Newton
    assert int((s != 0).sum()) == 0
    assert ((Ws[1] - Wn[1]).abs() / Wn[1].abs()).max() < 1e-14
    assert ((Ws[1] - srhd.u_from_v(torch.tensor(beta), 1.0)[0]).abs() / Wn[1].abs()).max() < 1e-14


@pytest.mark.parametrize("eos,method", [(IDEAL, NEWTON), (TM, CUBIC)])
def test_bisection_brute_force(eos, method):
    st = Setup(dim=3, p=0, eos=eos)
    rng = np.random.default_rng(26)
    rho, v, P = _states(rng, 6, 5.0, 1e-1, 1e1)
    U = srhd.prim3_to_cons(torch.tensor(rho), torch.tensor(v), torch.tensor(P), st)
    W, _ = cp.con2prim(U, st, method)
    for k in range(6):
        b_bis = cp.bisect_beta(U[:, k], st, iters=60)
        u = W[1:-1, k]
        b_rec = float(torch.sqrt((u ** 2).sum() / (1 + (u ** 2).sum())))
        assert abs(b_bis - b_rec) < 1e-9 * b_rec


@pytest.mark.parametrize("eos", [IDEAL, TM])
def test_failure_convention(eos):
    st = Setup(dim=2, p=0, eos=eos)
    U = torch.tensor([[1.0, -1.0, 1.0, 0.0],        # D
                      [0.5, 0.1, 5.0, 0.0],         # S_x (third: |S| too large)
                      [0.0, 0.0, 0.0, 0.0],         # S_y
                      [1.0, 1.0, 0.1, 0.0]])        # tau (fourth: D = 0)
    W, status = cp.con2prim(U, st)
    assert status.tolist() == [0, 1, 1, 1]
    assert torch.all(W[0, 1:] == cp.RHO_FLOOR) and torch.all(W[-1, 1:] == cp.P_FLOOR)
    assert torch.all(W[1:-1, 1:] == 0) and torch.isfinite(W).all()
