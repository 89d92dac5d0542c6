"""Reflecting walls on the GPU (the boundaries of the paper's reflecting-wall test,
Sec. 4): parity of the RHS, the steps and the adjoint with the FP64 oracle, the
equivalence with a doubled periodic mesh holding the mirror image, and mass and
energy conservation in a closed box over many steps."""
import pytest
import torch

from oracle import dg as odg
from oracle import timestep as ots
from paper_2205_00095_amd import workloads as wl

from ._util import oracle_state, perturbed, rel_err_per_var, rhs_bar, step_bar

pytestmark = pytest.mark.gpu

R = wl.REFLECT


def _solver(cfg, sync=True):
    from paper_2205_00095_amd.solver import Solver
    return Solver(cfg, sync=sync)


CASES = [
    ("wave1d", {"bc": (R, R, R)}, wl.FLUX_HLL),
    ("wave1d", {"bc": (R, R, R), "p": 3}, wl.FLUX_HLLC),
    ("kh_tm", {"n_elem": (8, 6, 1), "bc": (R, R, R)}, wl.FLUX_HLL),
    ("kh_ideal", {"n_elem": (7, 6, 1), "bc": (wl.PERIODIC, R, R), "init": "kh"}, wl.FLUX_HLLC),
    ("random3d", {"n_elem": (3, 3, 2), "p": 1, "bc": (R, R, R)}, wl.FLUX_HLL),
]


def _cfg(kind, over, flux):
    cfg = wl.make_config(kind, **over)
    cfg["precision"] = wl.FP64
    cfg["flux"] = flux
    return cfg


@pytest.mark.parametrize("kind,over,flux", CASES)
def test_wall_rhs_matches_oracle(kind, over, flux):
    cfg = _cfg(kind, over, flux)
    print(f"case walls rhs {kind} {over} flux {flux}", flush=True)
    st, U = oracle_state(cfg)
    R_ref = odg.rhs(U, st)
    bar, kappa = rhs_bar(U, st, R_ref)
    Rg = _solver(cfg).rhs(U.cuda()).cpu()
    err = rel_err_per_var(Rg, R_ref)
    print(f"err {err.tolist()} bar {bar.tolist()} kappa {kappa.tolist()}", flush=True)
    assert bool((err <= bar).all()), (err.tolist(), bar.tolist())


@pytest.mark.parametrize("kind,over,flux", [CASES[2], CASES[3]])
def test_wall_steps_match_oracle(kind, over, flux):
    cfg = _cfg(kind, over, flux)
    print(f"case walls steps {kind} {over} flux {flux}", flush=True)
    st, U = oracle_state(cfg)
    U_ref, bar, kappa = step_bar(U, cfg["dt"], 4, st)
    Ud = U.cuda().contiguous()
    _solver(cfg, sync=False).run(Ud, cfg["dt"], 4)
    err = rel_err_per_var(Ud.cpu(), U_ref)
    print(f"err {err.tolist()} bar {bar.tolist()} kappa {kappa.tolist()}", flush=True)
    assert bool((err <= bar).all()), (err.tolist(), bar.tolist())


def _mirror_x(U):
    M = U.flip(3).flip(6).clone()
    M[1] = -M[1]
    return M


@pytest.mark.parametrize("flux", [wl.FLUX_HLL, wl.FLUX_HLLC])
def test_wall_equals_doubled_periodic_mesh_on_gpu(flux):
    """Walls at both x ends give the RHS of a periodic mesh twice as long holding the
    state and its mirror image, on the GPU alone."""
    cfg = _cfg("kh_tm", {"n_elem": (6, 5, 1), "bc": (R, wl.OUTFLOW, R)}, flux)
    cfg2 = _cfg("kh_tm", {"n_elem": (12, 5, 1), "hi": (2.0, 1.0, 1.0), "bc": (wl.PERIODIC, wl.OUTFLOW, R)}, flux)
    print(f"case walls vs doubled periodic flux {flux}", flush=True)
    st, U = oracle_state(cfg)
    U2 = torch.cat([U, _mirror_x(U)], 3).contiguous()
    Ra = _solver(cfg).rhs(U.cuda()).cpu()
    Rb = _solver(cfg2).rhs(U2.cuda()).cpu()[:, :, :, :6]
    err = rel_err_per_var(Ra, Rb)
    print(f"err {err.tolist()}", flush=True)
    assert float(err.max()) <= 1e-12, err.tolist()


def test_closed_box_conserves_mass_and_energy_on_gpu():
    """Walls on every side of the Kelvin-Helmholtz box: total D and tau stay constant
    over 200 SSP-RK3 steps to rounding."""
    cfg = _cfg("kh_tm", {"n_elem": (32, 32, 1), "bc": (R, R, R)}, wl.FLUX_HLL)
    print("case closed box 32x32 p=3, 200 steps", flush=True)
    s = _solver(cfg, sync=False)
    U = s.set_state(torch.from_numpy(wl.pack_primitives(*wl.initial_primitives(cfg))).cuda())
    import numpy as np
    w = np.polynomial.legendre.leggauss(cfg["p"] + 1)[1]
    wt = torch.tensor(np.outer(w, w), device="cuda")
    tot0 = (U * wt).sum(dim=(1, 2, 3, 4, 5, 6))
    s.run(U, cfg["dt"], 200)
    tot = (U * wt).sum(dim=(1, 2, 3, 4, 5, 6))
    scale = (U.abs() * wt).sum(dim=(1, 2, 3, 4, 5, 6))
    drift = ((tot - tot0).abs() / scale).cpu()
    print(f"relative drift D {float(drift[0]):.2e} tau {float(drift[-1]):.2e}", flush=True)
    assert float(drift[0]) <= 1e-13 and float(drift[-1]) <= 1e-13
    assert s.diagnostics()["c2p_fail"] == 0


@pytest.mark.parametrize("kind,over,flux", [("kh_ideal", {"n_elem": (6, 5, 1), "bc": (R, R, R), "init": "kh"}, f)
                                            for f in (wl.FLUX_HLL, wl.FLUX_HLLC)]
                         + [("kh_tm", {"n_elem": (5, 4, 1), "bc": (wl.PERIODIC, R, R)}, wl.FLUX_HLLC)])
def test_wall_vjp_matches_oracle_autograd(kind, over, flux):
    cfg = _cfg(kind, over, flux)
    print(f"case walls rhs_vjp {kind} {over} flux {flux}", flush=True)
    st, U = oracle_state(cfg)
    g = torch.Generator().manual_seed(7)
    lamR = torch.randn(U.shape, generator=g, dtype=torch.float64)

    def ref_of(V):
        Vr = V.clone().requires_grad_(True)
        return torch.autograd.grad(odg.rhs(Vr, st), Vr, lamR)[0]

    ref = ref_of(U)
    sens = rel_err_per_var(ref_of(perturbed(U)), ref)
    assert float(sens.max()) < 1e-10, f"test data sits on a derivative kink: {sens.tolist()}"
    got = _solver(cfg).rhs_vjp(U.cuda(), lamR.cuda()).cpu()
    err = rel_err_per_var(got, ref)
    print(f"err {err.tolist()}", flush=True)
    assert float(err.max()) <= 1e-9, err.tolist()


FIX = wl.DIRICHLET
_STATES = {(0, 0): (1.2, 0.3, 0.05, 0.0, 0.9), (0, 1): (0.8, -0.1, 0.0, 0.0, 1.1),
           (1, 0): (1.0, 0.0, 0.2, 0.0, 1.0), (1, 1): (0.9, 0.1, -0.25, 0.0, 1.2)}
MIXED = [
    ("wave1d", {"bc": (FIX, 0, 0), "bc_hi": (R, 0, 0), "bc_state": _STATES}, wl.FLUX_HLL),
    ("wave1d", {"bc": (R, 0, 0), "bc_hi": (FIX, 0, 0), "bc_state": _STATES, "p": 3}, wl.FLUX_HLLC),
    ("kh_tm", {"n_elem": (7, 6, 1), "bc": (FIX, R, 0), "bc_hi": (wl.OUTFLOW, FIX, 0), "bc_state": _STATES},
     wl.FLUX_HLL),
    ("kh_ideal", {"n_elem": (6, 5, 1), "bc": (FIX, FIX, 0), "bc_state": _STATES, "init": "kh"}, wl.FLUX_HLLC),
    ("random3d", {"n_elem": (3, 3, 2), "p": 1, "bc": (R, wl.OUTFLOW, FIX), "bc_hi": (FIX, 0, R),
                  "bc_state": {**_STATES, (2, 0): (0.7, 0.1, 0.0, 0.3, 0.5)}}, wl.FLUX_HLL),
]


@pytest.mark.parametrize("kind,over,flux", MIXED)
def test_mixed_ends_rhs_matches_oracle(kind, over, flux):
    """Boundary types chosen per end (fixed states, walls, outflow) against the oracle."""
    cfg = _cfg(kind, over, flux)
    print(f"case mixed ends rhs {kind} flux {flux}", flush=True)
    st, U = oracle_state(cfg)
    R_ref = odg.rhs(U, st)
    bar, kappa = rhs_bar(U, st, R_ref)
    Rg = _solver(cfg).rhs(U.cuda()).cpu()
    err = rel_err_per_var(Rg, R_ref)
    print(f"err {err.tolist()} bar {bar.tolist()} kappa {kappa.tolist()}", flush=True)
    assert bool((err <= bar).all()), (err.tolist(), bar.tolist())


@pytest.mark.parametrize("kind,over,flux", [MIXED[2], MIXED[3]])
def test_mixed_ends_vjp_matches_oracle_autograd(kind, over, flux):
    cfg = _cfg(kind, over, flux)
    print(f"case mixed ends rhs_vjp {kind} flux {flux}", flush=True)
    st, U = oracle_state(cfg)
    g = torch.Generator().manual_seed(9)
    lamR = torch.randn(U.shape, generator=g, dtype=torch.float64)

    def ref_of(V):
        Vr = V.clone().requires_grad_(True)
        return torch.autograd.grad(odg.rhs(Vr, st), Vr, lamR)[0]

    ref = ref_of(U)
    sens = rel_err_per_var(ref_of(perturbed(U)), ref)
    assert float(sens.max()) < 1e-10, f"test data sits on a derivative kink: {sens.tolist()}"
    got = _solver(cfg).rhs_vjp(U.cuda(), lamR.cuda()).cpu()
    err = rel_err_per_var(got, ref)
    print(f"err {err.tolist()}", flush=True)
    assert float(err.max()) <= 1e-9, err.tolist()


def test_invalid_dirichlet_state_is_rejected():
    from paper_2205_00095_amd.solver import Solver
    cfg = _cfg("wave1d", {"bc": (FIX, 0, 0), "bc_state": {(0, 0): (1.0, 1.2, 0.0, 0.0, 1.0),
                                                          (0, 1): (1.0, 0.0, 0.0, 0.0, 1.0)}}, wl.FLUX_HLL)
    with pytest.raises(Exception):
        Solver(cfg)
    cfg = _cfg("wave1d", {"bc": (wl.PERIODIC, 0, 0), "bc_hi": (R, 0, 0)}, wl.FLUX_HLL)
    with pytest.raises(Exception):
        Solver(cfg)
