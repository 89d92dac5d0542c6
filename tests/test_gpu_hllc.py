"""The HLLC flux on the GPU (Sec. 2.4, the paper's second solver): parity of the RHS and
of SSP-RK steps with the FP64 oracle, the FP32-contraction form against the FP64 path,
an isolated contact that the GPU operator keeps exactly steady (HLL does not), and the
hand-written adjoint of the HLLC flux against the oracle's reverse mode."""
import numpy as np
import pytest
import torch

from oracle import dg as odg
from oracle import timestep as ots
from paper_2205_00095_amd import workloads as wl

from ._util import oracle_state, rel_err_per_var, rhs_bar, step_bar

pytestmark = pytest.mark.gpu

RHS_CASES = [
    ("wave1d", {}),
    ("kh_tm", {"n_elem": (12, 10, 1)}),
    ("kh_tm", {"n_elem": (9, 7, 1), "p": 1, "c": 2.0}),
    ("kh_ideal", {"n_elem": (10, 9, 1)}),
    ("kh_paper", {"nx": 6, "p": 2}),
    ("random3d", {"n_elem": (4, 3, 3), "p": 1}),
]


def _cfg(kind, over, prec=wl.FP64):
    cfg = wl.make_config(kind, **over)
    cfg["precision"] = prec
    cfg["flux"] = wl.FLUX_HLLC
    return cfg


def _solver(cfg, sync=True):
    from paper_2205_00095_amd.solver import Solver
    return Solver(cfg, sync=sync)


@pytest.mark.parametrize("kind,over", RHS_CASES)
def test_hllc_rhs_matches_oracle(kind, over):
    cfg = _cfg(kind, over)
    print(f"case hllc rhs {kind} {over}", flush=True)
    st, U = oracle_state(cfg)
    R_ref = odg.rhs(U, st)
    bar, kappa = rhs_bar(U, st, R_ref)
    s = _solver(cfg)
    R = s.rhs(U.cuda()).cpu()
    err = rel_err_per_var(R, R_ref)
    print(f"err {err.tolist()} bar {bar.tolist()} kappa {kappa.tolist()}", flush=True)
    assert bool((err <= bar).all()), (err.tolist(), bar.tolist())


@pytest.mark.parametrize("kind,over,nsteps,order", [("kh_tm", {"n_elem": (12, 10, 1)}, 4, 3),
                                                    ("kh_paper", {"nx": 6, "p": 1}, 3, 2),
                                                    ("wave1d", {}, 10, 3)])
def test_hllc_steps_match_oracle(kind, over, nsteps, order):
    cfg = _cfg(kind, over)
    print(f"case hllc steps {kind} {over} x{nsteps} order {order}", flush=True)
    st, U = oracle_state(cfg)
    U_ref, bar, kappa = step_bar(U, cfg["dt"], nsteps, st, order=order)
    s = _solver(cfg, sync=False)
    Ud = U.cuda().contiguous()
    s.run(Ud, cfg["dt"], nsteps, order=order)
    err = rel_err_per_var(Ud.cpu(), U_ref)
    print(f"err {err.tolist()} bar {bar.tolist()} kappa {kappa.tolist()}", flush=True)
    assert bool((err <= bar).all()), (err.tolist(), bar.tolist())


def test_hllc_fp32_form_within_bound():
    """FP32 contractions with the HLLC flux: RHS within 1e-5 of the FP64 path."""
    cfg64 = _cfg("kh_tm", {"n_elem": (24, 24, 1)})
    cfg32 = _cfg("kh_tm", {"n_elem": (24, 24, 1)}, prec=wl.FP32_CONTRACT)
    print("case hllc fp32 form 24x24", flush=True)
    st, U = oracle_state(cfg64)
    Ud = U.cuda()
    R64 = _solver(cfg64).rhs(Ud)
    R32 = _solver(cfg32).rhs(Ud)
    err = rel_err_per_var(R32.cpu(), R64.cpu())
    print(f"err {err.tolist()}", flush=True)
    assert float(err.max()) <= 1e-5


def _contact_state(cfg):
    """Piecewise-constant primitives: density 1 / 0.1 and tangential velocity 0.3 / -0.2
    in the left / right half of the periodic x range, zero normal velocity, P = 1 —
    stationary contacts at x = 0.5 and at the periodic wrap."""
    shape = wl.field_shape(cfg)
    nex = cfg["n_elem"][0]
    left = (np.arange(nex) < nex // 2).reshape(1, 1, nex, 1, 1, 1)
    rho = np.broadcast_to(np.where(left, 1.0, 0.1), shape).copy()
    v = np.zeros((2,) + shape)
    v[1] = np.broadcast_to(np.where(left, 0.3, -0.2), shape)
    P = np.ones(shape)
    return wl.pack_primitives(rho, v, P)


@pytest.mark.parametrize("p", [0, 2, 3])
def test_hllc_keeps_an_isolated_contact_steady(p):
    """Exact resolution of contacts (density and tangential-velocity jumps at equal
    pressure and zero normal velocity): every face flux equals the physical flux of
    either side, so the RHS vanishes to rounding with HLLC; HLL diffuses the jump."""
    out = {}
    for flux in (wl.FLUX_HLL, wl.FLUX_HLLC):
        cfg = wl.make_config("kh_ideal", n_elem=(8, 3, 1), p=p, bc=(wl.PERIODIC, wl.PERIODIC, wl.PERIODIC))
        cfg["flux"] = flux
        print(f"case contact p {p} flux {flux}", flush=True)
        s = _solver(cfg)
        U = s.set_state(torch.from_numpy(_contact_state(cfg)).cuda())
        R = s.rhs(U)
        scale = 2.0 / (1.0 / 8) * 1.0  # (2/dx) P: the size of one face flux term
        out[flux] = float(R.abs().max()) / scale
    print(f"max |R| / ((2/dx) P): HLL {out[wl.FLUX_HLL]:.3e} HLLC {out[wl.FLUX_HLLC]:.3e}", flush=True)
    assert out[wl.FLUX_HLLC] <= 1e-13 * (p + 1) ** 2
    assert out[wl.FLUX_HLL] > 1e-3


def _lam(shape, seed):
    g = torch.Generator().manual_seed(seed)
    return torch.randn(shape, generator=g, dtype=torch.float64)


def _perturbed_sensitivity(fn, U):
    from ._util import perturbed
    return rel_err_per_var(fn(perturbed(U)), fn(U))


VJP_CASES = [("kh_ideal", {"n_elem": (6, 5, 1), "init": "kh"}), ("kh_tm", {"n_elem": (5, 4, 1)}),
             ("wave1d", {"n_elem": (20, 1, 1)}), ("random3d", {"n_elem": (3, 2, 2), "p": 1}),
             ("kh_ideal", {"n_elem": (5, 4, 1), "p": 3, "init": "kh"})]


@pytest.mark.parametrize("kind,over", VJP_CASES)
def test_hllc_rhs_vjp_matches_oracle_autograd(kind, over):
    """dg_rhs_vjp with HLLC against the oracle's reverse mode (autograd through its HLLC)."""
    cfg = _cfg(kind, over)
    print(f"case hllc rhs_vjp {kind} {over}", flush=True)
    st, U = oracle_state(cfg)
    lamR = _lam(U.shape, 7)

    def ref_of(V):
        Vr = V.clone().requires_grad_(True)
        return torch.autograd.grad(odg.rhs(Vr, st), Vr, lamR)[0]

    ref = ref_of(U)
    sens = _perturbed_sensitivity(ref_of, U)
    assert float(sens.max()) < 1e-10, f"test data sits on a derivative kink: {sens.tolist()}"
    got = _solver(cfg).rhs_vjp(U.cuda(), lamR.cuda()).cpu()
    err = rel_err_per_var(got, ref)
    print(f"err {err.tolist()}", flush=True)
    assert float(err.max()) <= 1e-9, err.tolist()


@pytest.mark.parametrize("kind,over", [("kh_ideal", {"n_elem": (6, 5, 1), "init": "kh"}),
                                       ("kh_tm", {"n_elem": (4, 4, 1)})])
def test_hllc_step_vjp_matches_oracle_autograd(kind, over):
    cfg = _cfg(kind, over)
    print(f"case hllc step_vjp {kind} {over}", flush=True)
    st, U = oracle_state(cfg)
    lam = _lam(U.shape, 11)
    Ur = U.clone().requires_grad_(True)
    (ref,) = torch.autograd.grad(ots.step(Ur, cfg["dt"], st), Ur, lam)
    got = _solver(cfg).step_vjp(U.cuda(), cfg["dt"], lam.cuda()).cpu()
    err = rel_err_per_var(got, ref)
    print(f"err {err.tolist()}", flush=True)
    assert float(err.max()) <= 1e-9, err.tolist()


def test_hllc_fullsize_rhs():
    """The 256x256 p=3 Taub-Matthews Kelvin-Helmholtz mesh, every output against the
    (vectorised) oracle, in the launch configuration of the benchmark."""
    cfg = _cfg("kh_tm", {})
    print(f"case hllc fullsize {cfg['n_elem']}", flush=True)
    st, U = oracle_state(cfg)
    R_ref = odg.rhs(U, st)
    bar, kappa = rhs_bar(U, st, R_ref)
    R = _solver(cfg, sync=False).rhs(U.cuda()).cpu()
    err = rel_err_per_var(R, R_ref)
    print(f"err {err.tolist()} bar {bar.tolist()} kappa {kappa.tolist()}", flush=True)
    assert bool((err <= bar).all()), (err.tolist(), bar.tolist())


def test_hllc_trajectory_gradient_matches_oracle():
    """dJ/d(initial primitives) through 4 HLLC steps (checkpoint every 3) against the
    oracle's reverse mode through its HLLC."""
    from oracle import objective as oobj
    from oracle import srhd as osrhd
    from oracle.setup import Setup
    from paper_2205_00095_amd.adjoint import vy2_after
    cfg = _cfg("kh_ideal", {"n_elem": (4, 4, 1)})
    print("case hllc trajectory gradient", flush=True)
    st = Setup.from_config(cfg)
    rho, v, P = wl.initial_primitives(cfg)
    v = v.copy()
    v[1] += wl.kh_perturbation(cfg)
    src = torch.from_numpy(wl.pack_primitives(rho, v, P))
    dt = cfg["dt"] * 10
    s_r = src.clone().requires_grad_(True)
    U = osrhd.prim3_to_cons(s_r[0], s_r[1:3], s_r[3], st)
    Jref = oobj.vy2_integral(ots.run(U, dt, 4, st), st)
    (gref,) = torch.autograd.grad(Jref, s_r)
    sd = src.cuda().requires_grad_(True)
    J = vy2_after(_solver(cfg), sd, 4, dt, k=3)
    J.backward()
    assert abs(float(J) - float(Jref)) <= 1e-12 * abs(float(Jref))
    err = rel_err_per_var(sd.grad.cpu(), gref)
    print(f"err {err.tolist()}", flush=True)
    assert float(err.max()) <= 1e-9
