"""The slope limiter on the GPU (reading R29: minmod-bounded slopes applied as one
scaling factor per element, after every SSP-RK stage and before the physicality
operator; oracle/limiter.py).

Parity: limited SSP-RK steps of the paper's 1D Riemann problems (Sec. 4), its 2D
Riemann test 1 and a 3D spherical blast, each step started from the oracle's own
state, element by element within the step bar (the blast at rest within the fixed bar of
tests/_util.AMPLIFIED_BARS: there the oracle's own step moves by up to 1.2e-12 when its
input moves by one ulp, as the limiter's factor is a ratio of differences of
nearly equal averages), with the same numbers of limited,
flagged and smoothed elements as the oracle's step (elements whose limiter decision
sits within rounding of the guard threshold may differ; the tests count them on the
oracle side and allow that many).

Shock runs: the problems the operator alone could not carry at p >= 1 (the strong
blast wave, the reflecting wall) run with the limiter to the paper's final times at
p = 1 and 2 without a failed recovery or an inadmissible average, and converge."""
import math

import numpy as np
import pytest
import torch

from oracle import dg as odg
from oracle import limiter as olim
from oracle import srhd
from oracle import timestep as ots
from oracle.setup import Setup
from paper_2205_00095_amd import workloads as wl

from ._util import AMPLIFIED_BARS, rel_err_per_var, step_bar

pytestmark = pytest.mark.gpu


def _near_ties(V, st):
    """Elements of V whose limiter decision (some pair's |s - s~| against the guard
    EPS * scale) lies within rounding of the threshold."""
    w = odg.elem_weights(st)
    avg = olim.averages(V, st)
    sig = olim.scales(avg, st)
    amb = torch.zeros(avg.shape[1:], dtype=torch.bool)
    for d in range(st.dim):
        s = olim._slope(V, w, olim._xi(st, d), d)
        sl = olim._minmod(s, olim._neighbour_average(avg, d, +1, st) - avg,
                          avg - olim._neighbour_average(avg, d, -1, st))
        gap = ((s - sl).abs() - olim.EPS * sig).abs()
        amb |= (gap <= 1e-13 * sig).any(0)
    return int(amb.sum())


def _riemann_1d(prob, N, p, bc=None):
    from ._exact import riemann_problem
    L, R, gam, t, _ = riemann_problem(prob)
    cfg = wl.make_config("wave1d", n_elem=(N, 1, 1), p=p, bc=(wl.OUTFLOW,) * 3, gamma_ad=gam)
    cfg["flux"] = wl.FLUX_HLLC
    cfg["limiter"] = 1
    xi, _ = np.polynomial.legendre.leggauss(p + 1)
    x = (np.arange(N)[:, None] + 0.5 * (xi[None, :] + 1.0)) / N
    shape = wl.field_shape(cfg)
    pick = lambda a, b: np.where(x < 0.5, a, b).reshape(shape)  # noqa: E731
    prims = wl.pack_primitives(pick(L[0], R[0]), pick(L[1], R[1])[None], pick(L[2], R[2]))
    return cfg, prims, t


def _riemann_2d(N, p):
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "riemann_problems_2d.txt")
    with open(path) as fh:
        rows = [ln.split() for ln in fh if ln.strip() and not ln.startswith("#")]
    quads = {int(r[1]): [float(v) for v in r[2:]] for r in rows if int(r[0]) == 1}
    cfg = wl.make_config("kh_ideal", n_elem=(N, N, 1), p=p, lo=(-1.0, -1.0, 0.0), hi=(1.0, 1.0, 1.0),
                         bc=(wl.OUTFLOW,) * 3, gamma_ad=5.0 / 3.0)
    cfg.update(flux=wl.FLUX_HLLC, precision=wl.FP64, limiter=1)
    xi, _ = np.polynomial.legendre.leggauss(p + 1)
    c = -1.0 + 2.0 * (np.arange(N)[:, None] + 0.5 * (xi[None, :] + 1.0)) / N
    X, Y = np.broadcast_arrays(c[None, :, None, :], c[:, None, :, None])
    quad = np.where(X >= 0, np.where(Y >= 0, 1, 4), np.where(Y >= 0, 2, 3))
    shape = wl.field_shape(cfg)
    f = [np.choose(quad - 1, [quads[q][k] for q in (1, 2, 3, 4)]).reshape(shape) for k in range(4)]
    return cfg, wl.pack_primitives(f[0], np.stack([f[1], f[2]]), f[3])


def _blast_3d(N, p):
    """Pressure 100 inside a sphere of radius 0.3 about the centre of the unit cube, 0.1
    outside, density 1, at rest; ideal gas Gamma = 5/3, outflow boundaries."""
    cfg = wl.make_config("random3d", n_elem=(N, N, N), p=p, bc=(wl.OUTFLOW,) * 3, gamma_ad=5.0 / 3.0)
    cfg.update(flux=wl.FLUX_HLLC, precision=wl.FP64, limiter=1)
    X = wl.node_coords(cfg)
    r2 = sum((X[d] - 0.5) ** 2 for d in range(3))
    shape = wl.field_shape(cfg)
    P = np.where(r2 < 0.09, 100.0, 0.1).reshape(shape)
    return cfg, wl.pack_primitives(np.ones(shape), np.zeros((3,) + shape), P)


def _workload(kind, **over):
    cfg = wl.make_config(kind, **over)
    rho, v, P = wl.initial_primitives(cfg)
    return cfg, wl.pack_primitives(rho, v, P)


CASES = {
    # name: (builder, SSP-RK order, steps, fixed bar or None)
    "problem 4 N=64 p=1": (lambda: _riemann_1d(4, 64, 1)[:2], 2, 8, None),
    "problem 2 N=64 p=2": (lambda: _riemann_1d(2, 64, 2)[:2], 3, 8, None),
    "problem 1 N=48 p=3": (lambda: _riemann_1d(1, 48, 3)[:2], 3, 6, None),
    "2D test 1 16x16 p=1": (lambda: _riemann_2d(16, 1), 2, 4, None),
    "3D blast 6^3 p=1": (lambda: _blast_3d(6, 1), 2, 3, None),
    "3D blast 4^3 p=2": (lambda: _blast_3d(4, 2), 3, 2, None),
    # the benchmark's cylindrical blast at a size the oracle finishes in seconds
    "blast2d 24x24 p=2": (lambda: _workload("blast2d", n_elem=(24, 24, 1)), 3, 3,
                          AMPLIFIED_BARS["blast2d 24x24 p=2 limited step"]),
    # the Taub-Matthews recovery inside the limiter kernel (1-ulp response 4e-14)
    "blast2d TM 16x16 p=3": (lambda: _workload("blast2d", n_elem=(16, 16, 1), p=3, eos=wl.EOS_TM), 3, 3, None),
}


@pytest.mark.parametrize("case", list(CASES))
def test_limited_steps_match_oracle(case, monkeypatch):
    from paper_2205_00095_amd.solver import Solver
    build, order, nsteps, fixed = CASES[case]
    cfg, prims = build()
    st = Setup.from_config(cfg)
    assert st.limiter == 1
    P = torch.from_numpy(prims)
    nv = st.nvar
    U = srhd.prim3_to_cons(P[0], P[1:nv - 1], P[nv - 1], st).contiguous()
    dt = cfg["dt"]
    ties = [0]
    limit0 = olim.limit

    def counting(V, st_, stats=None):
        ties[0] += _near_ties(V, st_)
        return limit0(V, st_, stats)
    monkeypatch.setattr(olim, "limit", counting)
    s = Solver(cfg, sync=False)
    total = 0
    for k in range(nsteps):
        print(f"case {case}: step {k} from the oracle's state (order {order}, dt {dt:.3e})", flush=True)
        stats = {}
        ties[0] = 0
        U_next = ots.step(U, dt, st, phys=True, stats=stats, order=order)
        n_ties = ties[0]
        _, bar, kappa = step_bar(U, dt, 1, st, order=order)
        if fixed is not None:
            bar = torch.clamp(bar, min=fixed)
        Ud = U.cuda().contiguous()
        s.reset_diagnostics()
        s.step(Ud, dt, order=order)
        d = s.diagnostics()
        err = rel_err_per_var(Ud.cpu(), U_next)
        print(f"err {err.tolist()} bar {bar.tolist()} gpu {d} oracle {stats} near ties {n_ties}", flush=True)
        assert bool((err <= bar).all()), (err.tolist(), bar.tolist())
        assert abs(d["limited"] - stats.get("limited", 0)) <= n_ties
        assert d["flagged"] == stats.get("flagged", 0) and d["smoothed"] == stats.get("smoothed", 0)
        assert d["c2p_fail"] == 0 and d["bad_average"] == stats.get("bad_average", 0) == 0
        total += stats.get("limited", 0)
        U = U_next
    assert total > 0  # the limiter acted in every case


@pytest.mark.parametrize("order", [3, 2])
def test_limited_steps_through_an_inadmissible_element(order, monkeypatch):
    """One element of the blast with D = -1 at every node: its recovery fails in every
    stage (the floor state, counted), the stage launch marks those nodes, the limiter
    launch leaves the element unchanged (its average is inadmissible, counted) and
    recovers the marked nodes again from the usual start (failing again, counted).  Two
    steps from the oracle's state each: the state within the step bar (the oracle's
    1-ulp response here is at most 3.1e-13), and 9 failed recoveries and one
    inadmissible average per stage, as in the oracle."""
    from paper_2205_00095_amd.solver import Solver
    cfg, prims = _workload("blast2d", n_elem=(12, 12, 1))
    st = Setup.from_config(cfg)
    P = torch.from_numpy(prims)
    nv = st.nvar
    U = srhd.prim3_to_cons(P[0], P[1:nv - 1], P[nv - 1], st).contiguous()
    U[0, 0, 6, 5] = -1.0
    dt = cfg["dt"]
    ties = [0]
    limit0 = olim.limit

    def counting(V, st_, stats=None):
        ties[0] += _near_ties(V, st_)
        return limit0(V, st_, stats)
    monkeypatch.setattr(olim, "limit", counting)
    s = Solver(cfg, sync=False)
    for k in range(2):
        print(f"case inadmissible element, order {order}: step {k} from the oracle's state", flush=True)
        stats = {}
        ties[0] = 0
        U_next = ots.step(U, dt, st, phys=True, stats=stats, order=order)
        _, bar, _ = step_bar(U, dt, 1, st, order=order)
        Ud = U.cuda().contiguous()
        s.reset_diagnostics()
        s.step(Ud, dt, order=order)
        d = s.diagnostics()
        err = rel_err_per_var(Ud.cpu(), U_next)
        print(f"err {err.tolist()} bar {bar.tolist()} gpu {d} oracle {stats}", flush=True)
        assert bool((err <= bar).all()), (err.tolist(), bar.tolist())
        assert d["c2p_fail"] == stats["c2p_fail"] == 9 * order
        assert d["bad_average"] == stats["bad_average"] == order
        assert d["flagged"] == stats["flagged"] and d["smoothed"] == stats.get("smoothed", 0)
        assert abs(d["limited"] - stats.get("limited", 0)) <= ties[0]
        assert float(U_next[0, 0, 6, 5].max()) < 0.0  # the element is still inadmissible
        U = U_next


def test_fp32_form_with_the_limiter():
    """The FP32-contraction form under the limiter (the limiter itself, the operator and
    the recovery stay FP64): 20 steps of the 48x48 p=3 blast stay admissible and within
    1e-5 (L1, relative) of the FP64 run; the matrix-core sweeps give the vector form's
    result bit for bit."""
    from paper_2205_00095_amd.solver import Solver
    out = []
    for prec in (wl.FP64, wl.FP32_CONTRACT, wl.FP32_MFMA):
        cfg, prims = _workload("blast2d", n_elem=(48, 48, 1), p=3, precision=prec)
        s = Solver(cfg)
        U = s.set_state(torch.from_numpy(prims).cuda())
        s.run(U, cfg["dt"], 20)
        d = s.diagnostics()
        print(f"precision {prec}: {d}", flush=True)
        assert d["c2p_fail"] == 0 and d["bad_average"] == 0 and d["limited"] > 0
        out.append(U.cpu())
    rel = float((out[1] - out[0]).abs().sum() / out[0].abs().sum())
    print(f"L1 relative difference FP32 form vs FP64: {rel:.2e}", flush=True)
    assert rel <= 1e-5
    assert torch.equal(out[2], out[1])


DEGENERATE = [
    ("kh_tm", {"n_elem": (1, 1, 1), "bc": (wl.PERIODIC, wl.PERIODIC, wl.PERIODIC)}),
    ("kh_tm", {"n_elem": (1, 7, 1)}),
    ("kh_tm", {"n_elem": (9, 1, 1), "bc": (wl.PERIODIC, wl.REFLECT, wl.PERIODIC)}),
    ("wave1d", {"n_elem": (1, 1, 1)}),
    ("wave1d", {"n_elem": (3, 1, 1), "p": 1}),
]


@pytest.mark.parametrize("kind,over", DEGENERATE)
def test_limiter_on_degenerate_meshes(kind, over):
    """Two limited SSP-RK3 steps on a single element (its own periodic neighbour on every
    side), meshes one element wide and mostly empty tiles, against the oracle, with the
    same number of limited elements."""
    from paper_2205_00095_amd.solver import Solver
    from ._util import oracle_state
    cfg = wl.make_config(kind, **over)
    cfg.update(precision=wl.FP64, limiter=1)
    print(f"case {kind} {over} with the limiter", flush=True)
    st, U = oracle_state(cfg)
    stats = {}
    U_ref = U
    for _ in range(2):
        U_ref = ots.step(U_ref, cfg["dt"], st, stats=stats)
    _, bar, _ = step_bar(U, cfg["dt"], 2, st)
    if kind == "kh_tm" and over["n_elem"] == (1, 1, 1):
        bar = torch.clamp(bar, min=AMPLIFIED_BARS["kh_tm 1x1 p=3 limited 2 steps"])
    s = Solver(cfg)
    Ud = U.cuda().contiguous()
    s.run(Ud, cfg["dt"], 2)
    d = s.diagnostics()
    err = rel_err_per_var(Ud.cpu(), U_ref)
    print(f"err {err.tolist()} bar {bar.tolist()} gpu {d} oracle {stats}", flush=True)
    assert bool((err <= bar).all()), (err.tolist(), bar.tolist())
    assert d["limited"] == stats.get("limited", 0) and d["c2p_fail"] == 0


def test_order_zero_ignores_the_limiter():
    """At p = 0 the limiter has nothing to limit: a run with it is bit-identical to one without."""
    from paper_2205_00095_amd.solver import Solver
    cfg, prims, _ = _riemann_1d(2, 200, 0)
    out = []
    for lim in (0, 1):
        c = dict(cfg, limiter=lim)
        s = Solver(c)
        U = s.set_state(torch.from_numpy(prims).cuda())
        s.run(U, 0.1 / 200, 100, order=1)
        assert s.diagnostics()["limited"] == 0
        out.append(U.cpu())
    assert torch.equal(out[0], out[1])


def test_stepping_adjoints_reject_the_limiter():
    from paper_2205_00095_amd import _lib
    from paper_2205_00095_amd.solver import Solver
    cfg, prims, _ = _riemann_1d(4, 32, 1)
    s = Solver(cfg)
    U = s.set_state(torch.from_numpy(prims).cuda())
    lam = torch.ones_like(U)
    with pytest.raises(_lib.DGError, match="limiter"):
        s.step_vjp(U, cfg["dt"], lam)
    tape = torch.empty(s.tape_numel, dtype=torch.float64, device=U.device)
    with pytest.raises(_lib.DGError, match="limiter"):
        s.step_tape(U, cfg["dt"], tape)
    # the right-hand side and its adjoint do not involve the limiter
    s.rhs(U)
    s.rhs_vjp(U, lam)


def _l1_D(prob, N, p):
    """L1 error of D (Gauss-Legendre quadrature of the nodal values) against the exact
    solution at the paper's final time, limiter and operator on, SSP-RK order p + 1."""
    from paper_2205_00095_amd.solver import Solver
    from ._exact import riemann_exact, riemann_problem
    cfg, prims, t = _riemann_1d(prob, N, p)
    L, R, gam, _, _ = riemann_problem(prob)
    s = Solver(cfg)
    U = s.set_state(torch.from_numpy(prims).cuda())
    dt = 0.1 / (2 * p + 1) / N
    n = int(round(t / dt))
    s.run(U, dt, n, order=min(p + 1, 3))
    d = s.diagnostics()
    xi, w = np.polynomial.legendre.leggauss(p + 1)
    x = (np.arange(N)[:, None] + 0.5 * (xi[None, :] + 1.0)) / N
    rho, v, _ = riemann_exact(L, R, gam)["profile"]((x - 0.5) / (n * dt))
    De = rho / np.sqrt(1.0 - v * v)
    D = U[0].cpu().reshape(N, p + 1).numpy()
    return float((np.abs(D - De) * w[None, :]).sum() / (2 * N)), d


@pytest.mark.parametrize("prob,factor", [(1, 0.9), (2, 0.97), (4, 0.9)])
@pytest.mark.parametrize("p", [1, 2])
def test_paper_riemann_problems_with_the_limiter(prob, factor, p):
    """The paper's 1D Riemann problems 1, 2 (strong blast wave, pressure ratio 1e5) and 4
    at p = 1 and 2 with the limiter and the operator, 200 and 400 cells to t = 0.4: no
    failed recovery, no inadmissible average, and the L1 error of D falls with the mesh
    width by at least the factor given (problem 2's thin dense shell is far from
    resolved at these widths and its error falls slowly, as the paper reports for it;
    measured 0.643 -> 0.606 at p = 1)."""
    print(f"case Riemann problem {prob} at p = {p} with the limiter", flush=True)
    e1, d1 = _l1_D(prob, 200, p)
    e2, d2 = _l1_D(prob, 400, p)
    print(f"problem {prob} p {p}: L1(D) {e1:.4e} -> {e2:.4e}; diagnostics {d2}", flush=True)
    for d in (d1, d2):
        assert d["c2p_fail"] == 0 and d["bad_average"] == 0 and d["limited"] > 0
    assert e2 < factor * e1, (e1, e2)


@pytest.mark.parametrize("p", [1, 2])
def test_paper_wall_problem_with_the_limiter(p):
    """The paper's reflecting-wall problem (Sec. 4, its fifth 1D problem, 0.99999c into
    a wall at x = 1, P = 0.01, Gamma = 4/3, t = 1.5) at p = 1 and 2 with the limiter: the
    stopped gas behind the reflected shock has the Rankine-Hugoniot density and pressure
    and the shock sits where their speed puts it."""
    from paper_2205_00095_amd.solver import Solver
    from ._exact import jump_state, paper_wall_problem
    c = paper_wall_problem()
    V, rho2, P2, D1 = jump_state(c["gam"], c["v"], c["rho"], c["P"])
    N = 400
    cfg = wl.make_config("wave1d", n_elem=(N, 1, 1), p=p, bc=(wl.DIRICHLET, 0, 0), bc_hi=(wl.REFLECT, 0, 0),
                         gamma_ad=c["gam"], bc_state={(0, 0): (c["rho"], c["v"], 0.0, 0.0, c["P"])})
    cfg.update(flux=wl.FLUX_HLLC, limiter=1)
    print(f"case paper wall problem at p = {p} with the limiter", flush=True)
    shape = wl.field_shape(cfg)
    s = Solver(cfg)
    U = s.set_state(torch.from_numpy(wl.pack_primitives(np.full(shape, c["rho"]), np.full((1,) + shape, c["v"]),
                                                        np.full(shape, c["P"]))).cuda())
    dt = 0.1 / (2 * p + 1) / N
    n = int(round(c["t"] / dt))
    s.run(U, dt, n, order=p + 1)
    d = s.diagnostics()
    assert d["c2p_fail"] == 0 and d["bad_average"] == 0
    W = s.con2prim(U).cpu().reshape(3, N, p + 1).numpy().mean(2)
    D = U[0].cpu().reshape(N, p + 1).numpy().mean(1)
    x = (np.arange(N) + 0.5) / N
    xs = 1.0 + V * n * dt
    L = 1.0 - xs
    plateau = (x > xs + 0.2 * L) & (x < 1.0 - 0.2 * L)
    rho_p, P_p = W[0][plateau].mean(), W[2][plateau].mean()
    shock = x[np.where(D > 0.5 * (D1 + rho2))[0].min()]
    print(f"plateau rho {rho_p:.6f} (exact {rho2:.6f}) P {P_p:.6f} (exact {P2:.6f}); shock at {shock:.5f} "
          f"(exact {xs:.5f}); diagnostics {d}", flush=True)
    assert abs(rho_p / rho2 - 1.0) <= 1e-2
    assert abs(P_p / P2 - 1.0) <= 1e-3
    assert abs(shock - xs) <= 2.0 / N
    assert math.isfinite(rho_p)
