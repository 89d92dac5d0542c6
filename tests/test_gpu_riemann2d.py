"""The paper's 2D Riemann problems (Sec. 4, 2D Riemann problems, tests 1-3: four
quadrant states, Gamma = 5/3, outflow boundaries, t = 0.8;
tests/golden/riemann_problems_2d.txt) on the GPU: parity with the oracle over the first
steps, each step started from the oracle's own state (the flow is chaotic at the jumps:
two runs that differ by rounding drift apart by ~1e-5 in six steps, so a whole-run
comparison cannot separate a kernel error from that drift), and full runs at p = 0 and p = 1 (physicality operator on, no limiter) staying
admissible, and for tests 1 and 3, whose initial data are symmetric about the diagonal
(quadrants 2 and 4 mirror images), staying symmetric."""
import os

import numpy as np
import pytest
import torch

from oracle import timestep as ots
from paper_2205_00095_amd import workloads as wl

from ._util import AMPLIFIED_BARS, rel_err_per_var, step_bar

pytestmark = pytest.mark.gpu


GAMMA, T_FINAL = 5.0 / 3.0, 0.8


def _problem(test):
    path = os.path.join(os.path.dirname(__file__), "golden", "riemann_problems_2d.txt")
    with open(path) as fh:
        rows = [ln.split() for ln in fh if ln.strip() and not ln.startswith("#")]
    return {int(r[1]): [float(v) for v in r[2:]] for r in rows if int(r[0]) == test}


def _setup(N, p, test=1):
    quads, gam, t = _problem(test), GAMMA, T_FINAL
    cfg = wl.make_config("kh_ideal", n_elem=(N, N, 1), p=p, lo=(-1.0, -1.0, 0.0), hi=(1.0, 1.0, 1.0),
                         bc=(wl.OUTFLOW,) * 3, gamma_ad=gam)
    cfg["flux"] = wl.FLUX_HLLC
    cfg["precision"] = wl.FP64
    xi, _ = np.polynomial.legendre.leggauss(p + 1)
    c = -1.0 + 2.0 * (np.arange(N)[:, None] + 0.5 * (xi[None, :] + 1.0)) / N  # [element, node]
    X, Y = np.broadcast_arrays(c[None, :, None, :], c[:, None, :, None])    # [ey, ex, j, i]
    quad = np.where(X >= 0, np.where(Y >= 0, 1, 4), np.where(Y >= 0, 2, 3))
    shape = wl.field_shape(cfg)
    field = [np.choose(quad - 1, [quads[q][k] for q in (1, 2, 3, 4)]).reshape(shape) for k in range(4)]
    prims = wl.pack_primitives(field[0], np.stack([field[1], field[2]]), field[3])
    return cfg, prims, t


def test_first_steps_match_oracle():
    """Six SSPRK2 steps of test 1 at 16x16 p=1, each from the oracle's state, with the same
    numbers of flagged and smoothed elements and of trace fallbacks as the oracle's step.
    The operator smooths up to 30 elements per step here and amplifies rounding: a 1-ulp
    change of the input moves the oracle's step by up to 2.6e-12, above the
    cancellation-based bar (1e-12), so the fixed bar of tests/_util.AMPLIFIED_BARS holds."""
    from oracle import srhd
    from oracle.setup import Setup
    from paper_2205_00095_amd.solver import Solver
    cfg, prims, _ = _setup(16, 1)
    st = Setup.from_config(cfg)
    P = torch.from_numpy(prims)
    U = srhd.prim3_to_cons(P[0], P[1:3], P[3], st).contiguous()
    s = Solver(cfg, sync=False)
    for k in range(6):
        print(f"case 2D Riemann test 1, 16x16 p=1, step {k} from the oracle's state", flush=True)
        stats = {}
        U_next = ots.step(U, cfg["dt"], st, phys=True, stats=stats, order=2)
        _, bar, kappa = step_bar(U, cfg["dt"], 1, st, order=2)
        bar = torch.clamp(bar, min=AMPLIFIED_BARS["riemann2d test 1 16x16 p=1 step"])
        Ud = U.cuda().contiguous()
        s.reset_diagnostics()
        s.step(Ud, cfg["dt"], order=2)
        d = s.diagnostics()
        err = rel_err_per_var(Ud.cpu(), U_next)
        print(f"err {err.tolist()} bar {bar.tolist()} kappa {kappa.tolist()} gpu {d} oracle {stats}", flush=True)
        assert bool((err <= bar).all()), (err.tolist(), bar.tolist())
        assert d["flagged"] == stats.get("flagged", 0) and d["smoothed"] == stats.get("smoothed", 0)
        assert d["trace_fallback"] == stats.get("trace_fallbacks", 0)
        assert d["bad_average"] == stats.get("bad_average", 0) == 0
        U = U_next


@pytest.mark.parametrize("test", [1, 2, 3])
@pytest.mark.parametrize("N,p", [(256, 0), (128, 1)])
def test_full_run_admissible_and_symmetric(N, p, test):
    from paper_2205_00095_amd.solver import Solver
    cfg, prims, t = _setup(N, p, test)
    print(f"case 2D Riemann test {test}, {N}x{N} p={p} to t={t}", flush=True)
    s = Solver(cfg)
    U = s.set_state(torch.from_numpy(prims).cuda())
    dt = 0.1 / (2 * p + 1) * (2.0 / N)
    n = int(round(t / dt))
    s.run(U, dt, n, order=min(p + 1, 3))
    d = s.diagnostics()
    print(f"{n} steps, diagnostics {d}", flush=True)
    assert d["c2p_fail"] == 0 and d["bad_average"] == 0
    if p > 0 and test == 1:
        assert d["smoothed"] > 0  # the operator is what keeps p = 1 admissible here
    if test == 2:
        return  # no mirror symmetry in this one
    Uc = U.cpu()[:, 0, :, :, 0]  # [var, ey, ex, j, i]
    Ut = Uc.permute(0, 2, 1, 4, 3)
    mirror = torch.stack([Ut[0], Ut[2], Ut[1], Ut[3]])  # swap x and y, and S_x with S_y
    asym = float((Uc - mirror).abs().max() / Uc.abs().max())
    print(f"asymmetry about the diagonal {asym:.2e}", flush=True)
    # p = 0: symmetric to rounding; p = 1: the trace fallbacks and the operator take
    # discrete per-element decisions (thresholds, argmin) that turn rounding differences
    # between the x and y sweeps into small asymmetries, still far below the flow's scales
    assert asym <= (1e-12 if p == 0 else 1e-4)
