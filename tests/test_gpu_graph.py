"""SSP-RK runs captured in a HIP graph (`Solver.graph_run`) against the same runs
launched from the host: every replay, with eager library calls, torch work and
synchronisations between replays, gives bitwise the eager result (each tile's
arithmetic is independent of launch order), including the counters."""
import pytest
import torch

from paper_2205_00095_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _state(kind, **over):
    from paper_2205_00095_amd.solver import Solver
    cfg = wl.make_config(kind, **over)
    s = Solver(cfg)
    rho, v, P = wl.initial_primitives(cfg)
    U = s.set_state(torch.from_numpy(wl.pack_primitives(rho, v, P)).cuda())
    torch.cuda.synchronize()
    return cfg, s, U


@pytest.mark.parametrize("kind,over,nsteps,order", [
    ("wave1d", {}, 10, 3),                                   # the launch-bound 1D wave
    ("kh_tm", {"n_elem": (32, 32, 1)}, 4, 3),                # the TM Kelvin-Helmholtz mesh, smaller
    ("kh_paper", {"nx": 32, "p": 1}, 5, 2),                  # SSPRK2
    ("blast2d", {"n_elem": (32, 32, 1)}, 3, 3),              # with the slope limiter
])
def test_graph_replays_match_eager_runs(kind, over, nsteps, order):
    print(f"case {kind} {over}: {nsteps} steps of order {order}, captured and replayed 3 times", flush=True)
    cfg, s, U0 = _state(kind, **over)
    dt = cfg["dt"]
    # eager reference: 3 consecutive runs of nsteps from U0, with the counters of each
    Ue = U0.clone()
    eager, eager_diag = [], []
    for _ in range(3):
        s.reset_diagnostics()
        s.run(Ue, dt, nsteps, order)
        eager.append(Ue.clone())
        eager_diag.append(s.diagnostics())
    # captured: the graph advances Ug in place
    Ug = U0.clone()
    g = s.graph_run(Ug, dt, nsteps, order)
    torch.cuda.synchronize()
    assert torch.equal(Ug, U0)  # capture launches nothing
    for k in range(3):
        s.reset_diagnostics()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(Ug, eager[k]), f"replay {k}"
        assert s.diagnostics() == eager_diag[k]
        # eager work between replays: a library call and plain torch work
        R = s.rhs(Ug)
        _ = (R * 2.0).sum().item()
        torch.cuda.synchronize()
