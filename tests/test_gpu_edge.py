"""Degenerate mesh shapes against the oracle: a single element (its own periodic
neighbour), meshes one element wide, and tiles left mostly empty by the mesh edge."""
import pytest

from oracle import dg as odg
from oracle import timestep as ots
from paper_2205_00095_amd import workloads as wl

import torch

from ._util import AMPLIFIED_BARS, oracle_state, rel_err_per_var, rhs_bar, step_bar

pytestmark = pytest.mark.gpu

CASES = [
    ("kh_tm", {"n_elem": (1, 1, 1), "bc": (wl.PERIODIC, wl.PERIODIC, wl.PERIODIC)}),
    ("kh_tm", {"n_elem": (1, 7, 1)}),
    ("kh_tm", {"n_elem": (9, 1, 1), "bc": (wl.PERIODIC, wl.REFLECT, wl.PERIODIC)}),
    ("kh_ideal", {"n_elem": (5, 5, 1), "p": 0}),
    ("random3d", {"n_elem": (1, 1, 1), "p": 2}),
    ("random3d", {"n_elem": (4, 1, 3), "p": 3}),
    ("wave1d", {"n_elem": (1, 1, 1)}),
]


@pytest.mark.parametrize("kind,over", CASES)
def test_degenerate_meshes_match_oracle(kind, over):
    from paper_2205_00095_amd.solver import Solver
    cfg = wl.make_config(kind, **over)
    cfg["precision"] = wl.FP64
    print(f"case {kind} {over}", flush=True)
    st, U = oracle_state(cfg)
    R_ref = odg.rhs(U, st)
    bar, kappa = rhs_bar(U, st, R_ref)
    s = Solver(cfg)
    R = s.rhs(U.cuda()).cpu()
    err = rel_err_per_var(R, R_ref)
    print(f"rhs err {err.tolist()} bar {bar.tolist()} kappa {kappa.tolist()}", flush=True)
    assert bool((err <= bar).all()), (err.tolist(), bar.tolist())
    U_ref, bar2, kappa2 = step_bar(U, cfg["dt"], 2, st)
    if kind == "random3d" and over["p"] == 3:
        bar2 = torch.full_like(bar2, AMPLIFIED_BARS["random3d 4x1x3 p=3 2 steps"])
    Ud = U.cuda().contiguous()
    s.run(Ud, cfg["dt"], 2)
    err2 = rel_err_per_var(Ud.cpu(), U_ref)
    print(f"steps err {err2.tolist()} bar {bar2.tolist()} kappa {kappa2.tolist()}", flush=True)
    assert bool((err2 <= bar2).all()), (err2.tolist(), bar2.tolist())
