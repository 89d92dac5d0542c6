"""Degenerate mesh shapes against the oracle: a single element (its own periodic
neighbour), meshes one element wide, and tiles left mostly empty by the mesh edge."""
import pytest

from oracle import dg as odg
from oracle import timestep as ots
from paper_2205_00095_amd import workloads as wl

from ._util import oracle_state, parity_tol, rel_err_per_var

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
    tol, sens = parity_tol(lambda V: odg.rhs(V, st), U)
    s = Solver(cfg)
    R = s.rhs(U.cuda()).cpu()
    err = rel_err_per_var(R, R_ref)
    print(f"rhs err {err.tolist()} tol {tol.tolist()}", flush=True)
    assert bool((err <= tol).all()), (err.tolist(), sens.tolist())
    U_ref = ots.run(U, cfg["dt"], 2, st, phys=True)
    tol2, sens2 = parity_tol(lambda V: ots.run(V, cfg["dt"], 2, st, phys=True), U)
    Ud = U.cuda().contiguous()
    s.run(Ud, cfg["dt"], 2)
    err2 = rel_err_per_var(Ud.cpu(), U_ref)
    print(f"steps err {err2.tolist()} tol {tol2.tolist()}", flush=True)
    assert bool((err2 <= tol2).all()), (err2.tolist(), sens2.tolist())
