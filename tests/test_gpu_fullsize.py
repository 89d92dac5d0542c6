"""Full-size parity in the launch configuration the benchmark times, and the
FP32-contraction form's error against the FP64 oracle.

Full-size meshes: Kelvin-Helmholtz 256x256 p=3 (TM, FP64), 512x512 p=3 (TM,
FP32 contractions), 128x128 p=2 (ideal, FP64), and the 3D 64^3 p=2 random
stress field (FP32 contractions, physicality operator on).  The oracle is
vectorised, so it evaluates every output at these sizes.

FP32-contraction bar: <= 1e-5 normwise relative per conserved component on the
RHS (the volume and lift contractions run in FP32 with FP32 accumulation on
deviations from an FP64 reference per line of nodes; the traces and everything
else are FP64)."""
import pytest
import torch

from oracle import dg as odg
from oracle import timestep as ots
from paper_2205_00095_amd import workloads as wl

from ._util import oracle_state, rel_err_per_var, rhs_bar, step_bar

pytestmark = pytest.mark.gpu


def _solver(cfg, sync=False):
    from paper_2205_00095_amd.solver import Solver
    return Solver(cfg, sync=sync)


@pytest.mark.parametrize("kind,prec", [("kh_tm", wl.FP64), ("kh_ideal", wl.FP64), ("kh_tm_fp32", wl.FP64)])
def test_fullsize_rhs_fp64(kind, prec):
    cfg = wl.make_config(kind, precision=prec)
    print(f"case {kind} n_elem={cfg['n_elem']} p={cfg['p']}", flush=True)
    st, U = oracle_state(cfg)
    R_ref = odg.rhs(U, st)
    bar, kappa = rhs_bar(U, st, R_ref)
    R = _solver(cfg).rhs(U.cuda()).cpu()
    err = rel_err_per_var(R, R_ref)
    print(f"err {err.tolist()} bar {bar.tolist()} kappa {kappa.tolist()}", flush=True)
    assert bool((err <= bar).all()), (err.tolist(), bar.tolist())


def test_fullsize_step_kh_tm():
    """One SSP-RK3 step of the 256x256 p=3 TM Kelvin-Helmholtz mesh (the benchmark kernel)."""
    cfg = wl.make_config("kh_tm")
    st, U = oracle_state(cfg)
    U_ref, bar, kappa = step_bar(U, cfg["dt"], 1, st)
    s = _solver(cfg)
    Ud = U.cuda().contiguous()
    s.run(Ud, cfg["dt"], 1)
    err = rel_err_per_var(Ud.cpu(), U_ref)
    print(f"err {err.tolist()} bar {bar.tolist()} kappa {kappa.tolist()}", flush=True)
    assert bool((err <= 1e-12).all()), err.tolist()
    d = s.diagnostics()
    assert d["c2p_fail"] == 0 and d["flagged"] == 0 and d["trace_fallback"] == 0


@pytest.mark.parametrize("kind,over,prec", [("kh_tm_fp32", {}, wl.FP32_CONTRACT), ("kh_tm", {"n_elem": (12, 10, 1)}, wl.FP32_CONTRACT),
                                            ("kh_ideal", {"n_elem": (10, 9, 1)}, wl.FP32_CONTRACT),
                                            ("random3d", {"n_elem": (5, 4, 3)}, wl.FP32_CONTRACT),
                                            ("kh_tm_fp32", {}, wl.FP32_MFMA), ("kh_tm", {"n_elem": (12, 10, 1)}, wl.FP32_MFMA),
                                            ("kh_ideal", {"n_elem": (11, 9, 1), "p": 3}, wl.FP32_MFMA)])
def test_fp32_contraction_rhs_error(kind, over, prec):
    """FP32 form (sweeps on the vector ALUs, or on the matrix cores) against the FP64 oracle."""
    cfg = wl.make_config(kind, **over)
    cfg["precision"] = prec
    st, U = oracle_state(cfg)
    R_ref = odg.rhs(U, st)
    R = _solver(cfg).rhs(U.cuda()).cpu()
    err = rel_err_per_var(R, R_ref)
    print(f"{kind} {over} precision {prec}: FP32-contraction RHS error {err.tolist()}", flush=True)
    assert float(err.max()) <= 1e-5, err.tolist()


def test_fp32_contraction_uniform_state():
    cfg = wl.make_config("kh_tm", n_elem=(6, 5, 1), precision=wl.FP32_CONTRACT, bc=(0, 0, 0))
    st, U = oracle_state(cfg)
    U = U[:, :, :1, :1, :, :1, :1].expand_as(U).contiguous()
    R = _solver(cfg).rhs(U.cuda()).cpu()
    scale = 2 * cfg["n_elem"][0] * float(U.abs().max())
    assert float(R.abs().max()) <= 1e-14 * scale


def test_fullsize_random3d_rhs_fp32():
    """64^3 p=2 random stress field, FP32-contraction RHS vs the FP64 oracle."""
    cfg = wl.make_config("random3d")
    st, U = oracle_state(cfg)
    R_ref = odg.rhs(U, st)
    R = _solver(cfg).rhs(U.cuda()).cpu()
    err = rel_err_per_var(R, R_ref)
    print(f"random3d 64^3 FP32-contraction RHS error {err.tolist()}", flush=True)
    assert float(err.max()) <= 1e-5, err.tolist()


def test_fp32_contraction_drift_kh():
    """50 steps of a 32x32 p=3 TM Kelvin-Helmholtz mesh: L1 drift of the FP32 form vs FP64 (reported)."""
    cfg64 = wl.make_config("kh_tm", n_elem=(32, 32, 1))
    cfg32 = dict(cfg64, precision=wl.FP32_CONTRACT)
    st, U = oracle_state(cfg64)
    A = U.cuda().contiguous()
    B = U.cuda().contiguous()
    _solver(cfg64).run(A, cfg64["dt"], 50)
    _solver(cfg32).run(B, cfg32["dt"], 50)
    drift = ((A - B).abs().reshape(4, -1).sum(1) / A.abs().reshape(4, -1).sum(1)).cpu()
    print(f"FP32-contraction L1 drift after 50 steps: {drift.tolist()}", flush=True)
    assert float(drift.max()) < 1e-5


def test_fp32_mfma_sweeps_equal_the_vector_sweeps_to_fp32_rounding():
    """The matrix-core sweeps compute the same FP32 deviations as the vector ones; the two
    forms differ only by FP32 rounding order: per component well inside 1e-6 of the RHS."""
    cfg = wl.make_config("kh_tm", n_elem=(20, 12, 1))
    st, U = oracle_state(cfg)
    out = {}
    for prec in (wl.FP32_CONTRACT, wl.FP32_MFMA, wl.FP64):
        c = dict(cfg, precision=prec)
        out[prec] = _solver(c).rhs(U.cuda()).cpu()
    e_mv = rel_err_per_var(out[wl.FP32_MFMA], out[wl.FP32_CONTRACT])
    e_m64 = rel_err_per_var(out[wl.FP32_MFMA], out[wl.FP64])
    e_v64 = rel_err_per_var(out[wl.FP32_CONTRACT], out[wl.FP64])
    print(f"MFMA vs vector sweeps {e_mv.tolist()}; vs FP64 {e_m64.tolist()} (vector: {e_v64.tolist()})", flush=True)
    assert float(e_mv.max()) <= 1e-6
    assert float(e_m64.max()) <= 2 * float(e_v64.max()) + 1e-7


def test_fp32_mfma_is_rejected_off_its_shape():
    from paper_2205_00095_amd.solver import Solver
    cfg = wl.make_config("kh_ideal", n_elem=(4, 4, 1))
    cfg["precision"] = wl.FP32_MFMA       # p = 2: no matrix-core sweeps for it
    with pytest.raises(Exception):
        Solver(cfg)
