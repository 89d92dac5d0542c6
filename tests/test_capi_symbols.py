"""The C-ABI library loads without a GPU and exports every function include/dgsrhd.h declares."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2205_00095_amd", "libdgsrhd.so")
HEADER = os.path.join(ROOT, "include", "dgsrhd.h")


def _declared():
    text = open(HEADER).read()
    return re.findall(r"^\s*(?:int|void|size_t|const char\s*\*)\s+(dg_\w+)\s*\(", text, re.M)


def test_header_declares_the_boundary():
    names = set(_declared())
    for required in ("dg_init_mesh", "dg_set_state", "dg_rhs", "dg_enforce_physical", "dg_ssprk3_step",
                     "dg_rhs_vjp"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_signatures_cover_the_header():
    from paper_2205_00095_amd import _lib
    assert set(_declared()) == set(_lib.SIGNATURES)
    _lib.load()


def test_null_arguments_are_rejected_without_a_gpu():
    if not os.path.exists(LIB):
        pytest.skip("library not built")
    from paper_2205_00095_amd import _lib
    lib = _lib.load()
    assert lib.dg_init_mesh(None, None, None) == _lib.DG_EINVAL
    out = ctypes.c_void_p()
    assert lib.dg_init_mesh(None, None, ctypes.byref(out)) == _lib.DG_EINVAL
    assert lib.dg_rhs(None, None, None) == _lib.DG_EINVAL
    assert lib.dg_last_error(None) == b"null context"


def _desc(**over):
    """A valid 1D description through the Python binding (nothing is allocated here)."""
    from paper_2205_00095_amd import workloads as wl
    from paper_2205_00095_amd.solver import _desc_from_config
    cfg = wl.make_config("wave1d", **over)
    return _desc_from_config(cfg, False)


@pytest.mark.parametrize("change", [
    {"p": 5},                                                     # unsupported order
    {"flux": 7},                                                  # unknown flux
    {"bc": (0, 0, 0), "bc_hi": (2, 0, 0)},                        # a periodic dimension has no upper end
    {"bc": (3, 0, 0), "bc_state": {(0, 0): (-1.0, 0.0, 0.0, 0.0, 1.0), (0, 1): (1.0, 0.0, 0.0, 0.0, 1.0)}},
    {"bc": (3, 0, 0), "bc_state": {(0, 0): (1.0, 1.5, 0.0, 0.0, 1.0), (0, 1): (1.0, 0.0, 0.0, 0.0, 1.0)}},
    {"bc": (1, 0, 0), "bc_hi": (3, 0, 0)},                        # a Dirichlet end without its state
    {"precision": 2},                                             # matrix-core sweeps exist for 2D p = 3 only
    {"c2p_iters": -1},                                            # fixed iteration count out of range
    {"limiter": 2},                                               # no such limiter (the last field)
])
def test_invalid_descriptions_are_rejected_without_a_gpu(change):
    """Validation runs on the host before any device call; the checks read the fields the
    binding fills, so a layout mismatch between the binding and the header shows here."""
    if not os.path.exists(LIB):
        pytest.skip("library not built")
    from paper_2205_00095_amd import _lib
    lib = _lib.load()
    over = dict(change)
    flux = over.pop("flux", None)
    d = _desc(**over)
    if flux is not None:
        d.flux = flux
    out = ctypes.c_void_p()
    assert lib.dg_init_mesh(ctypes.byref(d), None, ctypes.byref(out)) == _lib.DG_EINVAL
    assert not out.value


def test_noalloc_rejections_happen_on_the_host():
    """dg_rhs_noalloc validates the description, the pointers and the mesh size against its
    static scratch before any device call (fake pointers are never dereferenced)."""
    if not os.path.exists(LIB):
        pytest.skip("library not built")
    from paper_2205_00095_amd import _lib
    lib = _lib.load()
    fake_u, fake_r = ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2000)
    assert lib.dg_rhs_noalloc(None, None, fake_u, fake_r, None) == _lib.DG_EINVAL
    d = _desc()
    assert lib.dg_rhs_noalloc(ctypes.byref(d), None, None, fake_r, None) == _lib.DG_EINVAL
    assert lib.dg_rhs_noalloc(ctypes.byref(d), None, fake_u, fake_u, None) == _lib.DG_EINVAL
    bad = _desc(p=5)
    assert lib.dg_rhs_noalloc(ctypes.byref(bad), None, fake_u, fake_r, None) == _lib.DG_EINVAL
    # 3D p=2 (the shapes whose primitives are staged in the scratch): 5 variables x 27
    # nodes per element; one element more than the scratch holds
    from paper_2205_00095_amd import workloads as wl
    from paper_2205_00095_amd.solver import _desc_from_config
    n_fit = _lib.RHS_NOALLOC_MAX_STATE // 135
    big = _desc_from_config(wl.make_config("random3d", n_elem=(n_fit + 1, 1, 1)), False)
    assert lib.dg_rhs_noalloc(ctypes.byref(big), None, fake_u, fake_r, None) == _lib.DG_EINVAL


def test_noalloc_limit_matches_the_header():
    from paper_2205_00095_amd import _lib
    text = open(HEADER).read()
    m = re.search(r"#define\s+DG_RHS_NOALLOC_MAX_STATE\s+(\d+)u", text)
    assert m and int(m.group(1)) == _lib.RHS_NOALLOC_MAX_STATE
