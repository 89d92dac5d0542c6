"""Pins of the oracle's physicality-enforcing operator (Sec. 2.5)."""
import numpy as np
import pytest
import torch

from oracle import dg, physicality, srhd
from oracle.setup import IDEAL, Setup


def _flagged_cells(st, rng, ncell):
    """Elements with admissible averages and some inadmissible nodes (both failure kinds)."""
    n = (st.p + 1) ** st.dim
    cells = []
    while len(cells) < ncell:
        rho = 10 ** rng.uniform(-1, 1, n)
        P = 10 ** rng.uniform(-1, 1, n)
        g = rng.uniform(1, 4, n)
        nv = rng.standard_normal((st.dim, n))
        nv /= np.linalg.norm(nv, axis=0)
        v = nv * np.sqrt(1 - 1 / g ** 2)
        U = srhd.prim3_to_cons(torch.tensor(rho), torch.tensor(v), torch.tensor(P), st)
        k = rng.integers(1, 4)
        idx = rng.choice(n, k, replace=False)
        for i in idx:
            kind = rng.integers(3)
            if kind == 0:
                U[0, i] = -rng.uniform(0.01, 0.5) * U[0].mean()       # D < 0
            elif kind == 1:
                U[1:-1, i] *= rng.uniform(1.5, 4.0)                   # |S| too large (q < 0)
            else:
                U[-1, i] = -rng.uniform(0.5, 2.0) * U[0, i]           # E < 0 (tau < -D c^2)
        if bool(srhd.admissible(U, st).all()):
            continue
        w = dg.elem_weights(st).reshape(-1)
        Ub = (U * w).sum(1) / w.sum()
        if bool(srhd.admissible(Ub[:, None], st).all()):
            cells.append((U, Ub))
    return cells


def _bisect(Ui, Ub, st, iters=80):
    """Largest s with U_bar + s (U_i - U_bar) admissible, by bisection (brute force)."""
    def ok(s):
        return bool(srhd.admissible((Ub + s * (Ui - Ub))[:, None], st).all())
    if ok(1.0):
        return 1.0
    lo, hi = 0.0, 1.0
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if ok(mid) else (lo, mid)
    return lo


@pytest.mark.parametrize("dim,p", [(1, 2), (2, 2), (3, 1)])
def test_node_factor_matches_bisection(dim, p):
    st = Setup(dim=dim, p=p, eos=IDEAL)
    rng = np.random.default_rng(31 + dim)
    stage2 = 0
    for U, Ub in _flagged_cells(st, rng, 12):
        s = physicality.node_factor(U, Ub, st, st.phys_eps)
        for i in range(U.shape[1]):
            sb = _bisect(U[:, i], Ub, st)
            assert float(s[i]) <= sb + 1e-15
            assert float(s[i]) >= sb - 1e-9
            Ui = U[:, i]
            stage2 += int(bool((Ui[0] > 0) and (Ui[-1] + Ui[0] > 0)
                               and not bool(srhd.admissible(Ui[:, None], st).all())))
    assert stage2 > 0  # the quadratic branch was exercised


def _mesh_with_flagged(st, rng):
    cells = _flagged_cells(st, rng, int(np.prod(st.n_elem)) // 2)
    U = torch.zeros((st.nvar,) + st.shape())
    flat = U.reshape(st.nvar, -1, (st.p + 1) ** st.dim)
    # half the elements flagged, the other half admissible random states
    good = _flagged_cells(st, rng, 1)[0][0].clone()
    good[0] = good[0].abs() + 1.0
    good[1:-1] *= 0.1
    good[-1] = good[-1].abs() + 1.0
    for e in range(flat.shape[1]):
        flat[:, e] = cells[e // 2][0] if e % 2 == 0 else good
    return flat.reshape(U.shape)


def test_operator_invariants():
    st = Setup(dim=2, p=2, n_elem=(4, 4, 1), eos=IDEAL)
    rng = np.random.default_rng(40)
    U = _mesh_with_flagged(st, rng)
    stats = {}
    V = physicality.enforce(U, st, stats)
    assert stats["smoothed"] == 8 and stats.get("bad_average", 0) == 0
    w = dg.elem_weights(st)
    avg_before = (U * w).sum((4, 5, 6))
    avg_after = (V * w).sum((4, 5, 6))
    assert torch.allclose(avg_after, avg_before, rtol=1e-14, atol=1e-14 * float(avg_before.abs().max()))
    assert bool(srhd.admissible(V, st).all())
    flagged = ~srhd.admissible(U, st).flatten(3).all(-1)
    assert torch.equal(V[:, ~flagged], U[:, ~flagged])           # unflagged untouched, bitwise
    assert torch.equal(physicality.enforce(V, st), V)             # idempotent


def test_inadmissible_average_left_unchanged():
    st = Setup(dim=1, p=2, n_elem=(1, 1, 1), eos=IDEAL)
    U = torch.tensor([[1.0, -3.0, 1.0], [0.0, 0.0, 0.0], [1.0, 1.0, 1.0]]).reshape(3, 1, 1, 1, 1, 1, 3)
    stats = {}
    V = physicality.enforce(U, st, stats)
    assert torch.equal(U, V) and stats["bad_average"] == 1
