"""The term-magnitude sum behind the RHS parity bars bounds the RHS it describes.

T_i sums the magnitudes of the terms whose signed sum is R_i, so |R_i| <= T_i at
every node (the triangle inequality; equality where no term cancels), and T is the
same for a state and its mirror image.  A magnitude that dropped a term (the
pressure in the momentum flux, one direction, the lift) would fall below |R| on
these workloads."""
import pytest
import torch

from oracle import dg as odg
from paper_2205_00095_amd import workloads as wl

from ._conditioning import rhs_cancellation, rhs_term_magnitude
from ._util import oracle_state


@pytest.mark.parametrize("kind,over", [("wave1d", {}), ("kh_tm", {"n_elem": (6, 5, 1)}),
                                       ("kh_ideal", {"n_elem": (5, 4, 1), "p": 1}),
                                       ("random3d", {"n_elem": (3, 2, 2)})])
def test_term_magnitude_bounds_the_rhs(kind, over):
    cfg = wl.make_config(kind, **over)
    st, U = oracle_state(cfg)
    R = odg.rhs(U, st)
    T = rhs_term_magnitude(U, st)
    assert bool((R.abs() <= T * (1 + 1e-12)).all())
    kappa = rhs_cancellation(U, st, R)
    assert bool((kappa >= 1.0 - 1e-12).all())


def test_term_magnitude_is_mirror_symmetric():
    """Reflecting the state along x (x -> 1 - x, S_x -> -S_x) reflects T: magnitudes carry
    no direction, so a sign slip between the + and - faces would show here."""
    cfg = wl.make_config("kh_tm", n_elem=(6, 5, 1))
    st, U = oracle_state(cfg)
    M = U.flip(3).flip(6).clone()
    M[1] = -M[1]
    T = rhs_term_magnitude(U, st)
    TM = rhs_term_magnitude(M, st)
    assert torch.allclose(TM, T.flip(3).flip(6), rtol=1e-12, atol=0)
