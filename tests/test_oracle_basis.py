"""Pins of the oracle's Gauss-Legendre nodal basis (Sec. 2.3) against textbook facts."""
import numpy as np
import pytest

from oracle import basis


@pytest.mark.parametrize("p", [0, 1, 2, 3, 4])
def test_quadrature_exact_to_2p_plus_1(p):
    t = basis.tables(p)
    for k in range(2 * p + 2):
        exact = (1.0 - (-1.0) ** (k + 1)) / (k + 1)
        assert abs((t["w"] * t["x"] ** k).sum() - exact) < 1e-14


def test_known_rules():
    t = basis.tables(2)
    assert np.allclose(t["x"], [-np.sqrt(0.6), 0.0, np.sqrt(0.6)], atol=1e-15)
    assert np.allclose(t["w"], [5 / 9, 8 / 9, 5 / 9], atol=1e-15)
    t1 = basis.tables(1)
    assert np.allclose(t1["x"], [-1 / np.sqrt(3), 1 / np.sqrt(3)], atol=1e-15)


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_differentiates_polynomials_exactly(p):
    t = basis.tables(p)
    x = t["x"]
    for k in range(p + 1):
        f = x ** k
        fp = k * x ** (k - 1) if k > 0 else 0 * x
        # interpolant derivative at node a: sum_i f_i l_i'(x_a) = (dl^T f)_a
        assert np.allclose(t["dl"].T @ f, fp, atol=1e-12)


@pytest.mark.parametrize("p", [0, 1, 2, 3, 4])
def test_summation_by_parts(p):
    t = basis.tables(p)
    Dm = t["dl"].T          # Dm[a, i] = l_i'(x_a)
    Wm = np.diag(t["w"])
    lhs = Wm @ Dm + Dm.T @ Wm
    rhs = np.outer(t["lp"], t["lp"]) - np.outer(t["lm"], t["lm"])
    assert np.allclose(lhs, rhs, atol=1e-12)


@pytest.mark.parametrize("p", [0, 1, 2, 3])
def test_boundary_interpolation(p):
    t = basis.tables(p)
    for k in range(p + 1):
        assert abs((t["lp"] * t["x"] ** k).sum() - 1.0) < 1e-13
        assert abs((t["lm"] * t["x"] ** k).sum() - (-1.0) ** k) < 1e-13
    # dhat has the documented definition and the weighted column sums vanish
    assert np.allclose((t["w"][:, None] * t["dhat"]).sum(0), 0.0, atol=1e-12)
