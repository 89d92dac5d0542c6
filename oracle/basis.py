"""Nodal Lagrange basis on Gauss-Legendre nodes (Sec. 2.3: phi_i(x_j) = delta_ij).

Test infrastructure.  The paper names a Lagrange nodal basis but not the node
family; the reading used here is Gauss-Legendre nodes with the volume and face
quadratures collocated with the nodes, so the mass matrix is diagonal.

Tables (reference element [-1, 1]):
  x, w        GL nodes and weights (numpy.polynomial.legendre.leggauss)
  dl[i, a]    l_i'(x_a), from numpy Polynomial objects built from the roots
  dhat[i, a]  w_a l_i'(x_a) / w_i   (volume term: M^-1 of int F dphi_i/dx)
  lp, lm      l_i(+1), l_i(-1)      (face traces and lift)

Pinned by tests/test_oracle_basis.py: exact differentiation of degree-p
polynomials, the summation-by-parts identity W D + D^T W = lp lp^T - lm lm^T,
partition of unity of lp/lm, and exactness of the quadrature to degree 2p+1.
"""
from __future__ import annotations

from functools import lru_cache

import numpy as np
from numpy.polynomial import legendre as npleg
from numpy.polynomial import polynomial as nppoly


@lru_cache(maxsize=None)
def tables(p: int) -> dict:
    x, w = npleg.leggauss(p + 1)
    n = p + 1
    ell = []
    for i in range(n):
        others = np.delete(x, i)
        num = nppoly.Polynomial.fromroots(others) if others.size else nppoly.Polynomial([1.0])
        ell.append(num / num(x[i]))
    dl = np.array([[ell[i].deriv()(x[a]) for a in range(n)] for i in range(n)])
    dhat = (w[None, :] * dl) / w[:, None]
    lp = np.array([ell[i](1.0) for i in range(n)])
    lm = np.array([ell[i](-1.0) for i in range(n)])
    return dict(x=x, w=w, dl=dl, dhat=dhat, lp=lp, lm=lm, polys=ell)
