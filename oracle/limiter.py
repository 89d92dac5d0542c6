"""Slope limiter for basis orders >= 1.  Test infrastructure.

The paper stabilises its p >= 1 shock runs with a slope limiter beside the
physicality operator (Sec. 2.3, naming the minmod limiter of van Leer 1979 and
the limiter of Moe, Rossmanith & Seal 2015; Sec. 4 uses the latter in its 1D
Riemann problems) but prints neither algorithm.

Reading R29: minmod-bounded slopes applied in scaling form, per element:
  * averages  u_bar_k = sum_i w_i u_{k,i} / sum_i w_i  (tensor Gauss-Legendre weights)
    of every conserved component k;
  * slope of component k along d, the coefficient of xi_d in the element's
    Legendre expansion (its L2 projection onto xi_d on [-1, 1]^dim):
        s = sum_i w_i xi_{d,i} u_{k,i} / sum_i w_i xi_{d,i}^2,
    summed over mirror pairs of nodes (xi_{d,i} = -xi_{d,m}, equal weights) as
    w_i xi_{d,i} (u_{k,i} - u_{k,m}) / 2, so that a constant element has slope 0;
  * the minmod bound of that slope by the differences to the neighbours' averages
    along d (Cockburn & Shu's generalized slope limiter: s measures the change from
    the centre to the face, bounded by the full differences):
        s~ = minmod(s, u_bar_{d+} - u_bar, u_bar - u_bar_{d-}),
    periodic wrap; at a non-periodic end the element's own average (difference 0);
    minmod is the argument of least magnitude when all have one sign, else 0;
  * one factor for the whole element, the least ratio s~ / s over components and
    directions, counting only pairs where the bound moves the slope by more than
    EPS times the component's scale (the element's average energy
    E = |tau_bar + D_bar c^2| over c^2 for D, over c for S, E for tau), so that
    rounding noise in a flat component does not flatten the others:
        theta = min(1, min over those pairs of s~ / s);
  * where theta < 1 every node moves towards the average:
        u_i <- u_bar + theta (u_i - u_bar)   (all components, all modes).
Averages are unchanged (the limiter conserves).  With one factor for all
components every node stays on the segment between itself and the average, so an
element whose nodes and average are admissible stays admissible (the admissible
set is convex); the componentwise form (each component replaced by its limited
linear function) lost that and gave an inadmissible average within the first step
of the strong blast wave (problem 2) at p = 1.  Applied after each SSP-RK stage,
before the physicality operator.

Pinned by tests/test_oracle_limiter.py: the slope against numpy's Legendre
fit, averages preserved, linear data left unchanged, a jump inside an element
scaled to the neighbour difference, a spike cut to a constant, the minmod bounds
and sign agreement of every limited slope, idempotence, and total variation of
the averages not increasing over limited forward-Euler steps on a Riemann problem
(while it grows without the limiter).
"""
from __future__ import annotations

import torch

from . import basis
from .dg import elem_weights
from .setup import PERIODIC

EPS = 1e-10


def _minmod(a, b, c):
    same = ((a > 0) & (b > 0) & (c > 0)) | ((a < 0) & (b < 0) & (c < 0))
    m = torch.minimum(torch.minimum(a.abs(), b.abs()), c.abs())
    return torch.where(same, torch.sign(a) * m, torch.zeros_like(a))


def _xi(st, d):
    """Reference coordinate xi_d of every node, shaped like one element [1,1,1,1,nk,nj,ni]."""
    x = torch.as_tensor(basis.tables(st.p)["x"], dtype=torch.float64)
    shp = [1] * 7
    shp[6 - d] = st.p + 1
    return x.reshape(shp)


def _slope(U, w, xi, d):
    """Amplitude of the linear mode along d, with mirror nodes paired (exactly 0 on constants)."""
    odd = 0.5 * (U - torch.flip(U, dims=(6 - d,)))
    return (odd * w * xi).sum((4, 5, 6)) / (w * xi * xi).sum()


def _neighbour_average(avg, d, side, st):
    """Average of the neighbour along d (side +1 / -1); the element's own at a non-periodic end.
    avg: [nvar, nez, ney, nex]; the element axis of d is 3 - d."""
    ea = 3 - d
    n = avg.shape[ea]
    nb = torch.roll(avg, shifts=-side, dims=ea)
    if st.bc[d] != PERIODIC:
        # non-periodic (both ends): the end element sees itself
        idx = n - 1 if side > 0 else 0
        sl = [slice(None)] * 4
        sl[ea] = slice(idx, idx + 1)
        nb[tuple(sl)] = avg[tuple(sl)]
    return nb


def averages(U, st):
    w = elem_weights(st)
    return (U * w).sum((4, 5, 6)) / w.sum()


def scales(avg, st):
    """Per-component scale of each element: E/c^2 (D), E/c (S), E (tau), E = |tau + D c^2|."""
    c = st.c
    E = (avg[-1] + avg[0] * c * c).abs()
    return torch.stack([E / (c * c)] + [E / c] * st.dim + [E])


def theta(U, st):
    """Scaling factor of every element [nez, ney, nex]."""
    w = elem_weights(st)
    avg = averages(U, st)
    sig = scales(avg, st)
    th = torch.ones(avg.shape[1:], dtype=torch.float64)
    for d in range(st.dim):
        s = _slope(U, w, _xi(st, d), d)
        sl = _minmod(s, _neighbour_average(avg, d, +1, st) - avg, avg - _neighbour_average(avg, d, -1, st))
        act = (s - sl).abs() > EPS * sig
        ratio = torch.where(act, sl / torch.where(act, s, torch.ones_like(s)), torch.ones_like(s))
        th = torch.minimum(th, ratio.min(0).values)
    return th


def limit(U, st, stats=None):
    """Apply the slope limiter to every element of U [nvar, nez, ney, nex, nk, nj, ni]."""
    if st.p == 0:
        return U
    th = theta(U, st)
    lim = th < 1.0
    if stats is not None:
        stats["limited"] = stats.get("limited", 0) + int(lim.sum())
    if not bool(lim.any()):
        return U
    avg = averages(U, st)[..., None, None, None]
    scaled = avg + th[None, ..., None, None, None] * (U - avg)
    return torch.where(lim[None, ..., None, None, None], scaled, U)
