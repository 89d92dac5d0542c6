"""Slope limiter for basis orders >= 1.  Test infrastructure.

The paper stabilises its p >= 1 shock runs with a slope limiter beside the
physicality operator (Sec. 2.3, naming the minmod limiter of van Leer 1979 and
the limiter of Moe, Rossmanith & Seal 2015; Sec. 4 uses them in its 1D Riemann
problems) but prints neither algorithm.

Reading R29: the componentwise minmod slope limiter of DG schemes in the
gradient (MUSCL) form, applied to every conserved component of every element:
  * average  u_bar = sum_i w_i u_i / sum_i w_i  (tensor Gauss-Legendre weights);
  * slope along d, the amplitude of the element's linear mode in xi_d (its L2
    projection onto xi_d on the reference element [-1, 1]^dim):
        s_d = sum_i w_i xi_{d,i} u_i / sum_i w_i xi_{d,i}^2,
    summed over mirror pairs of nodes (xi_{d,i} = -xi_{d,m}, equal weights) as
    w_i xi_{d,i} (u_i - u_m) / 2, so that a constant element has slope exactly 0;
  * limited slope  s~_d = minmod(s_d, (u_bar_{d+} - u_bar)/2, (u_bar - u_bar_{d-})/2),
    u_bar_{d+-} the averages of the neighbours along d (periodic wrap; at a
    non-periodic end the element's own average, so the slope there is zero);
    half the difference because the centres are one element width apart while s
    is the change from the centre to the face; minmod is the argument of least
    magnitude when all have one sign, else 0;
  * if s~_d = s_d for every d the component is left as it is, else it becomes the
    linear function u_bar + sum_d s~_d xi_d (higher modes dropped).
The average is unchanged either way (the limiter conserves).  Applied after each
SSP-RK stage, before the physicality operator.

Pinned by tests/test_oracle_limiter.py: averages preserved, linear data left
unchanged, a jump inside an element cut back to a constant, the minmod bounds
and sign agreement of every limited slope, idempotence, and total variation of
the averages not increasing over a limited forward-Euler step on a Riemann
problem.
"""
from __future__ import annotations

import torch

from . import basis
from .dg import elem_weights
from .setup import PERIODIC


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


def limit(U, st, stats=None):
    """Apply the slope limiter to every element of U [nvar, nez, ney, nex, nk, nj, ni]."""
    if st.p == 0:
        return U
    w = elem_weights(st)
    wsum = w.sum()
    avg = (U * w).sum((4, 5, 6)) / wsum                      # [nvar, nez, ney, nex]
    slopes, limited = [], []
    for d in range(st.dim):
        xi = _xi(st, d)
        s = _slope(U, w, xi, d)
        fwd = 0.5 * (_neighbour_average(avg, d, +1, st) - avg)
        bwd = 0.5 * (avg - _neighbour_average(avg, d, -1, st))
        sl = _minmod(s, fwd, bwd)
        slopes.append(sl)
        limited.append(sl != s)
    changed = limited[0]
    for m in limited[1:]:
        changed = changed | m                                  # [nvar, nez, ney, nex]
    if stats is not None:
        stats["limited"] = stats.get("limited", 0) + int(changed.sum())
    if not bool(changed.any()):
        return U
    lin = avg[..., None, None, None] + sum(slopes[d][..., None, None, None] * _xi(st, d) for d in range(st.dim))
    return torch.where(changed[..., None, None, None], lin, U)
