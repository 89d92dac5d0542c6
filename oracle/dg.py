"""DG weak-form right-hand side (Sec. 2.3, 2.4).  Test infrastructure.

Layout of every nodal array: [nvar, nez, ney, nex, nk, nj, ni] (C order, x node
index fastest); unused dimensions have extent 1.  Direction d = 0, 1, 2 (x, y,
z) has its element axis at 3 - d and its node axis at 6 - d.

Steps, in the order of Sec. 2.3:
 1. primitives at the nodes, W_i = p(U_i)  (con2prim);
 2. volume term, Eq. (quad-vol-flux) with the quadrature collocated at the
    nodes, divided by the diagonal mass matrix:
        V_i = sum_d (2/dx_d) sum_a dhat[i_d, a] F^d(W_(i with i_d -> a));
 3. primitive traces on every face by interpolation, Eq. (interpolation):
        W^+ = sum_a l_a(+1) W_a,   W^- = sum_a l_a(-1) W_a  along d.
    Reading: a trace with rho <= 0 or P <= 0 is replaced by the primitive
    state of the node nearest to that face on the same line (counted);
 4. exterior states: periodic neighbour, outflow (exterior = interior), a
    reflecting wall (the interior trace with its normal velocity negated) or a
    fixed (Dirichlet) state, chosen per end of each dimension;
 5. HLL (or HLLC) numerical flux at every face point, Eq. (quad-surface-flux);
 6. lift with the inverse mass:
        S_i = -sum_d (2/dx_d)(1/w_{i_d}) [l_{i_d}(+1) Fhat^+ - l_{i_d}(-1) Fhat^-];
 7. R = V + S  (= dU/dt).

Pinned by tests/test_oracle_dg.py: zero RHS for a uniform state, exact
discrete conservation on a periodic mesh, mirror and axis-swap symmetries, a
2D field constant in y equals the 1D operator, p = 0 equals a first-order HLL
finite-volume update written independently, a reflecting wall equals a periodic
mesh of twice the size holding the mirrored state, a closed box conserves mass
and energy, and (test_oracle_timestep.py) order ~p+1 on the exact translated
density wave.  The trace fallback of step 3 is pinned by element lines whose
interpolated density (1D, - face) or pressure (2D, + face along y) goes
negative: that face point carries the nearest node's primitives bit for bit and
is counted once.
"""
from __future__ import annotations

import torch

from . import basis
from .con2prim import con2prim
from .setup import DIRICHLET, PERIODIC, REFLECT
from .srhd import face_flux, flux


def _t(a):
    return torch.as_tensor(a, dtype=torch.float64)


def volume_term(W, st):
    tb = basis.tables(st.p)
    dhat = _t(tb["dhat"])
    V = torch.zeros_like(W)
    for d in range(st.dim):
        ax = 6 - d
        F = flux(W, d, st)
        Vd = torch.movedim(torch.tensordot(F, dhat, dims=([ax], [1])), -1, ax)
        V = V + (2.0 / st.dx(d)) * Vd
    return V


def traces(W, d, st):
    """(W^-, W^+, n_fallback) along direction d; the node axis is removed."""
    tb = basis.tables(st.p)
    ax = 6 - d
    Wm = torch.tensordot(W, _t(tb["lm"]), dims=([ax], [0]))
    Wp = torch.tensordot(W, _t(tb["lp"]), dims=([ax], [0]))
    # node-axis position in the trace arrays is gone; element axes are unchanged
    W0 = W.select(ax, 0)
    Wq = W.select(ax, st.p)
    bad_m = (Wm[0] <= 0) | (Wm[-1] <= 0)
    bad_p = (Wp[0] <= 0) | (Wp[-1] <= 0)
    Wm = torch.where(bad_m[None], W0, Wm)
    Wp = torch.where(bad_p[None], Wq, Wp)
    return Wm, Wp, int(bad_m.sum()) + int(bad_p.sum())


def face_states(Wm, Wp, d, st):
    """Left/right states on faces 0..n along d (face f sits between elements f-1 and f)."""
    ea = 3 - d
    n = Wm.shape[ea]
    first_m = Wm.narrow(ea, 0, 1)
    last_p = Wp.narrow(ea, n - 1, 1)
    if st.bc[d] == PERIODIC:
        WL = torch.cat([last_p, Wp], ea)
        WR = torch.cat([Wm, first_m], ea)
    else:
        WL = torch.cat([_exterior(first_m, d, st, 0), Wp], ea)
        WR = torch.cat([Wm, _exterior(last_p, d, st, 1)], ea)
    return WL, WR


def _exterior(Wt, d, st, end):
    """Exterior state at a boundary face from the interior trace Wt: outflow (the trace
    itself), a reflecting wall (its mirror image) or a fixed (Dirichlet) state."""
    kind = st.end_type(d, end)
    if kind == REFLECT:
        return _mirrored(Wt, d)
    if kind == DIRICHLET:
        from .srhd import u_from_v
        rho, vx, vy, vz, P = st.bc_state[(d, end)]
        u = u_from_v(torch.tensor([vx, vy, vz][:st.dim]), st.c)
        w = torch.cat([torch.tensor([rho]), u, torch.tensor([P])])
        return w.reshape((-1,) + (1,) * (Wt.dim() - 1)).expand_as(Wt).clone()
    return Wt


def _mirrored(W, d):
    """Primitive states reflected across a plane normal to d: u_d -> -u_d."""
    M = W.clone()
    M[1 + d] = -M[1 + d]
    return M


def surface_term(W, st, stats=None):
    tb = basis.tables(st.p)
    S = torch.zeros_like(W)
    nfb = 0
    for d in range(st.dim):
        ax, ea = 6 - d, 3 - d
        Wm, Wp, nb = traces(W, d, st)
        nfb += nb
        WL, WR = face_states(Wm, Wp, d, st)
        Fh = face_flux(WL, WR, d, st)
        n = W.shape[ea]
        Fplus = Fh.narrow(ea, 1, n).unsqueeze(ax)
        Fminus = Fh.narrow(ea, 0, n).unsqueeze(ax)
        shp = [1] * 7
        shp[ax] = st.p + 1
        cp = (_t(tb["lp"]) / _t(tb["w"])).reshape(shp)
        cm = (_t(tb["lm"]) / _t(tb["w"])).reshape(shp)
        S = S - (2.0 / st.dx(d)) * (cp * Fplus - cm * Fminus)
    if stats is not None:
        stats["trace_fallbacks"] = stats.get("trace_fallbacks", 0) + nfb
    return S


def rhs(U, st, stats=None):
    """R(U) = M^-1 (volume - surface); U [nvar, nez, ney, nex, nk, nj, ni]."""
    W, status = con2prim(U, st)
    if stats is not None:
        stats["c2p_fail"] = stats.get("c2p_fail", 0) + int((status != 0).sum())
    return volume_term(W, st) + surface_term(W, st, stats)


def elem_weights(st):
    """Tensor-product GL weights of one element, shaped [1,1,1,1,nk,nj,ni]."""
    w = _t(basis.tables(st.p)["w"])
    one = torch.ones(1, dtype=torch.float64)
    wz = w if st.dim > 2 else one
    wy = w if st.dim > 1 else one
    return (wz[:, None, None] * wy[None, :, None] * w[None, None, :]).reshape(1, 1, 1, 1, *(
        wz.numel(), wy.numel(), w.numel()))


def cell_volume(st):
    v = 1.0
    for d in range(st.dim):
        v *= st.dx(d)
    return v
