"""Pins of the oracle's DG right-hand side (Sec. 2.3, 2.4) against invariants and reductions."""
import numpy as np
import pytest
import torch

from oracle import con2prim as cp
from oracle import dg, srhd
from oracle.setup import IDEAL, OUTFLOW, PERIODIC, TM, Setup


def _random_state(st, rng, gmax=3.0, smooth=False):
    shape = st.shape()
    if smooth:
        # smooth periodic field over the mesh (sin of node coordinates)
        q = st.p + 1
        xi, _ = np.polynomial.legendre.leggauss(q)
        coords = []
        for d in range(3):
            n = st.n_elem[d] if d < st.dim else 1
            if d < st.dim:
                pos = (np.arange(n)[:, None] + 0.5 * (xi[None] + 1)) / n
            else:
                pos = np.zeros((1, 1))
            b = [1] * 6
            b[2 - d], b[5 - d] = pos.shape
            coords.append(np.broadcast_to(pos.reshape(b), shape))
        ph = sum(2 * np.pi * coords[d] * (d + 1) for d in range(st.dim))
        rho = 1.0 + 0.3 * np.sin(ph)
        P = 1.0 + 0.2 * np.cos(ph)
        v = np.stack([0.3 * np.cos(ph + d) for d in range(st.dim)])
    else:
        rho = 10 ** rng.uniform(-0.5, 0.5, shape)
        P = 10 ** rng.uniform(-0.5, 0.5, shape)
        g = rng.uniform(1.0, gmax, shape)
        nv = rng.standard_normal((st.dim,) + shape)
        nv /= np.sqrt((nv ** 2).sum(0))
        v = nv * np.sqrt(1 - 1 / g ** 2)
    return srhd.prim3_to_cons(torch.tensor(rho), torch.tensor(v), torch.tensor(P), st)


CASES = [(1, 2, IDEAL), (1, 0, TM), (2, 1, TM), (2, 3, IDEAL), (2, 2, TM), (3, 2, IDEAL), (3, 1, TM)]


@pytest.mark.parametrize("dim,p,eos", CASES)
def test_uniform_state_gives_zero(dim, p, eos):
    st = Setup(dim=dim, p=p, n_elem=(4, 3, 2)[:dim] + (1,) * (3 - dim), eos=eos,
               bc=(PERIODIC, OUTFLOW, PERIODIC))
    rng = np.random.default_rng(dim * 10 + p)
    U0 = _random_state(Setup(dim=dim, p=0, eos=eos), rng)  # one random state
    U = U0.reshape(st.nvar, *([1] * 6)).expand((st.nvar,) + st.shape()).clone()
    R = dg.rhs(U, st)
    W, _ = cp.con2prim(U, st)
    fmax = max(float(srhd.flux(W, d, st).abs().max()) * 2 / st.dx(d) for d in range(dim))
    assert float(R.abs().max()) <= 1e-13 * fmax * (p + 1) ** 2


@pytest.mark.parametrize("dim,p,eos", CASES)
def test_discrete_conservation_periodic(dim, p, eos):
    st = Setup(dim=dim, p=p, n_elem=(5, 4, 3)[:dim] + (1,) * (3 - dim), eos=eos)
    U = _random_state(st, np.random.default_rng(7))
    R = dg.rhs(U, st)
    wR = R * dg.elem_weights(st)
    tot = wR.sum((1, 2, 3, 4, 5, 6))
    scale = wR.abs().sum((1, 2, 3, 4, 5, 6))
    assert float((tot.abs() / scale).max()) < 1e-13


def test_mirror_symmetry_x():
    st = Setup(dim=2, p=2, n_elem=(6, 5, 1), eos=TM, bc=(PERIODIC, OUTFLOW, PERIODIC))
    U = _random_state(st, np.random.default_rng(8))

    def mirror(A):
        B = A.flip(3).flip(6).clone()
        B[1] = -B[1]
        return B

    R = dg.rhs(U, st)
    Rm = dg.rhs(mirror(U), st)
    assert torch.allclose(Rm, mirror(R), rtol=1e-12, atol=1e-12 * float(R.abs().max()))


def test_axis_swap_symmetry_2d():
    st = Setup(dim=2, p=3, n_elem=(4, 4, 1), eos=IDEAL)
    U = _random_state(st, np.random.default_rng(9))

    def swap(A):
        B = A.transpose(2, 3).transpose(5, 6).clone()
        B[[1, 2]] = B[[2, 1]]
        return B

    R = dg.rhs(U, st)
    Rs = dg.rhs(swap(U), st)
    assert torch.allclose(Rs, swap(R), rtol=1e-12, atol=1e-12 * float(R.abs().max()))


@pytest.mark.parametrize("eos", [IDEAL, TM])
def test_2d_constant_in_y_equals_1d(eos):
    p = 2
    st1 = Setup(dim=1, p=p, n_elem=(7, 1, 1), eos=eos)
    st2 = Setup(dim=2, p=p, n_elem=(7, 3, 1), eos=eos, hi=(1.0, 0.4, 1.0),
                bc=(PERIODIC, OUTFLOW, PERIODIC))
    U1 = _random_state(st1, np.random.default_rng(10))
    # embed: (D, Sx, tau) -> (D, Sx, 0, tau), constant along y
    U2 = torch.zeros((4,) + st2.shape())
    for k2, k1 in ((0, 0), (1, 1), (3, 2)):
        U2[k2] = U1[k1].expand(1, 3, 7, 1, p + 1, p + 1)
    R1 = dg.rhs(U1, st1)
    R2 = dg.rhs(U2, st2)
    scale = float(R1.abs().max())
    for k2, k1 in ((0, 0), (1, 1), (3, 2)):
        assert torch.allclose(R2[k2], R1[k1].expand_as(R2[k2]), atol=1e-13 * scale)
    assert float(R2[2].abs().max()) < 1e-13 * scale


@pytest.mark.parametrize("eos", [IDEAL, TM])
def test_p0_is_first_order_hll_finite_volume(eos):
    """p = 0 removes the volume term: R_e = -(F(U_e, U_e+1) - F(U_e-1, U_e))/dx (Sec. 2.3)."""
    n = 9
    st = Setup(dim=1, p=0, n_elem=(n, 1, 1), eos=eos, hi=(2.0, 1.0, 1.0))
    U = _random_state(st, np.random.default_rng(12), gmax=5.0)
    R = dg.rhs(U, st)
    W, _ = cp.con2prim(U, st)
    Wc = W.reshape(3, n)
    ref = torch.zeros(3, n)
    for e in range(n):
        left = srhd.hll(Wc[:, (e - 1) % n, None], Wc[:, e, None], 0, st)[:, 0]
        right = srhd.hll(Wc[:, e, None], Wc[:, (e + 1) % n, None], 0, st)[:, 0]
        ref[:, e] = -(right - left) / st.dx(0)
    assert torch.allclose(R.reshape(3, n), ref, rtol=1e-13, atol=1e-13)


def test_outflow_boundary_face_uses_interior_flux():
    """Outflow: the boundary face flux is the physical flux of the interior trace."""
    st = Setup(dim=1, p=0, n_elem=(3, 1, 1), eos=IDEAL, bc=(OUTFLOW, PERIODIC, PERIODIC))
    U = _random_state(st, np.random.default_rng(13))
    W, _ = cp.con2prim(U, st)
    Wc = W.reshape(3, 3)
    R = dg.rhs(U, st).reshape(3, 3)
    f0 = srhd.flux(Wc[:, :1], 0, st)[:, 0]
    f01 = srhd.hll(Wc[:, 0, None], Wc[:, 1, None], 0, st)[:, 0]
    assert torch.allclose(R[:, 0], -(f01 - f0) / st.dx(0), rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("dim,p,eos", [(1, 2, IDEAL), (2, 2, TM), (3, 1, IDEAL)])
def test_hllc_rhs_uniform_zero_and_conservative(dim, p, eos):
    """The operator with the HLLC flux: zero for a uniform state, discretely conservative
    on a periodic mesh."""
    from oracle.setup import HLLC
    st = Setup(dim=dim, p=p, n_elem=(4, 3, 2)[:dim] + (1,) * (3 - dim), eos=eos, flux=HLLC)
    rng = np.random.default_rng(40 + dim)
    U0 = _random_state(Setup(dim=dim, p=0, eos=eos), rng)
    U = U0.reshape(st.nvar, *([1] * 6)).expand((st.nvar,) + st.shape()).clone()
    R = dg.rhs(U, st)
    W, _ = cp.con2prim(U, st)
    fmax = max(float(srhd.flux(W, d, st).abs().max()) * 2 / st.dx(d) for d in range(dim))
    assert float(R.abs().max()) <= 1e-13 * fmax * (p + 1) ** 2
    U = _random_state(st, rng)
    wR = dg.rhs(U, st) * dg.elem_weights(st)
    tot = wR.sum((1, 2, 3, 4, 5, 6))
    scale = wR.abs().sum((1, 2, 3, 4, 5, 6))
    assert float((tot.abs() / scale).max()) < 1e-13


def _mirror_x(U):
    """The state reflected across x = const: element and node order along x reversed,
    S_x negated (D, S_y, S_z and tau are even)."""
    M = U.flip(3).flip(6).clone()
    M[1] = -M[1]
    return M


@pytest.mark.parametrize("dim,p,eos,flux", [(1, 2, IDEAL, 0), (1, 3, TM, 1), (2, 1, TM, 0), (2, 2, IDEAL, 1)])
def test_reflecting_wall_equals_mirrored_periodic_mesh(dim, p, eos, flux):
    """Walls at both ends in x give the RHS of a periodic mesh of twice the length that
    holds the state followed by its mirror image (the image supplies the exterior
    state at each wall)."""
    from oracle.setup import REFLECT
    ny = 3 if dim > 1 else 1
    st = Setup(dim=dim, p=p, n_elem=(5, ny, 1), eos=eos, bc=(REFLECT, PERIODIC, PERIODIC), flux=flux)
    st2 = Setup(dim=dim, p=p, n_elem=(10, ny, 1), lo=(0.0, 0.0, 0.0), hi=(2.0, 1.0, 1.0), eos=eos,
                bc=(PERIODIC, PERIODIC, PERIODIC), flux=flux)
    U = _random_state(st, np.random.default_rng(60 + dim + p), gmax=2.0)
    U2 = torch.cat([U, _mirror_x(U)], 3)
    R = dg.rhs(U, st)
    R2 = dg.rhs(U2, st2)[:, :, :, :5]
    err = (R - R2).abs().amax(dim=(1, 2, 3, 4, 5, 6)) / R2.abs().amax(dim=(1, 2, 3, 4, 5, 6))
    assert float(err.max()) < 1e-12, err.tolist()


@pytest.mark.parametrize("dim,p,eos,flux", [(2, 2, TM, 0), (3, 1, IDEAL, 1)])
def test_closed_box_conserves_mass_and_energy(dim, p, eos, flux):
    """Walls on every side: no mass or energy crosses the boundary (the HLL and HLLC
    mass and energy fluxes vanish between a state and its mirror image)."""
    from oracle.setup import REFLECT
    st = Setup(dim=dim, p=p, n_elem=(4, 3, 3)[:dim] + (1,) * (3 - dim), eos=eos, bc=(REFLECT,) * 3, flux=flux)
    U = _random_state(st, np.random.default_rng(70 + dim))
    wR = dg.rhs(U, st) * dg.elem_weights(st)
    tot = wR.sum((1, 2, 3, 4, 5, 6))
    scale = wR.abs().sum((1, 2, 3, 4, 5, 6))
    assert float(tot[0].abs() / scale[0]) < 1e-13 and float(tot[-1].abs() / scale[-1]) < 1e-13
    # momentum is not conserved: the walls push back
    assert float((tot[1:-1].abs() / scale[1:-1]).max()) > 1e-6


def test_dirichlet_ends_take_the_fixed_state_in_the_flux():
    """p = 0, three cells: the boundary fluxes are the numerical flux between the fixed
    exterior state and the adjacent cell (fixed state on the outer side)."""
    from oracle.setup import DIRICHLET, REFLECT
    lo_state, hi_state = (2.0, 0.3, 0.0, 0.0, 1.5), (0.5, -0.2, 0.0, 0.0, 0.4)
    st = Setup(dim=1, p=0, n_elem=(3, 1, 1), bc=(DIRICHLET, 0, 0), bc_hi=(DIRICHLET, 0, 0),
               bc_state={(0, 0): lo_state, (0, 1): hi_state})
    U = _random_state(st, np.random.default_rng(80))
    W, _ = cp.con2prim(U, st)
    R = dg.rhs(U, st)

    def prim(s):
        return torch.cat([torch.tensor([s[0]]), srhd.u_from_v(torch.tensor([s[1]]), 1.0), torch.tensor([s[4]])])[:, None]

    Wc = [W[:, 0, 0, i, 0, 0, 0][:, None] for i in range(3)]
    F = [srhd.hll(prim(lo_state), Wc[0], 0, st), srhd.hll(Wc[0], Wc[1], 0, st),
         srhd.hll(Wc[1], Wc[2], 0, st), srhd.hll(Wc[2], prim(hi_state), 0, st)]
    for i in range(3):
        expect = -(F[i + 1] - F[i])[:, 0] / st.dx(0)
        got = R[:, 0, 0, i, 0, 0, 0]
        assert torch.allclose(got, expect, rtol=1e-13, atol=1e-13 * float(expect.abs().max())), (i, got, expect)
    # a wall at the upper end instead: the mirror image is the exterior state there
    st2 = Setup(dim=1, p=0, n_elem=(3, 1, 1), bc=(DIRICHLET, 0, 0), bc_hi=(REFLECT, 0, 0),
                bc_state={(0, 0): lo_state})
    R2 = dg.rhs(U, st2)
    Wm = Wc[2].clone()
    Wm[1] = -Wm[1]
    expect = -(srhd.hll(Wc[2], Wm, 0, st) - F[2])[:, 0] / st.dx(0)
    assert torch.allclose(R2[:, 0, 0, 2, 0, 0, 0], expect, rtol=1e-13, atol=1e-13 * float(expect.abs().max()))


def test_uniform_state_with_matching_dirichlet_ends_is_steady():
    from oracle.setup import DIRICHLET
    v = (0.2, -0.1)
    st = Setup(dim=2, p=2, n_elem=(4, 3, 1), eos=TM, bc=(DIRICHLET, DIRICHLET, 0),
               bc_state={(d, e): (1.3, v[0], v[1], 0.0, 0.7) for d in range(2) for e in range(2)})
    rho = torch.full(st.shape(), 1.3)
    vel = torch.stack([torch.full(st.shape(), v[0]), torch.full(st.shape(), v[1])])
    U = srhd.prim3_to_cons(rho, vel, torch.full(st.shape(), 0.7), st)
    R = dg.rhs(U, st)
    W, _ = cp.con2prim(U, st)
    fmax = max(float(srhd.flux(W, d, st).abs().max()) * 2 / st.dx(d) for d in range(2))
    assert float(R.abs().max()) <= 1e-13 * fmax * 9


# ---- reading R12: a trace whose interpolated rho or P is <= 0 takes the primitive
# state of the node nearest that face on the same line, and is counted

def _prims_from_nodes(st, rho, v, P):
    return srhd.prim3_to_cons(torch.tensor(rho), torch.tensor(v), torch.tensor(P), st)


def test_trace_fallback_density_1d():
    """p = 2: l(-1) = (1.4789, -0.6667, 0.1878) on the GL nodes, so node densities
    (0.01, 1, 1) interpolate to about -0.46 at x = -1: the - trace must equal node 0's
    primitives exactly; the + trace (about 0.81) is the interpolant itself."""
    st = Setup(dim=1, p=2, n_elem=(3, 1, 1), eos=IDEAL)
    shape = st.shape()
    rho = np.ones(shape)
    rho[0, 0, 1, 0, 0, :] = (0.01, 1.0, 1.0)   # element 1
    v = np.full((1,) + shape, 0.2)
    P = np.full(shape, 0.5)
    U = _prims_from_nodes(st, rho, v, P)
    W, _ = cp.con2prim(U, st)
    Wm, Wp, nfb = dg.traces(W, 0, st)
    assert nfb == 1
    # element 1's - trace is its node 0 (the node nearest x = -1), bit for bit
    assert torch.equal(Wm[:, 0, 0, 1, 0, 0], W[:, 0, 0, 1, 0, 0, 0])
    r = np.sqrt(0.6)  # l_a(+1) on the nodes (-r, 0, r), written out from the product formula
    lp = np.array([(1.0 - r) / 1.2, -2.0 / 3.0, (1.0 + r) / 1.2])
    for k in range(st.nvar):
        ref = float((torch.tensor(lp) * W[k, 0, 0, 1, 0, 0, :]).sum())
        assert abs(float(Wp[k, 0, 0, 1, 0, 0]) - ref) <= 1e-15 * max(1.0, abs(ref))
    assert float(Wp[0, 0, 0, 1, 0, 0]) > 0.5
    # the other elements are uniform: their traces are the node states
    assert torch.allclose(Wm[:, 0, 0, 0, 0, 0], W[:, 0, 0, 0, 0, 0, 1], rtol=1e-14, atol=0)


def test_trace_fallback_pressure_2d_along_y():
    """The same for the pressure on the + face along y of a p = 3 element: pressures
    (1, 1, 1, 0.001) up one column interpolate to < 0 at y = +1 (l(+1) has weight
    -0.81 on the third node and 1.53 on the fourth), so that face point takes the
    primitives of the node nearest y = +1; the counter counts that one point."""
    st = Setup(dim=2, p=3, n_elem=(2, 2, 1), eos=TM, bc=(PERIODIC, OUTFLOW, PERIODIC))
    shape = st.shape()
    rho = np.ones(shape)
    P = np.ones(shape)
    # element (ex=1, ey=0), column i = 2: nodes j = 0..3
    P[0, 0, 1, 0, :, 2] = (1.0, 1.0, 1.0, 0.001)
    v = np.zeros((2,) + shape)
    v[0] = 0.1
    U = _prims_from_nodes(st, rho, v, P)
    W, _ = cp.con2prim(U, st)
    Wm, Wp, nfb = dg.traces(W, 1, st)
    assert nfb == 1
    assert float(Wp[-1, 0, 0, 1, 0, 2]) == float(W[-1, 0, 0, 1, 0, 3, 2])
    assert torch.equal(Wp[:, 0, 0, 1, 0, 2], W[:, 0, 0, 1, 0, 3, 2])
    # the surface term counts the same fallback through its stats
    stats = {}
    dg.surface_term(W, st, stats)
    assert stats["trace_fallbacks"] == 1
