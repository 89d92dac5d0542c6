"""Seeded synthetic workloads (initial primitive fields) for the DG SRHD path.

This module is the only code shared by the GPU path and the CPU oracle.  It
holds no step of the method itself: no equation of state, no
primitive-to-conserved map, no basis contraction.  It only

* describes each workload as a plain dictionary (mesh, equation of state,
  time step, step count), and
* evaluates the initial primitive fields (rest-mass density, 3-velocity,
  pressure) at the node positions of a Gauss-Legendre nodal mesh.  The sample
  positions come from ``numpy.polynomial.legendre.leggauss``; the discrete
  operators on each side build their own tables.

Layouts: a scalar field has shape ``[nez, ney, nex, nk, nj, ni]`` (C order, the
x node index ``i`` fastest); a vector field has a leading component axis of
length ``dim``.  Unused dimensions have extent 1.

Workloads (the paper's tests they stand in for are named per function):

* ``wave1d``    smooth density wave advected at v=0.5 (exact translated
                solution), 1D periodic, ideal EOS.
* ``kh``        relativistic Kelvin-Helmholtz shear layers (stands in for the
                paper's Kelvin-Helmholtz performance and growth-rate runs).
* ``random3d``  3D periodic cube of i.i.d. lognormal densities/pressures and
                random-direction velocities with Lorentz factor up to 20, a
                stress case for the physicality-enforcing operator.
* ``blast2d``   cylindrical blast wave (pressure ratio 1000 across a circle), 2D,
                outflow, slope limiter on: the shock workload at scale (the
                paper's limited runs are its 1D Riemann problems).
"""
from __future__ import annotations

import numpy as np

PERIODIC, OUTFLOW, REFLECT, DIRICHLET = 0, 1, 2, 3
EOS_IDEAL, EOS_TM = 0, 1
C2P_NEWTON, C2P_QUARTIC, C2P_CUBIC, C2P_BRENT = 0, 1, 2, 3
FP64, FP32_CONTRACT, FP32_MFMA = 0, 1, 2
FLUX_HLL, FLUX_HLLC = 0, 1


def cfl_dt(cfg: dict) -> float:
    """Fixed step: C * min_d(dx_d) / c with C = 0.1/(2p+1)."""
    dim, p = cfg["dim"], cfg["p"]
    dx = [(cfg["hi"][d] - cfg["lo"][d]) / cfg["n_elem"][d] for d in range(dim)]
    return 0.1 / (2 * p + 1) * min(dx) / cfg["c"]


def make_config(kind: str, **over) -> dict:
    """Return the workload dictionary for one of the named configurations.

    Named configurations:
      ``wave1d``      1D, 64 elements, p=2, ideal Gamma=4/3, 100 SSP-RK3 steps.
      ``kh_tm``       2D KH, Taub-Matthews EOS, 256x256 elements, p=3, FP64.
      ``kh_tm_fp32``  2D KH, Taub-Matthews EOS, 512x512 elements, p=3,
                      FP32 contractions, 50 steps.
      ``kh_ideal``    2D KH, ideal Gamma=4/3, 128x128 elements, p=2, FP64,
                      200 steps (the adjoint workload).
      ``kh_paper``    the paper's KH performance setup (Sec. 4): one shear
                      interface on [-0.5,0.5]x[-1,1], nx x 2nx elements
                      (``nx=`` keyword, default 256), ideal Gamma=4/3, p from
                      the keyword (default 2) with the RK order p+1.
      ``sound``       a small-amplitude sound wave at rest on the periodic unit
                      square/cube (``dim=`` 1, 2 or 3, wave vector 2 pi (1,..,1)),
                      ideal Gamma=4/3: the linear-wave convergence test.
      ``random3d``    3D periodic 64^3 elements, p=2, ideal Gamma=4/3,
                      FP32 contractions, physicality operator on, 20 steps.
      ``blast2d``     2D cylindrical blast, 512x512 elements, p=2, ideal
                      Gamma=5/3, HLLC, slope limiter and operator on, 20 steps.
    Keyword overrides replace entries (e.g. ``n_elem=(8, 8, 1)``).
    """
    if kind == "wave1d":
        cfg = dict(dim=1, p=2, n_elem=(64, 1, 1), lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0),
                   bc=(PERIODIC, PERIODIC, PERIODIC), eos=EOS_IDEAL, gamma_ad=4.0 / 3.0,
                   c=1.0, c2p=C2P_NEWTON, precision=FP64, phys=True, steps=100, init="wave1d")
    elif kind in ("kh_tm", "kh_tm_fp32", "kh_ideal"):
        n = {"kh_tm": 256, "kh_tm_fp32": 512, "kh_ideal": 128}[kind]
        cfg = dict(dim=2, p=3, n_elem=(n, n, 1), lo=(0.0, -1.0, 0.0), hi=(1.0, 1.0, 1.0),
                   bc=(PERIODIC, OUTFLOW, PERIODIC), eos=EOS_TM, gamma_ad=4.0 / 3.0,
                   c=1.0, c2p=C2P_NEWTON, precision=FP64, phys=True, steps=100, init="kh")
        if kind == "kh_tm_fp32":
            cfg.update(precision=FP32_CONTRACT, steps=50)
        if kind == "kh_ideal":
            cfg.update(p=2, eos=EOS_IDEAL, c2p=C2P_NEWTON, steps=200, init="kh_adjoint")
    elif kind == "kh_paper":
        nx = over.pop("nx", 256)
        p = over.get("p", 2)
        cfg = dict(dim=2, p=p, n_elem=(nx, 2 * nx, 1), lo=(-0.5, -1.0, 0.0), hi=(0.5, 1.0, 1.0),
                   bc=(PERIODIC, OUTFLOW, PERIODIC), eos=EOS_IDEAL, gamma_ad=4.0 / 3.0,
                   c=1.0, c2p=C2P_NEWTON, precision=FP64, phys=True, steps=100, init="kh_paper",
                   rk_order=min(p + 1, 3))
    elif kind == "sound":
        dim = over.get("dim", 1)
        cfg = dict(dim=dim, p=2, n_elem=(16, 16 if dim > 1 else 1, 16 if dim > 2 else 1), lo=(0.0, 0.0, 0.0),
                   hi=(1.0, 1.0, 1.0), bc=(PERIODIC, PERIODIC, PERIODIC), eos=EOS_IDEAL, gamma_ad=4.0 / 3.0,
                   c=1.0, c2p=C2P_NEWTON, precision=FP64, phys=True, steps=100, init="sound")
    elif kind == "random3d":
        cfg = dict(dim=3, p=2, n_elem=(64, 64, 64), lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0),
                   bc=(PERIODIC, PERIODIC, PERIODIC), eos=EOS_IDEAL, gamma_ad=4.0 / 3.0,
                   c=1.0, c2p=C2P_NEWTON, precision=FP32_CONTRACT, phys=True, steps=20,
                   init="random3d")
    elif kind == "blast2d":
        # p = 2 with SSP-RK3 and the slope limiter, as the paper's limited shock runs
        cfg = dict(dim=2, p=2, n_elem=(512, 512, 1), lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0),
                   bc=(OUTFLOW, OUTFLOW, OUTFLOW), eos=EOS_IDEAL, gamma_ad=5.0 / 3.0,
                   c=1.0, c2p=C2P_NEWTON, precision=FP64, phys=True, steps=20, init="blast",
                   flux=FLUX_HLLC, limiter=1)
    else:
        raise ValueError(f"unknown workload {kind!r}")
    cfg["kind"] = kind
    cfg.update(over)
    cfg["n_elem"] = tuple(int(v) for v in cfg["n_elem"])
    if "dt" not in over:
        cfg["dt"] = cfl_dt(cfg)
    return cfg


def n_var(cfg: dict) -> int:
    return 2 + cfg["dim"]


def field_shape(cfg: dict) -> tuple:
    """Shape [nez, ney, nex, nk, nj, ni] of one scalar nodal field."""
    dim, p = cfg["dim"], cfg["p"]
    nx, ny, nz = cfg["n_elem"]
    q = p + 1
    return (nz if dim > 2 else 1, ny if dim > 1 else 1, nx,
            q if dim > 2 else 1, q if dim > 1 else 1, q)


def n_dof(cfg: dict) -> int:
    """Nodes per component: n_elements * (p+1)^dim."""
    return int(np.prod(field_shape(cfg)))


def node_coords(cfg: dict) -> list:
    """Physical coordinates (x, y, z) of every node, each shaped like field_shape."""
    dim, p = cfg["dim"], cfg["p"]
    xi, _ = np.polynomial.legendre.leggauss(p + 1)
    shape = field_shape(cfg)
    out = []
    for d in range(3):
        if d >= dim:
            out.append(np.full(shape, 0.5 * (cfg["lo"][d] + cfg["hi"][d])))
            continue
        n = cfg["n_elem"][d]
        h = (cfg["hi"][d] - cfg["lo"][d]) / n
        e = np.arange(n)
        pos = cfg["lo"][d] + (e[:, None] + 0.5 * (xi[None, :] + 1.0)) * h  # [n, q]
        # element axis index in shape: x->2, y->1, z->0 ; node axis: x->5, y->4, z->3
        ea, na = 2 - d, 5 - d
        bshape = [1] * 6
        bshape[ea], bshape[na] = n, p + 1
        out.append(np.broadcast_to(pos.reshape(bshape), shape).copy())
    return out


def wave1d_primitives(cfg: dict, t: float = 0.0):
    """Smooth density wave rho = 1 + 0.5 sin(2 pi (x - 0.5 t)), v = 0.5 c, P = 1.

    With uniform velocity and pressure every flux advects, so the translated
    profile is an exact solution of the SRHD system (a contact/entropy wave;
    the 1D member of the paper's linear-wave family).
    """
    x = node_coords(cfg)[0]
    rho = 1.0 + 0.5 * np.sin(2.0 * np.pi * (x - 0.5 * cfg["c"] * t))
    v = np.zeros((cfg["dim"],) + rho.shape)
    v[0] = 0.5 * cfg["c"]
    P = np.ones_like(rho)
    return rho, v, P


def kh_primitives(cfg: dict, seed: int = 2):
    """Two smooth relativistic shear layers at |y| = 0.5 (x periodic, y outflow).

    rho = 0.55 - 0.45 tanh((|y|-0.5)/0.01)           (1 inside, 0.1 outside)
    v_x = 0.5 tanh((|y|-0.5)/0.01)                     (+-0.5 c)
    v_y = 0.01 sin(2 pi x) exp(-(|y|-0.5)^2/0.01) + U(-1e-4, 1e-4) per node
    P   = 1.
    For ``init == "kh_adjoint"`` the uniform noise is replaced by nothing; the
    perturbation field of the gradient is added separately (kh_perturbation).
    """
    x, y, _ = node_coords(cfg)
    c = cfg["c"]
    a = np.abs(y) - 0.5
    rho = 0.55 - 0.45 * np.tanh(a / 0.01)
    v = np.zeros((cfg["dim"],) + rho.shape)
    v[0] = 0.5 * c * np.tanh(a / 0.01)
    v[1] = 0.01 * c * np.sin(2.0 * np.pi * x) * np.exp(-a * a / 0.01)
    if cfg.get("init", "kh") == "kh":
        rng = np.random.default_rng(seed)
        v[1] += c * rng.uniform(-1e-4, 1e-4, size=rho.shape)
    P = np.ones_like(rho)
    return rho, v, P


def kh_paper_primitives(cfg: dict):
    """One smooth relativistic shear interface at y = 0 (the paper's KH setup of
    its Sec. 4 with the unprinted profile read as):
    rho = 1, P = c^2, v_x = 0.25 c tanh(y / 0.01),
    v_y = 0.05 * 0.25 c sin(2 pi x) exp(-y^2 / 0.01)."""
    x, y, _ = node_coords(cfg)
    c = cfg["c"]
    rho = np.ones_like(x)
    v = np.zeros((cfg["dim"],) + x.shape)
    v[0] = 0.25 * c * np.tanh(y / 0.01)
    v[1] = 0.05 * 0.25 * c * np.sin(2.0 * np.pi * x) * np.exp(-y * y / 0.01)
    P = np.full_like(x, c * c)
    return rho, v, P


def sound_primitives(cfg: dict, t: float = 0.0, amp: float = 1e-6):
    """Right-going acoustic eigenvector of special-relativistic hydrodynamics
    linearised about rest (rho0 = 1, P0 = 1, c = 1, ideal gas): with
    cs^2 = Gamma P0 / (rho0 h0), h0 = 1 + Gamma/(Gamma-1) P0/rho0 and phase
    phi = k.x - |k| cs t, the exact linear solution is
    v = amp sin(phi) k/|k|,  P = P0 + rho0 h0 cs amp sin(phi),
    rho = rho0 + rho0 amp sin(phi) / cs.
    One period later it returns to the initial state; its deviation from the
    nonlinear solution is O(amp^2)."""
    coords = node_coords(cfg)
    dim = cfg["dim"]
    gam = cfg["gamma_ad"]
    rho0, P0 = 1.0, 1.0
    h0 = 1.0 + gam / (gam - 1.0) * P0 / rho0
    cs = np.sqrt(gam * P0 / (rho0 * h0))
    k = np.full(dim, 2.0 * np.pi)
    kn = np.linalg.norm(k)
    phase = sum(k[d] * coords[d] for d in range(dim)) - kn * cs * t
    w = amp * np.sin(phase)
    v = np.stack([w * k[d] / kn for d in range(dim)])
    P = P0 + rho0 * h0 * cs * w
    rho = rho0 + rho0 * w / cs
    return rho, v, P


def wave_frame(dim: int):
    """Unit wave vector and transverse directions of the linear-wave tests (Sec. 4): in 3D
    the rotation of the paper about a = (0, -1, 1)/sqrt(2) by theta = atan(sqrt(2)) (its
    wave-angle formula with N = 3, n = 2) applied to e_x, e_y, e_z (e_x goes to the body
    diagonal); in 2D the in-plane diagonal and its in-plane normal; in 1D e_x."""
    if dim == 1:
        return np.array([1.0]), []
    if dim == 2:
        return np.array([1.0, 1.0]) / np.sqrt(2.0), [np.array([-1.0, 1.0]) / np.sqrt(2.0)]
    a = np.array([0.0, -1.0, 1.0]) / np.sqrt(2.0)
    th = np.arctan(np.sqrt(2.0))
    K = np.array([[0.0, -a[2], a[1]], [a[2], 0.0, -a[0]], [-a[1], a[0], 0.0]])
    R = np.cos(th) * np.eye(3) + (1.0 - np.cos(th)) * np.outer(a, a) + np.sin(th) * K
    return R[:, 0], [R[:, 1], R[:, 2]]


def zero_mode_primitives(cfg: dict, mode: str, amp: float = 1e-6):
    """The linear waves of zero speed at rest (rho0 = P0 = 1, phase k.x with k = 2 pi
    times the diagonal of the unit cell, as sound_primitives): 'entropy' (the 0^(1)
    family: rho = rho0 + amp sin(k.x), v = 0, P = P0) and 'shear2' / 'shear3' (0^(2),
    0^(3): v = amp sin(k.x) t with t the first / second transverse direction of
    wave_frame, rho = rho0, P = P0).  A density profile at rest under uniform pressure,
    and a parallel shear flow with uniform density and pressure (its velocity normal to
    the direction it varies in, so it carries no mass or momentum across the planes of
    constant phase), are exact stationary solutions of the full equations: the exact
    solution at every time is the initial state."""
    coords = node_coords(cfg)
    dim = cfg["dim"]
    k = np.full(dim, 2.0 * np.pi)
    phase = sum(k[d] * coords[d] for d in range(dim))
    w = amp * np.sin(phase)
    rho = np.ones_like(w)
    P = np.ones_like(w)
    v = np.zeros((dim,) + w.shape)
    if mode == "entropy":
        rho = rho + w
    else:
        _, ts = wave_frame(dim)
        t = ts[0] if mode == "shear2" else ts[1]
        v = np.stack([w * t[d] for d in range(dim)])
    return rho, v, P


def sound_period(cfg: dict) -> float:
    """Time for the sound wave of sound_primitives to travel one wavelength."""
    gam = cfg["gamma_ad"]
    h0 = 1.0 + gam / (gam - 1.0)
    cs = np.sqrt(gam / h0)
    return 1.0 / (np.sqrt(cfg["dim"]) * cs)


def kh_perturbation(cfg: dict, seed: int = 4, sigma: float = 1e-3):
    """Seeded Gaussian per-node perturbation of the initial v_y (sigma = 1e-3 c)."""
    rng = np.random.default_rng(seed)
    return cfg["c"] * sigma * rng.standard_normal(field_shape(cfg))


def random_directions(cfg: dict, count: int, seed: int = 41):
    """``count`` seeded unit vectors in the space of per-node v_y perturbations."""
    rng = np.random.default_rng(seed)
    out = rng.standard_normal((count,) + field_shape(cfg))
    out /= np.sqrt((out.reshape(count, -1) ** 2).sum(axis=1)).reshape((count,) + (1,) * 6)
    return out


def random3d_primitives(cfg: dict, seed: int = 5):
    """i.i.d. per node: rho, P ~ clip(exp(N(0, 1.5^2)), 1e-4, 1e2); direction
    uniform on the sphere; Lorentz factor ~ U[1, 20]."""
    rng = np.random.default_rng(seed)
    shape = field_shape(cfg)
    rho = np.clip(np.exp(rng.normal(0.0, 1.5, size=shape)), 1e-4, 1e2)
    P = np.clip(np.exp(rng.normal(0.0, 1.5, size=shape)), 1e-4, 1e2)
    lor = rng.uniform(1.0, 20.0, size=shape)
    n = rng.standard_normal((3,) + shape)
    n /= np.sqrt((n * n).sum(axis=0))
    speed = cfg["c"] * np.sqrt(1.0 - 1.0 / (lor * lor))
    v = (n * speed)[: cfg["dim"]]
    return rho, v, P


def blast_primitives(cfg: dict):
    """At rest, density 1; pressure 100 within radius 0.2 of the domain's centre, 0.1
    outside (a cylinder in 2D, a sphere in 3D)."""
    X = node_coords(cfg)
    r2 = sum((X[d] - 0.5 * (cfg["lo"][d] + cfg["hi"][d])) ** 2 for d in range(cfg["dim"]))
    shape = field_shape(cfg)
    P = np.where(r2 < 0.04, 100.0, 0.1)
    return np.ones(shape), np.zeros((cfg["dim"],) + shape), P


def initial_primitives(cfg: dict, seed: int | None = None):
    """Dispatch on cfg['init']; returns (rho, v, P) with v the 3-velocity."""
    init = cfg.get("init")
    if init == "wave1d":
        return wave1d_primitives(cfg)
    if init in ("kh", "kh_adjoint"):
        return kh_primitives(cfg, seed=2 if seed is None else seed)
    if init == "random3d":
        return random3d_primitives(cfg, seed=5 if seed is None else seed)
    if init == "kh_paper":
        return kh_paper_primitives(cfg)
    if init == "sound":
        return sound_primitives(cfg)
    if init in ("entropy", "shear2", "shear3"):
        return zero_mode_primitives(cfg, init)
    if init == "blast":
        return blast_primitives(cfg)
    raise ValueError(f"unknown init {init!r}")


def pack_primitives(rho, v, P) -> np.ndarray:
    """Stack (rho, v_1..v_dim, P) into one [n_var, ...] float64 array."""
    return np.ascontiguousarray(np.concatenate([rho[None], v, P[None]], axis=0), dtype=np.float64)


def c2p_grid(n: int = 25, c: float = 3.0e8, D: float = 1.0):
    """The paper's recovery-accuracy grid: n log-spaced Lorentz factors in
    [1, 100] times n log-spaced pressures in [1e5, 1e10] Pa, D = 1 kg/m^3,
    c = 3e8 m/s.  Returns (gamma, P) meshgrids (gamma varies along axis 1)."""
    g = np.logspace(0.0, 2.0, n)
    P = np.logspace(5.0, 10.0, n)
    G, PP = np.meshgrid(g, P)
    return G, PP

