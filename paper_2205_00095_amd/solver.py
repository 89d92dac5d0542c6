"""Python face of the C ABI: one ``Solver`` per mesh, torch tensors for device memory.

Every method marshals torch tensor pointers and the current HIP stream into one
C-ABI call; the arithmetic runs in the library's gfx950 kernels.  Tensors must
be float64, contiguous, on the GPU, shaped [n_var, nez, ney, nex, nk, nj, ni].
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from .workloads import field_shape


def _desc_from_config(cfg: dict, sync: bool) -> _lib.MeshDesc:
    d = _lib.MeshDesc()
    d.dim, d.p = cfg["dim"], cfg["p"]
    for k in range(3):
        d.n_elem[k] = int(cfg["n_elem"][k]) if k < cfg["dim"] else 1
        d.lo[k] = float(cfg["lo"][k])
        d.hi[k] = float(cfg["hi"][k])
        d.bc[k] = int(cfg["bc"][k])
    d.eos = int(cfg["eos"])
    d.gamma_ad = float(cfg["gamma_ad"])
    d.c_light = float(cfg["c"])
    d.c2p = int(cfg.get("c2p", -1))
    d.precision = int(cfg.get("precision", 0))
    d.phys = 1 if cfg.get("phys", True) else 0
    d.phys_eps = float(cfg.get("phys_eps", 1e-12))
    d.sync_mode = 1 if sync else 0
    d.flux = int(cfg.get("flux", 0))
    for k, t in enumerate(cfg.get("bc_hi", (0, 0, 0))):
        d.bc_hi[k] = int(t)
    d.c2p_iters = int(cfg.get("c2p_iters", 0))
    d.limiter = int(cfg.get("limiter", 0))
    for (k, end), state in cfg.get("bc_state", {}).items():
        for i in range(5):
            d.bc_state[(k * 2 + end) * 5 + i] = float(state[i])
    return d


class Solver:
    """DG SRHD solver context on the current GPU (see include/dgsrhd.h)."""

    def __init__(self, cfg: dict, sync: bool = False):
        if not torch.cuda.is_available():
            raise RuntimeError("dgsrhd needs a ROCm GPU (torch.cuda.is_available() is False)")
        self.lib = _lib.load()
        self.cfg = dict(cfg)
        self.nvar = cfg["dim"] + 2
        self.shape = (self.nvar,) + field_shape(cfg)
        self.numel = 1
        for s in self.shape:
            self.numel *= s
        self.device = torch.device("cuda", torch.cuda.current_device())
        desc = _desc_from_config(cfg, sync)
        ctx = ctypes.c_void_p()
        rc = self.lib.dg_init_mesh(ctypes.byref(desc), ctypes.c_void_p(self._stream()), ctypes.byref(ctx))
        if rc != 0:
            raise _lib.DGError(rc, "dg_init_mesh", "invalid description or allocation failure")
        self.ctx = ctx
        n = self.lib.dg_state_size(self.ctx)
        if n != self.numel:
            raise RuntimeError(f"state size mismatch {n} != {self.numel}")

    # ------------------------------------------------------------ plumbing
    @staticmethod
    def _stream() -> int:
        return torch.cuda.current_stream().cuda_stream

    def _sync_stream(self):
        rc = self.lib.dg_set_stream(self.ctx, ctypes.c_void_p(self._stream()))
        self._check(rc, "dg_set_stream")

    def _check(self, rc: int, where: str):
        if rc != 0:
            msg = self.lib.dg_last_error(self.ctx).decode(errors="replace")
            raise _lib.DGError(rc, where, msg)

    def _ptr(self, t: torch.Tensor, name: str) -> ctypes.c_void_p:
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a torch tensor")
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous float64 GPU tensor")
        if t.numel() != self.numel:
            raise ValueError(f"{name} has {t.numel()} elements, expected {self.numel}")
        return ctypes.c_void_p(t.data_ptr())

    def empty(self) -> torch.Tensor:
        return torch.empty(self.shape, dtype=torch.float64, device=self.device)

    # ------------------------------------------------------------ C-ABI calls
    def set_state(self, src: torch.Tensor, kind: int = _lib.PRIMITIVE, out: torch.Tensor | None = None):
        U = self.empty() if out is None else out
        self._sync_stream()
        self._check(self.lib.dg_set_state(self.ctx, kind, self._ptr(src, "src"), self._ptr(U, "U")),
                    "dg_set_state")
        return U

    def con2prim(self, U: torch.Tensor, out: torch.Tensor | None = None):
        W = self.empty() if out is None else out
        self._sync_stream()
        self._check(self.lib.dg_con2prim(self.ctx, self._ptr(U, "U"), self._ptr(W, "W")), "dg_con2prim")
        return W

    def rhs(self, U: torch.Tensor, out: torch.Tensor | None = None):
        R = self.empty() if out is None else out
        self._sync_stream()
        self._check(self.lib.dg_rhs(self.ctx, self._ptr(U, "U"), self._ptr(R, "R")), "dg_rhs")
        return R

    def enforce(self, U: torch.Tensor):
        self._sync_stream()
        self._check(self.lib.dg_enforce_physical(self.ctx, self._ptr(U, "U")), "dg_enforce_physical")
        return U

    def step(self, U: torch.Tensor, dt: float, order: int = 3):
        """One SSP-RK step of the given order (1, 2, 3) in place on U."""
        self._sync_stream()
        if order == 3:
            self._check(self.lib.dg_ssprk3_step(self.ctx, self._ptr(U, "U"), float(dt)), "dg_ssprk3_step")
        else:
            self._check(self.lib.dg_ssprk_step(self.ctx, self._ptr(U, "U"), float(dt), int(order)), "dg_ssprk_step")
        return U

    def run(self, U: torch.Tensor, dt: float, nsteps: int, order: int = 3):
        """nsteps SSP-RK steps of the given order (1, 2, 3) in place on U."""
        self._sync_stream()
        if order == 3:
            self._check(self.lib.dg_ssprk3_run(self.ctx, self._ptr(U, "U"), float(dt), int(nsteps)),
                        "dg_ssprk3_run")
        else:
            self._check(self.lib.dg_ssprk_run(self.ctx, self._ptr(U, "U"), float(dt), int(nsteps), int(order)),
                        "dg_ssprk_run")
        return U

    def graph_run(self, U: torch.Tensor, dt: float, nsteps: int, order: int = 3):
        """Capture `run(U, dt, nsteps, order)` into a HIP graph and return it (a
        torch.cuda.CUDAGraph): each replay advances U by nsteps steps, launching the
        library's kernels without the host (for launch-bound meshes).  The context's
        stream is moved to the capture stream before the capture begins, so the graph
        holds only the library's kernel launches.  Replays use the context's scratch
        like any call: replays and other calls on this context must be ordered (one
        stream, or the caller's events)."""
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            self._sync_stream()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            self.run(U, dt, nsteps, order)
        torch.cuda.current_stream().wait_stream(s)
        return g

    def rhs_vjp(self, U: torch.Tensor, lamR: torch.Tensor, out: torch.Tensor | None = None):
        lamU = self.empty() if out is None else out
        self._sync_stream()
        self._check(self.lib.dg_rhs_vjp(self.ctx, self._ptr(U, "U"), self._ptr(lamR, "lamR"),
                                        self._ptr(lamU, "lamU")), "dg_rhs_vjp")
        return lamU

    def step_vjp(self, Un: torch.Tensor, dt: float, lam_next: torch.Tensor, out: torch.Tensor | None = None):
        lam = self.empty() if out is None else out
        self._sync_stream()
        self._check(self.lib.dg_ssprk3_step_vjp(self.ctx, self._ptr(Un, "Un"), float(dt),
                                                self._ptr(lam_next, "lam_next"), self._ptr(lam, "lam_n")),
                    "dg_ssprk3_step_vjp")
        return lam

    @property
    def tape_numel(self) -> int:
        return int(self.lib.dg_tape_size(self.ctx))

    def _tape_ptr(self, tape: torch.Tensor) -> ctypes.c_void_p:
        if tape.dtype != torch.float64 or not tape.is_cuda or not tape.is_contiguous():
            raise ValueError("tape must be a contiguous float64 GPU tensor")
        if tape.numel() != self.tape_numel:
            raise ValueError(f"tape has {tape.numel()} elements, expected {self.tape_numel}")
        return ctypes.c_void_p(tape.data_ptr())

    def step_tape(self, U: torch.Tensor, dt: float, tape: torch.Tensor):
        self._sync_stream()
        self._check(self.lib.dg_ssprk3_step_tape(self.ctx, self._ptr(U, "U"), float(dt), self._tape_ptr(tape)),
                    "dg_ssprk3_step_tape")
        return U

    def step_vjp_tape(self, tape: torch.Tensor, dt: float, lam_next: torch.Tensor, out: torch.Tensor | None = None):
        lam = self.empty() if out is None else out
        self._sync_stream()
        self._check(self.lib.dg_ssprk3_step_vjp_tape(self.ctx, self._tape_ptr(tape), float(dt),
                                                     self._ptr(lam_next, "lam_next"), self._ptr(lam, "lam_n")),
                    "dg_ssprk3_step_vjp_tape")
        return lam

    def _tapes_ptr(self, tapes: torch.Tensor, nsteps: int) -> ctypes.c_void_p:
        if tapes.dtype != torch.float64 or not tapes.is_cuda or not tapes.is_contiguous():
            raise ValueError("tapes must be a contiguous float64 GPU tensor")
        if tapes.numel() < nsteps * self.tape_numel:
            raise ValueError(f"tapes holds {tapes.numel()} elements, need {nsteps * self.tape_numel}")
        return ctypes.c_void_p(tapes.data_ptr())

    def run_tape(self, U: torch.Tensor, dt: float, nsteps: int, tapes: torch.Tensor):
        self._sync_stream()
        self._check(self.lib.dg_ssprk3_run_tape(self.ctx, self._ptr(U, "U"), float(dt), int(nsteps),
                                                self._tapes_ptr(tapes, nsteps)), "dg_ssprk3_run_tape")
        return U

    def run_vjp_tape(self, tapes: torch.Tensor, dt: float, nsteps: int, lam: torch.Tensor):
        self._sync_stream()
        self._check(self.lib.dg_ssprk3_run_vjp_tape(self.ctx, self._tapes_ptr(tapes, nsteps), float(dt),
                                                    int(nsteps), self._ptr(lam, "lam")), "dg_ssprk3_run_vjp_tape")
        return lam

    def objective_vy2(self, U: torch.Tensor, grad: bool = False):
        J = ctypes.c_double()
        g = self.empty() if grad else None
        self._sync_stream()
        self._check(self.lib.dg_objective_vy2(self.ctx, self._ptr(U, "U"), ctypes.byref(J),
                                              self._ptr(g, "dJdU") if grad else None), "dg_objective_vy2")
        return (J.value, g) if grad else J.value

    def set_state_vjp(self, src: torch.Tensor, lamU: torch.Tensor, out: torch.Tensor | None = None):
        lam = self.empty() if out is None else out
        self._sync_stream()
        self._check(self.lib.dg_set_state_vjp(self.ctx, self._ptr(src, "src"), self._ptr(lamU, "lamU"),
                                              self._ptr(lam, "lam_src")), "dg_set_state_vjp")
        return lam

    def diagnostics(self) -> dict:
        d = _lib.Diag()
        self._check(self.lib.dg_get_diagnostics(self.ctx, ctypes.byref(d)), "dg_get_diagnostics")
        return {name: getattr(d, name) for name, _ in _lib.Diag._fields_}

    def reset_diagnostics(self):
        self._sync_stream()
        self._check(self.lib.dg_reset_diagnostics(self.ctx), "dg_reset_diagnostics")

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.dg_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def primitives_tensor(rho, v, P, device="cuda") -> torch.Tensor:
    """Stack numpy (rho, v, P) into the [n_var, ...] float64 device layout."""
    import numpy as np
    arr = np.concatenate([rho[None], v, P[None]], axis=0)
    return torch.from_numpy(np.ascontiguousarray(arr, dtype=np.float64)).to(device)


def rhs_noalloc(cfg: dict, U: torch.Tensor, R: torch.Tensor, diag: bool = False, sync: bool = False):
    """dg_rhs through the allocation-free entry point (no context, static device scratch).

    R must be preallocated by the caller; with diag=True the call synchronises and
    returns the counters of this call as a dict, else None."""
    if not torch.cuda.is_available():
        raise RuntimeError("dgsrhd needs a ROCm GPU (torch.cuda.is_available() is False)")
    lib = _lib.load()
    shape = (cfg["dim"] + 2,) + field_shape(cfg)
    numel = 1
    for s in shape:
        numel *= s
    for name, t in (("U", U), ("R", R)):
        if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous float64 GPU tensor")
        if t.numel() != numel:
            raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")
    desc = _desc_from_config(cfg, sync)
    d = _lib.Diag() if diag else None
    rc = lib.dg_rhs_noalloc(ctypes.byref(desc), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream),
                            ctypes.c_void_p(U.data_ptr()), ctypes.c_void_p(R.data_ptr()),
                            ctypes.byref(d) if diag else None)
    if rc != 0:
        raise _lib.DGError(rc, "dg_rhs_noalloc", "see stderr")
    return {name: getattr(d, name) for name, _ in _lib.Diag._fields_} if diag else None
