"""Mesh / physics description used by every oracle routine (test infrastructure)."""
from __future__ import annotations

from dataclasses import dataclass, field

PERIODIC, OUTFLOW, REFLECT, DIRICHLET = 0, 1, 2, 3
IDEAL, TM = 0, 1
NEWTON, QUARTIC, CUBIC, BRENT = 0, 1, 2, 3
HLL, HLLC = 0, 1


@dataclass
class Setup:
    dim: int
    p: int
    n_elem: tuple = (1, 1, 1)
    lo: tuple = (0.0, 0.0, 0.0)
    hi: tuple = (1.0, 1.0, 1.0)
    bc: tuple = (PERIODIC, PERIODIC, PERIODIC)
    bc_hi: tuple = (0, 0, 0)  # type at the upper end when it differs from bc[d]; 0 keeps bc[d]
    bc_state: dict = field(default_factory=dict)  # (d, end) -> (rho, v_x, v_y, v_z, P) of a fixed end
    eos: int = IDEAL
    gamma_ad: float = 4.0 / 3.0
    c: float = 1.0
    c2p: int = -1            # -1: the paper's default solver for the EOS (Newton / cubic)
    phys_eps: float = 1e-12
    flux: int = HLL          # numerical flux: HLL or HLLC (Sec. 2.4)
    c2p_iters: int = 0       # > 0: fixed iteration count of the iterative recovery solvers (Sec. 3.3)
    limiter: int = 0         # 1: the minmod slope limiter after every stage, before the operator
    extra: dict = field(default_factory=dict)

    @staticmethod
    def from_config(cfg: dict) -> "Setup":
        return Setup(dim=cfg["dim"], p=cfg["p"], n_elem=tuple(cfg["n_elem"]), lo=tuple(cfg["lo"]),
                     hi=tuple(cfg["hi"]), bc=tuple(cfg["bc"]), eos=cfg["eos"],
                     gamma_ad=cfg["gamma_ad"], c=cfg["c"], c2p=cfg["c2p"],
                     flux=cfg.get("flux", HLL), bc_hi=tuple(cfg.get("bc_hi", (0, 0, 0))),
                     bc_state=dict(cfg.get("bc_state", {})), c2p_iters=int(cfg.get("c2p_iters", 0)),
                     limiter=int(cfg.get("limiter", 0)))

    @property
    def nvar(self) -> int:
        return 2 + self.dim

    def end_type(self, d: int, end: int) -> int:
        """Boundary type at the lower (end 0) or upper (end 1) end of dimension d."""
        return self.bc_hi[d] if end == 1 and self.bc_hi[d] != 0 else self.bc[d]

    def dx(self, d: int) -> float:
        return (self.hi[d] - self.lo[d]) / self.n_elem[d]

    def shape(self) -> tuple:
        """[nez, ney, nex, nk, nj, ni] of one nodal component."""
        q = self.p + 1
        nx, ny, nz = self.n_elem
        return (nz if self.dim > 2 else 1, ny if self.dim > 1 else 1, nx,
                q if self.dim > 2 else 1, q if self.dim > 1 else 1, q)
