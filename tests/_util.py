"""Small helpers shared by the tests (no method arithmetic)."""
import numpy as np
import torch

from oracle.setup import Setup
from oracle import srhd
from paper_2205_00095_amd import workloads as wl


def oracle_state(cfg, seed=None):
    """(Setup, U) for a workload: the oracle's own prim->cons of the seeded primitives."""
    st = Setup.from_config(cfg)
    rho, v, P = wl.initial_primitives(cfg, seed)
    U = srhd.prim3_to_cons(torch.from_numpy(rho), torch.from_numpy(v), torch.from_numpy(P), st)
    return st, U.reshape((st.nvar,) + wl.field_shape(cfg))


def rel_err_per_var(a, b):
    """max_k ||a_k - b_k||_inf / ||b_k||_inf over conserved components k."""
    a = a.reshape(a.shape[0], -1)
    b = b.reshape(b.shape[0], -1)
    num = (a - b).abs().max(1).values
    den = b.abs().max(1).values.clamp(min=1e-300)
    return (num / den)


def perturbed(U, rel=1e-15, seed=0):
    """U with every entry scaled by (1 + rel * N(0,1)) (a few ulps at rel = 1e-15)."""
    g = torch.Generator().manual_seed(seed)
    return U * (1.0 + rel * torch.randn(U.shape, generator=g, dtype=torch.float64))


def parity_tol(fn, U, floor=1e-12):
    """Acceptance bar for GPU-vs-oracle parity of X = fn(U): 1e-12 normwise relative per
    component, or 4x the oracle's own response to ~5-ulp relative perturbations of its
    input (max over two seeds) when the problem's FP64 conditioning makes that larger
    (cancellation-dominated RHS, chaotic stress data).  Returns (tol, sensitivity)."""
    X0 = fn(U)
    sens = torch.maximum(rel_err_per_var(fn(perturbed(U, seed=0)), X0),
                         rel_err_per_var(fn(perturbed(U, seed=1)), X0))
    # one or two random perturbations under-sample the worst case: allow 4x
    return torch.clamp(4.0 * sens, min=floor), sens
