"""Plain FP64 CPU oracle of the DG special-relativistic hydrodynamics path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or links
this package: it is used by ``tests/``, by the smoke check of the package entry
module and by the CPU-baseline leg of the benchmark.  It shares no code with
the GPU path (kernels, headers, basis tables or helpers); the only common
module is the seeded workload generator, which holds none of the method's
arithmetic.

Everything is plain PyTorch on the CPU in float64 (autograd-capable, which
gives the oracle its own reverse-mode gradient) plus numpy/scipy library
routines for the Gauss-Legendre rule, polynomial algebra and Brent's method.
Each step follows the paper in its order and notation:

* ``basis``        nodal Lagrange basis on Gauss-Legendre nodes (Sec. 2.3)
* ``eos``          ideal and Taub-Matthews equations of state (Sec. 2.2)
* ``srhd``         primitive-to-conserved map, fluxes (Sec. 2.1), wavespeeds
                   and the HLL and HLLC numerical fluxes (Sec. 2.4)
* ``con2prim``     the four conserved-to-primitive solvers (Sec. 3.1, 3.2)
* ``dg``           the DG weak-form right-hand side (Sec. 2.3, Eqs. for the
                   volume and surface quadratures) with periodic, outflow,
                   reflecting-wall and fixed-state boundaries
* ``physicality``  the physicality-enforcing operator (Sec. 2.5)
* ``timestep``     SSP-RK1/2/3 with the operator after each stage (Sec. 2.3)
* ``objective``    the integral of v_y^2 (the Kelvin-Helmholtz diagnostic)

Parity status per function is stated in each module header.  Every function
is pinned; the analytic ideal-gas quartic solver (``con2prim.ideal_quartic``)
is pinned on the velocities where its formula holds its digits (beta in
[0.3, 0.99]) and only measured below that.
"""
from .setup import Setup  # noqa: F401
