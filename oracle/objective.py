"""Kelvin-Helmholtz diagnostic: J = integral of v_y^2 over the domain.  Test infrastructure.

The paper tracks the spatial mean of v_y^2 (Sec. 4, Kelvin-Helmholtz linear
growth phase); J is that integral without the 1/|Omega| factor, evaluated with
the collocated GL quadrature: J = sum_e sum_i (prod_d dx_d/2) w_i v_y,i^2,
v_y = u_y / gamma from the recovered primitives.  Its gradient is taken by
torch autograd through con2prim (the oracle's reverse mode).

Pinned by tests/test_oracle_objective.py against closed-form integrals: a
uniform v_y gives v_y^2 x area (2D and 3D), a separable polynomial field of
degree <= p per element gives its exact integral, and A sin(2 pi x) gives A^2
on the Kelvin-Helmholtz domain (a dropped Jacobian factor, a missing weight or
u_y in place of v_y fails them).
"""
from __future__ import annotations

from .con2prim import con2prim
from .dg import elem_weights
from .srhd import lorentz


def vy2_integral(U, st):
    W, _ = con2prim(U, st)
    u = W[1:-1]
    vy = u[1] / lorentz(u, st.c)
    jac = 1.0
    for d in range(st.dim):
        jac *= 0.5 * st.dx(d)
    return (jac * elem_weights(st)[0] * vy * vy).sum()
