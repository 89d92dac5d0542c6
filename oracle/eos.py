"""Equations of state h(rho, P) and sound speed (Sec. 2.2).  Test infrastructure.

Ideal gas:        h = c^2 + Gamma/(Gamma-1) Theta,        c_s^2/c^2 = Gamma Theta / h
Taub-Matthews:    h = 5/2 Theta + 3/2 sqrt(Theta^2 + 4/9 c^4)
                  c_s^2/c^2 = (3 Theta^2 + 5 Theta s) / (12 Theta^2 + 2 c^4 + 12 Theta s),
                  s = sqrt(Theta^2 + 4/9 c^4)
with Theta = P / rho.

``h_excess`` returns h - c^2 evaluated without cancellation (for the
Taub-Matthews form, 3/2 (s - 2/3 c^2) is rewritten as 3/2 Theta^2/(s + 2/3 c^2));
the conserved energy is stored as tau = E - D c^2, which needs h - c^2 to full
relative precision in the cold limit.

Pinned by tests/test_oracle_eos.py: the general sound-speed definition
c_s^2 = -rho/(n h) dh/drho, n = rho dh/dP - 1 evaluated by automatic
differentiation of h(rho, P); the TM limits Gamma_eq -> 5/3 (cold) and
Gamma_eq -> 4/3, c_s^2 -> c^2/3 (hot).
"""
from __future__ import annotations

import torch

from .setup import IDEAL, TM


def h_excess(theta, eos: int, gamma_ad: float, c: float):
    """h - c^2 as a function of Theta = P/rho."""
    if eos == IDEAL:
        return gamma_ad / (gamma_ad - 1.0) * theta
    if eos == TM:
        s = torch.sqrt(theta * theta + (4.0 / 9.0) * c ** 4)
        return 2.5 * theta + 1.5 * theta * theta / (s + (2.0 / 3.0) * c * c)
    raise ValueError(eos)


def enthalpy(theta, eos: int, gamma_ad: float, c: float):
    return c * c + h_excess(theta, eos, gamma_ad, c)


def sound_speed_sq(theta, eos: int, gamma_ad: float, c: float):
    """c_s^2 (not divided by c^2)."""
    if eos == IDEAL:
        return c * c * gamma_ad * theta / enthalpy(theta, eos, gamma_ad, c)
    if eos == TM:
        s = torch.sqrt(theta * theta + (4.0 / 9.0) * c ** 4)
        num = 3.0 * theta * theta + 5.0 * theta * s
        den = 12.0 * theta * theta + 2.0 * c ** 4 + 12.0 * theta * s
        return c * c * num / den
    raise ValueError(eos)


def gamma_eq(theta, eos: int, gamma_ad: float, c: float):
    """Equivalent adiabatic index (h - c^2)/(h - c^2 - Theta)."""
    he = h_excess(theta, eos, gamma_ad, c)
    return he / (he - theta)
