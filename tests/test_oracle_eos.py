"""Pins of the oracle's equations of state (Sec. 2.2)."""
import numpy as np
import pytest
import torch

from oracle import eos
from oracle.setup import IDEAL, TM


def _h_of(rho, P, kind, G, c):
    return eos.enthalpy(P / rho, kind, G, c)


@pytest.mark.parametrize("kind", [IDEAL, TM])
def test_general_sound_speed_definition(kind):
    """c_s^2 = -rho/(n h) dh/drho with n = rho dh/dP - 1 (Sec. 2.2, c = 1)."""
    G, c = 4.0 / 3.0, 1.0
    rng = np.random.default_rng(1)
    for _ in range(20):
        rho = torch.tensor(10 ** rng.uniform(-2, 2), requires_grad=True)
        P = torch.tensor(10 ** rng.uniform(-2, 2), requires_grad=True)
        h = _h_of(rho, P, kind, G, c)
        dh_drho, dh_dP = torch.autograd.grad(h, (rho, P))
        n = rho * dh_dP - 1.0
        cs2_def = -rho / (n * h) * dh_drho
        cs2 = eos.sound_speed_sq(P / rho, kind, G, c)
        assert abs(float((cs2_def - cs2).detach())) < 1e-13 * float(cs2.detach()) + 1e-16


def test_tm_is_the_mathews_relation():
    """The Taub-Matthews enthalpy solves (h - 4 Theta)(h - Theta) = c^4."""
    for c in (1.0, 3.0e8):
        th = torch.logspace(-6, 2, 50) * c * c  # (h - 4 Theta) cancels when hot
        h = eos.enthalpy(th, TM, 0.0, c)
        assert torch.allclose((h - 4 * th) * (h - th) / c ** 4, torch.ones_like(th), rtol=1e-9)


def test_tm_limits():
    c = 1.0
    cold, hot = torch.tensor(1e-7), torch.tensor(1e7)
    assert abs(float(eos.gamma_eq(cold, TM, 0, c)) - 5 / 3) < 1e-6
    assert abs(float(eos.gamma_eq(hot, TM, 0, c)) - 4 / 3) < 1e-6
    assert abs(float(eos.sound_speed_sq(hot, TM, 0, c)) - 1 / 3) < 1e-6
    # cold TM sound speed -> Gamma Theta with Gamma = 5/3
    assert abs(float(eos.sound_speed_sq(cold, TM, 0, c)) / 1e-7 - 5 / 3) < 1e-5


def test_ideal_closed_forms():
    c, G = 2.0, 5.0 / 3.0
    th = torch.tensor([0.1, 1.0, 10.0])
    h = eos.enthalpy(th, IDEAL, G, c)
    assert torch.allclose(h, c * c + G / (G - 1) * th, rtol=1e-15)
    assert torch.allclose(eos.sound_speed_sq(th, IDEAL, G, c), c * c * G * th / h, rtol=1e-15)
    assert torch.allclose(eos.gamma_eq(th, IDEAL, G, c), torch.full_like(th, G), rtol=1e-14)


def test_h_excess_matches_direct_difference():
    c = 1.0
    th = torch.logspace(-3, 3, 30)
    for kind in (IDEAL, TM):
        direct = eos.enthalpy(th, kind, 4 / 3, c) - c * c
        assert torch.allclose(eos.h_excess(th, kind, 4 / 3, c), direct, rtol=1e-12)
