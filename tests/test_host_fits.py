"""Host-side fits of the transport measurements on synthetic signals with
known rates (CPU): the shear-wave decay fit, the damped-cosine fit of the
sound wave, and the Carnahan-Starling sound speed against a numerical
derivative of the equation of state."""
import math

import numpy as np
import pytest

from paper_1304_7880_amd import transport


def test_decay_fit_recovers_rate():
    k = 2 * math.pi / 64
    t = np.arange(0, 2000, 10, dtype=np.float64)
    nu = 0.37
    amps = 1e-4 * np.exp(-nu * k * k * t)
    assert abs(transport.decay_fit(t, amps, k, 200) - nu) < 1e-12 * nu


@pytest.mark.parametrize("omega,gamma,phase,dt", [(0.05, 1e-3, 0.0, 2.0), (0.3, 0.02, 1.1, 1.0),
                                                  (0.01, 0.0, -0.4, 5.0)])
def test_damped_cosine_fit_recovers_frequency_and_rate(omega, gamma, phase, dt):
    t = np.arange(100, 3000, dt, dtype=np.float64)
    amps = 3e-3 * np.exp(-gamma * t) * np.cos(omega * t + phase)
    om, ga = transport.fit_damped_cosine(t, amps)
    assert abs(om - omega) < 1e-9 * omega
    assert abs(ga - gamma) < 1e-9 * max(gamma, omega)


def test_damped_cosine_fit_refuses_non_oscillating_samples():
    t = np.arange(0, 100, 1.0)
    with pytest.raises(ValueError):
        transport.fit_damped_cosine(t, np.exp(-0.05 * t))              # overdamped
    with pytest.raises(ValueError):
        transport.fit_damped_cosine(t[:3], np.cos(0.1 * t[:3]))         # too short
    with pytest.raises(ValueError):
        transport.fit_damped_cosine(np.r_[t[:5], 7.5], np.ones(6))       # unequal spacing


@pytest.mark.parametrize("eta", [0.05, 0.2, 0.35, 0.45])
def test_carnahan_starling_sound_speed(eta):
    kT = 1.0 / 3.0

    def p_over_eta(e):  # P / kT in units of 6/(pi sigma^3): eta Z_CS(eta)
        return e * (1 + e + e * e - e ** 3) / (1 - e) ** 3

    h = 1e-5
    d = (p_over_eta(eta + h) - p_over_eta(eta - h)) / (2 * h)
    assert abs(transport.carnahan_starling_c2(eta, kT) - kT * d) < 1e-8 * kT * d
    assert transport.carnahan_starling_c2(0.0, kT) == kT
