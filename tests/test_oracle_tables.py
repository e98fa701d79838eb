"""Pins of the oracle's stencils (ball and contact shell) and constants.

The ball is the lattice stand-in for the Fischer-Methfessel smoothing sphere
of diameter sigma (Sec. 3); the shell is the stand-in for the integral over
the unit vector k at contact distance sigma (Sec. 3, the fields C, A and the
forces F^mf, F^v).  The counts below were obtained by brute-force enumeration
and are checked against both the oracle and an independent count here.
"""
import itertools
import math

import numpy as np
import pytest

from oracle import ref

BALL = {4: 33, 6: 123, 8: 257, 10: 515}
SHELL = {4: 210, 6: 450, 8: 762, 10: 1250}


def _brute(sigma, pred):
    R = int(sigma) + 2
    return sorted(p for p in itertools.product(range(-R, R + 1), repeat=3) if pred(sum(c * c for c in p)))


@pytest.mark.parametrize("sigma", [4, 6, 8, 10])
def test_counts(sigma):
    b, s = ref.ball(sigma), ref.shell(sigma)
    assert len(b) == BALL[sigma]
    assert len(s) == SHELL[sigma]
    # independent enumeration by squared radius
    assert sorted(map(tuple, b.tolist())) == _brute(sigma, lambda r2: 4 * r2 <= sigma * sigma)
    assert sorted(map(tuple, s.tolist())) == _brute(sigma, lambda r2: sigma * sigma - sigma + 1 <= r2 <= sigma * sigma + sigma)


def _cubic_group():
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product((-1, 1), repeat=3):
            M = np.zeros((3, 3), dtype=int)
            for i, p in enumerate(perm):
                M[i, p] = signs[i]
            yield M


@pytest.mark.parametrize("sigma", [3, 4, 6, 8, 10, 5.5])
def test_cubic_symmetry_and_moments(sigma):
    s = ref.shell(sigma).astype(np.int64)
    S = set(map(tuple, s.tolist()))
    group = list(_cubic_group())
    assert len(group) == 48
    for M in group:
        assert set(map(tuple, (s @ M.T).tolist())) == S
    k = s / np.linalg.norm(s, axis=1)[:, None]
    assert np.abs(k.sum(0)).max() < 1e-12
    m2 = k.T @ k
    assert np.allclose(m2, np.eye(3) * len(s) / 3.0, atol=1e-11)
    # mean radius close to sigma (the discrete shell's radius error)
    rbar = np.linalg.norm(s, axis=1).mean() / sigma
    assert abs(rbar - 1.0) < 0.05


def test_contact_value():
    # Carnahan-Starling g(eta) = (1 - eta/2)/(1 - eta)^3; ideal gas limit and a
    # value checked by hand: g(0.5) = 0.75 / 0.125 = 6.
    assert ref.gcs(0.0) == 1.0
    assert abs(ref.gcs(0.5) - 6.0) < 1e-14
    # compressibility factor Z = 1 + 4 eta g: equals the CS equation of state
    for eta in (0.1, 0.2, 0.35, 0.4):
        Z = 1 + 4 * eta * ref.gcs(eta)
        Zcs = (1 + eta + eta ** 2 - eta ** 3) / (1 - eta) ** 3
        assert abs(Z - Zcs) < 1e-13 * Zcs


def test_equilibrium_moments():
    rng = np.random.default_rng(1)
    for _ in range(5):
        rho = rng.uniform(0.5, 2.0)
        u = rng.uniform(-0.1, 0.1, 3)
        f = ref.equilibrium(rho, u)
        c = ref.CV.astype(float)
        assert abs(f.sum() - rho) < 1e-14
        assert np.allclose(c.T @ f, rho * u, atol=1e-15)
        P = np.einsum("a,ai,aj->ij", f, c, c)
        assert np.allclose(P, rho / 3.0 * np.eye(3) + rho * np.outer(u, u), atol=1e-15)


def test_collision_source_moments():
    """Hermite pins of the collision sources (SMDB A-term, Guo forcing)."""
    rng = np.random.default_rng(2)
    c = ref.CV.astype(float)
    for tau in (0.7, 1.0, 1.6):
        k = 1.0 - 0.5 / tau
        rho, u = 1.3, rng.uniform(-0.05, 0.05, 3)
        feq = ref.equilibrium(rho, u)
        # A-source alone: zero mass and momentum, second moment k*A0
        B = rng.normal(size=(3, 3))
        A0 = 0.5 * (B + B.T)
        A0 -= np.eye(3) * np.trace(A0) / 3.0
        d = ref.collide_node(feq, rho, u, np.zeros(3), A0, tau) - feq
        assert abs(d.sum()) < 1e-15
        assert np.abs(c.T @ d).max() < 1e-15
        assert np.allclose(np.einsum("a,ai,aj->ij", d, c, c), k * A0, atol=1e-14)
        # Guo forcing alone: zero mass, momentum k*F, second moment k(uF + Fu)
        F = rng.uniform(-1e-3, 1e-3, 3)
        d = ref.collide_node(feq, rho, u, F, np.zeros(9), tau) - feq
        assert abs(d.sum()) < 1e-16
        assert np.allclose(c.T @ d, k * F, atol=1e-17)
        assert np.allclose(np.einsum("a,ai,aj->ij", d, c, c), k * (np.outer(u, F) + np.outer(F, u)), atol=1e-16)
        # BGK relaxation of a non-equilibrium part
        fneq = rng.normal(scale=1e-3, size=19)
        d = ref.collide_node(feq + fneq, rho, u, np.zeros(3), np.zeros(9), tau) - feq
        assert np.allclose(d, fneq * (1 - 1.0 / tau), atol=1e-15)
