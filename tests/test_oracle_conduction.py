"""Pins of the energy-balance-at-rest oracle (oracle/conduction.py) against
what the paper and the mathematics fix:

- uniform temperature: no change at all (exactly);
- the discrete energy identity: the face fluxes telescope, so the heat
  content changes only by the collisional source, sum (3/2) n dT/dt = sum Q,
  periodic and between adiabatic walls (1e-13);
- a temperature wave T0 (1 + eps sin qz) at uniform density: the
  sin(qz)-harmonic of dT/dt is (2/(3n)) [-lambda_k T0 eps (2 - 2 cos q)
  + B_q sin(q) / (2 omega0) + Q_q] with lambda_k = (5/2) n T0 / omega0 and the
  harmonics B_q, Q_q of the thermal fields (themselves pinned in
  test_oracle_thermal.py) -- the discrete Laplacian, the face-averaged
  correction flux and the source, exactly to rounding;
- its long-wave limit is Sec. 4's conduction, dT/dt = (2/(3n)) lambda
  d2T/dz2 with lambda = (5/2) n T / omega0 + b/(2 omega0) + lambda_coll (eq.
  thermalcond's kinetic and collisional terms; the cross term from eq.
  qexplicit's delta q = B/(2 omega0), twice eq. c1exp22's), b and lambda_coll
  the Sec. 4 values times the lattice shell's radius moments (2e-4, by
  extrapolation in q^2 from two waves);
- adiabatic walls: no heat crosses them (the rate next to the lower wall
  does not see the top plane, beyond the shell's reach);
- mirror symmetry: the rate of a mirrored state is the mirrored rate (in z
  between walls, in x in a periodic box), which fixes the face conductivity
  as symmetric in the two nodes and each component of B to its own axis;
- forward Euler: one step of length dt is T + dt dT/dt.
"""
import math

import numpy as np
import pytest

from oracle import conduction, ref
from paper_1304_7880_amd.workloads import packing_to_density, random_fields, random_temperature


def g_cs(eta):
    return (1 - eta / 2) / (1 - eta) ** 3


def test_uniform_temperature_does_not_change():
    cfg = ref.Config(7, 6, 9, True, 3.0, 1.0)
    n, _ = random_fields(7, 6, 9, packing_to_density(0.3, 3.0), 0.1, 0.0, seed=2)
    r = conduction.rate(cfg, n, np.full(cfg.N, 0.37), 1.0)
    assert not r.any()


@pytest.mark.parametrize("walls", [True, False])
def test_heat_changes_only_by_the_source(walls):
    nx, ny, nz, sigma = 9, 8, 11, 3.0
    cfg = ref.Config(nx, ny, nz, walls, sigma, 1.0)
    n, _ = random_fields(nx, ny, nz, packing_to_density(0.3, sigma), 0.1, 0.0, seed=4)
    T = random_temperature(nx, ny, nz, 1.0 / 3.0, 0.2, seed=5)
    r = conduction.rate(cfg, n, T, 1.3)
    Q, _, _ = ref.thermal(cfg, n, ref.nbar(cfg, n), np.zeros(3 * cfg.N), T)
    lhs, rhs = float((1.5 * n * r).sum()), float(Q.sum())
    scale = float(np.abs(1.5 * n * r).sum())
    assert abs(lhs - rhs) < 1e-13 * scale
    assert abs(rhs) < 0.1 * scale      # the fluxes carry most of the change; the identity is not trivial


def _wave(sigma, eta, L, omega0, eps=1e-4, T0=1.0 / 3.0, axis=2):
    """A temperature wave along x (axis 0), y (1) or z (2) of a periodic
    box L long on that axis and 4 wide on the others."""
    shape = [4, 4, 4]
    shape[axis] = L
    cfg = ref.Config(shape[0], shape[1], shape[2], False, sigma, 1.0)
    x, y, z = np.meshgrid(np.arange(shape[0]), np.arange(shape[1]), np.arange(shape[2]), indexing="ij")
    coord = (x, y, z)[axis].transpose(2, 1, 0).ravel().astype(np.float64)   # node order x fastest
    q = 2 * math.pi / L
    n0 = packing_to_density(eta, sigma)
    rho = np.full(cfg.N, n0)
    T = T0 * (1 + eps * np.sin(q * coord))
    r = conduction.rate(cfg, rho, T, omega0)
    Q, B, _ = ref.thermal(cfg, rho, ref.nbar(cfg, rho), np.zeros(3 * cfg.N), T)
    s, c = np.sin(q * coord), np.cos(q * coord)
    h = lambda f, b: float(f @ b) / float(b @ b)
    return q, n0, h(r, s), h(Q, s), h(B[axis * cfg.N:(axis + 1) * cfg.N], c)


@pytest.mark.parametrize("sigma,eta,omega0,axis", [(4.0, 0.25, 1.0, 2), (6.0, 0.35, 1.0 / 0.8, 2),
                                                   (4.0, 0.3, 1.0, 0), (4.0, 0.3, 1.0, 1)])
def test_temperature_wave_harmonic_closed_form(sigma, eta, omega0, axis):
    eps, T0 = 1e-4, 1.0 / 3.0
    q, n0, r_q, Q_q, B_q = _wave(sigma, eta, 64, omega0, eps, T0, axis)
    lam_k = 2.5 * n0 * T0 / omega0
    pred = 2.0 / (3.0 * n0) * (-lam_k * T0 * eps * (2 - 2 * math.cos(q)) + B_q * math.sin(q) / (2 * omega0) + Q_q)
    assert abs(r_q - pred) < 1e-10 * abs(pred)


def test_long_wave_limit_is_the_sec4_conductivity():
    sigma, eta, omega0, eps, T0 = 8.0, 0.25, 1.0, 1e-4, 1.0 / 3.0
    e = ref.shell(sigma).astype(np.float64)
    d = np.linalg.norm(e, axis=1)
    r1, r2 = d.mean() / sigma, (d * d).mean() / sigma ** 2
    lam = []
    qs = []
    for L in (128, 256):
        q, n0, r_q, _, _ = _wave(sigma, eta, L, omega0, eps, T0)
        qs.append(q)
        lam.append(-r_q * 1.5 * n0 / (T0 * eps * q * q))     # dT/dt = (2/(3n)) lambda d2T/dz2
    (q1, q2), (l1, l2) = qs, lam
    lam0 = (q1 * q1 * l2 - q2 * q2 * l1) / (q1 * q1 - q2 * q2)
    g = g_cs(eta)
    kin = 2.5 * n0 * T0 / omega0
    cross = 8 * math.pi / 3 * T0 * n0 ** 2 * g * sigma ** 3 * r1 / (2 * omega0)
    coll = 2.0 / 3.0 * math.sqrt(math.pi * T0) * g * n0 ** 2 * sigma ** 4 * r2
    assert abs(lam0 / (kin + cross + coll) - 1) < 2e-4, (lam0, kin, cross, coll)


def test_forward_euler_step():
    nx, ny, nz, sigma = 6, 5, 8, 3.0
    cfg = ref.Config(nx, ny, nz, True, sigma, 1.0)
    n, _ = random_fields(nx, ny, nz, packing_to_density(0.3, sigma), 0.1, 0.0, seed=6)
    T = random_temperature(nx, ny, nz, 1.0 / 3.0, 0.1, seed=7)
    T1 = conduction.steps(cfg, n, T, 1.0, 0.05, 1)
    assert np.array_equal(T1, T + 0.05 * conduction.rate(cfg, n, T, 1.0))


def test_adiabatic_walls_pass_no_heat():
    nx, ny, nz, sigma = 6, 5, 14, 3.0          # shell reach 3: plane 0 sees planes 0 .. 4 at most
    cfg = ref.Config(nx, ny, nz, True, sigma, 1.0)
    n, _ = random_fields(nx, ny, nz, packing_to_density(0.3, sigma), 0.1, 0.0, seed=8)
    T = random_temperature(nx, ny, nz, 1.0 / 3.0, 0.1, seed=9)
    r0 = conduction.rate(cfg, n, T, 1.0)
    T2 = T.copy()
    T2[(nz - 1) * nx * ny:] *= 1.3
    r2 = conduction.rate(cfg, n, T2, 1.0)
    m = nx * ny
    assert np.array_equal(r0[:4 * m], r2[:4 * m])
    assert not np.array_equal(r0[(nz - 1) * m:], r2[(nz - 1) * m:])


@pytest.mark.parametrize("walls", [True, False])
def test_mirror_symmetry(walls):
    nx, ny, nz, sigma = 7, 6, 10, 3.0
    cfg = ref.Config(nx, ny, nz, walls, sigma, 1.0)
    n, _ = random_fields(nx, ny, nz, packing_to_density(0.3, sigma), 0.1, 0.0, seed=10)
    T = random_temperature(nx, ny, nz, 1.0 / 3.0, 0.2, seed=11)
    r = conduction.rate(cfg, n, T, 1.0).reshape(nz, ny, nx)
    # mirror in z between the walls; in x (periodic: x -> -x mod nx) in the periodic box
    if walls:
        flip = lambda a: a.reshape(nz, ny, nx)[::-1].ravel()
        rm = conduction.rate(cfg, flip(n), flip(T), 1.0).reshape(nz, ny, nx)[::-1]
    else:
        flip = lambda a: np.roll(a.reshape(nz, ny, nx)[:, :, ::-1], 1, axis=2).ravel()
        rm = np.roll(conduction.rate(cfg, flip(n), flip(T), 1.0).reshape(nz, ny, nx)[:, :, ::-1], 1, axis=2)
    assert np.abs(rm - r).max() < 1e-13 * np.abs(r).max()
