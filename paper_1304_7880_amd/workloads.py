"""Seeded synthetic workloads of the WDLB step.

This module only prepares inputs (geometry, parameters and initial fields);
it holds none of the method's arithmetic and imports nothing from the GPU
library or the oracle, so both sides can be fed the same arrays.

The five workloads are the slit-pore and bulk set-ups on which the method is
exercised (Sec. 5 of the paper: a bulk shear wave at sigma = 8 for the
viscosity against packing fraction, and Poiseuille flow between two parallel
smooth walls), at the sizes used by the tests and the benchmark.  The
paper's own data are not available, so every input is generated here from a
seed.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np


def packing_to_density(eta: float, sigma: float) -> float:
    """Number density of a hard-sphere fluid of packing fraction eta."""
    return 6.0 * eta / (math.pi * sigma ** 3)


@dataclass(frozen=True)
class Workload:
    name: str
    nx: int
    ny: int
    nz: int
    walls_z: bool
    sigma: float
    eta: float
    tau: float
    g: tuple = (0.0, 0.0, 0.0)
    steps: int = 1
    noise: float = 0.0           # relative amplitude of the uniform density noise
    shear_amp: float = 0.0       # amplitude of u_x = a sin(2 pi z / nz)
    seed: int = 0
    nonlocal_: bool = True
    smdb: bool = True
    precision: str = "fp32"

    @property
    def N(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def n0(self) -> float:
        return packing_to_density(self.eta, self.sigma)

    def with_(self, **kw) -> "Workload":
        return replace(self, **kw)


# The slit-pore and bulk workloads, largest first where it matters.
SLAB_SMALL = Workload("slab 4x4x16, sigma=4, eta=0.2, tau=1.0, g_x=1e-6", 4, 4, 16, True, 4.0, 0.2, 1.0,
                      (1e-6, 0.0, 0.0), steps=2000, precision="fp64")
SLAB_64 = Workload("slab 64x64x64 (H=64), sigma=6, eta=0.35, tau=0.8, g_x=1e-6, +-1% noise", 64, 64, 64, True,
                   6.0, 0.35, 0.8, (1e-6, 0.0, 0.0), steps=20000, noise=0.01, seed=2013)
BULK_128 = Workload("bulk 128^3 periodic, sigma=8, shear wave u_x=1e-4 sin(2 pi z/128)", 128, 128, 128, False,
                    8.0, 0.25, 1.0, (0.0, 0.0, 0.0), steps=5000, shear_amp=1e-4)
BULK_ETAS = (0.05, 0.15, 0.25, 0.35, 0.45)
SLAB_LARGE = Workload("slab 512x512x256 (H=256), sigma=10, eta=0.40, tau=0.7, g_x=5e-7", 512, 512, 256, True,
                      10.0, 0.40, 0.7, (5e-7, 0.0, 0.0), steps=10000, precision="bf16")
SLAB_LARGE_SUB = SLAB_LARGE.with_(name="slab 64x64x256 (H=256), sigma=10, eta=0.40, tau=0.7, g_x=5e-7",
                                  nx=64, ny=64)


def initial_fields(w: Workload):
    """(n[N], u[3N]) float64, x fastest: n = n0 (1 + noise xi), xi ~ U[-1, 1)
    from numpy's PCG64 seeded with w.seed; u_x = shear_amp sin(2 pi z / nz)."""
    N = w.N
    n = np.full(N, w.n0, dtype=np.float64)
    if w.noise:
        rng = np.random.default_rng(w.seed)
        n *= 1.0 + w.noise * rng.uniform(-1.0, 1.0, N)
    u = np.zeros(3 * N, dtype=np.float64)
    if w.shear_amp:
        z = np.arange(w.nz, dtype=np.float64)
        ux = w.shear_amp * np.sin(2.0 * math.pi * z / w.nz)
        u[:N] = np.repeat(ux, w.nx * w.ny)
    return n, u


def random_fields(nx, ny, nz, n0, rel=0.05, uamp=0.01, seed=0):
    """Random smooth-free test fields: n = n0 (1 + rel xi), u = uamp xi' (3N)."""
    rng = np.random.default_rng(seed)
    N = nx * ny * nz
    n = n0 * (1.0 + rel * rng.uniform(-1.0, 1.0, N))
    u = uamp * rng.uniform(-1.0, 1.0, 3 * N)
    return n, u


def random_temperature(nx, ny, nz, T0=1.0 / 3.0, rel=0.1, seed=0):
    """Random temperature field T = T0 (1 + rel xi), xi uniform in [-1, 1] (N)."""
    rng = np.random.default_rng(seed)
    return T0 * (1.0 + rel * rng.uniform(-1.0, 1.0, nx * ny * nz))


# --------------------------------------------------------------------------
# Serving workload: slit-pore solves arriving as a Poisson stream.
# --------------------------------------------------------------------------
@dataclass(frozen=True)
class Request:
    H: int
    eta: float
    gx: float
    tau: float
    arrival_s: float


def serving_requests(n=512, rate_hz=200.0, H_range=(8, 96), eta_range=(0.05, 0.45), g_exp=(-7.0, -5.0),
                     tau=1.0, seed=4):
    """n requests: exponential inter-arrival times (mean 1/rate), H uniform
    integer, eta uniform, g_x log-uniform."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, n)
    t = np.cumsum(gaps) - gaps[0]
    H = rng.integers(H_range[0], H_range[1] + 1, n)
    eta = rng.uniform(eta_range[0], eta_range[1], n)
    gx = 10.0 ** rng.uniform(g_exp[0], g_exp[1], n)
    return [Request(int(H[i]), float(eta[i]), float(gx[i]), float(tau), float(t[i])) for i in range(n)]
