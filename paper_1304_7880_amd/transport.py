"""Transport coefficients measured with the WDLB step: the paper's two
experiments (Sec. 5: the bulk viscosity against packing fraction from the
decay of a transverse shear wave, and the effective viscosity of a slit pore
against its width from Poiseuille flow), and the longitudinal wave of the
small-gradient theory (Sec. 4: sound speed from the Carnahan-Starling
equation of state, sound attenuation from the shear and bulk viscosities).

Everything here drives the library through its C ABI (wdlb.Context) and
post-processes FP64 plane means read back from the device; no step of the
method runs here.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import wdlb
from .workloads import packing_to_density


@dataclass
class ShearDecay:
    nu: float            # kinematic viscosity from the decay rate, nu = Gamma / k^2
    times: np.ndarray    # steps at which the amplitude was read
    amp: np.ndarray      # A(t) = (2/n) sum_z u_x(z) sin(2 pi z / n)
    seconds: float       # device + host time of the run


def decay_fit(times, amps, k, skip_steps, floor=1e-6):
    """nu from a least-squares fit of ln A(t) = ln A0 - nu k^2 t over the
    reads after skip_steps (the initial non-hydrodynamic transient) whose
    amplitude is still above floor * A(0) (later ones are at rounding level)."""
    sel = (times >= skip_steps) & (amps > floor * amps[0])
    if sel.sum() < 3:
        raise ValueError("too few resolved amplitudes to fit a decay rate")
    return -np.polyfit(times[sel], np.log(amps[sel]), 1)[0] / (k * k)


def shear_wave_viscosity(eta, sigma=8.0, n=128, nxy=None, steps=5000, every=10, tau=1.0, amp=1e-4,
                         smdb=True, precision="fp32_local64", skip=0.2) -> ShearDecay:
    """Periodic box n x n x n (or nxy x nxy x n), u_x = amp sin(2 pi z / n)
    at rest density n0(eta); nu from decay_fit over the steps after the
    first `skip` fraction of the run."""
    import time

    import torch
    nxy = n if nxy is None else nxy
    ctx = wdlb.Context(nxy, nxy, n, False, precision, sigma, eta, tau, (0.0, 0.0, 0.0), True, smdb)
    z = np.arange(n, dtype=np.float64)
    s = np.sin(2.0 * math.pi * z / n)
    N = nxy * nxy * n
    u = np.zeros(3 * N)
    u[:N] = np.repeat(amp * s, nxy * nxy)
    ctx.init_fields(np.full(N, packing_to_density(eta, sigma)), u)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    times, amps = [], []
    t = 0
    while t <= steps:
        _, ux = ctx.read_profiles()
        times.append(t)
        amps.append(2.0 / n * float(ux @ s))
        if t == steps:
            break
        ctx.step(every)
        t += every
    ctx.sync()
    secs = time.perf_counter() - t0
    ctx.destroy()
    times, amps = np.asarray(times, dtype=np.float64), np.asarray(amps)
    return ShearDecay(decay_fit(times, amps, 2.0 * math.pi / n, skip * steps), times, amps, secs)


@dataclass
class SlitFlow:
    nu_eff: float        # g H^2 / (12 u_pore)
    u_pore: float
    j_pore: float
    steps: int
    converged: bool


def slit_effective_viscosity(H, eta, sigma=8.0, g=1e-6, nxy=16, tau=1.0, tol=1e-8, every=100,
                             max_steps=200000, smdb=True, precision="fp32_local64") -> SlitFlow:
    """Poiseuille flow between the walls of a slit of H fluid planes, run
    until the pore flux changes by less than tol (relative) over `every`
    steps; the effective viscosity is the one a parabolic profile of the
    same mean velocity would have, nu_eff = g H^2 / (12 u_pore)."""
    ctx = wdlb.Context(nxy, nxy, H, True, precision, sigma, eta, tau, (g, 0.0, 0.0), True, smdb)
    ctx.init_uniform((0.0, 0.0, 0.0))
    steps, Jprev, J, U, conv = 0, None, 0.0, 0.0, False
    while steps < max_steps:
        ctx.step(every)
        steps += every
        J, U, _ = ctx.read_flux()
        if Jprev is not None and abs(J - Jprev) <= tol * abs(J):
            conv = True
            break
        Jprev = J
    ctx.destroy()
    return SlitFlow(g * H * H / (12.0 * U), U, J, steps, conv)


@dataclass
class SoundWave:
    c2: float            # squared sound speed, (omega^2 + Gamma^2) / q^2
    nu_long: float       # longitudinal kinematic viscosity 2 Gamma / q^2 (= 4/3 nu_shear + nu_bulk)
    omega: float         # angular frequency per step
    gamma: float         # amplitude decay rate per step
    times: np.ndarray    # steps at which the amplitude was read
    amp: np.ndarray      # B(t) = (2/n) sum_z (n(z)/n0 - 1) sin(2 pi z / n)
    seconds: float


def fit_damped_cosine(times, amps):
    """omega and Gamma of B(t) = B0 exp(-Gamma t) cos(omega t + phi) sampled at
    equal steps dt: such samples obey B[k+1] = a1 B[k] + a2 B[k-1] with
    a1 = 2 exp(-Gamma dt) cos(omega dt), a2 = -exp(-2 Gamma dt); a1, a2 by
    least squares (the samples must cover well over one period)."""
    times, amps = np.asarray(times, dtype=np.float64), np.asarray(amps, dtype=np.float64)
    dt = times[1] - times[0]
    if len(amps) < 4 or not np.allclose(np.diff(times), dt):
        raise ValueError("need at least four equally spaced samples")
    X = np.stack([amps[1:-1], amps[:-2]], axis=1)
    a1, a2 = np.linalg.lstsq(X, amps[2:], rcond=None)[0]
    if not a2 < 0:
        raise ValueError("the samples do not decay as a damped oscillation")
    r = math.sqrt(-a2)
    c = a1 / (2.0 * r)
    if not -1.0 < c < 1.0:
        raise ValueError("the samples do not oscillate (overdamped or too coarsely sampled)")
    return math.acos(c) / dt, -math.log(r) / dt


def carnahan_starling_c2(eta, kT=1.0 / 3.0):
    """Isothermal sound speed squared of the Carnahan-Starling fluid, c^2 =
    kT d(n Z)/dn with Z = (1 + eta + eta^2 - eta^3)/(1 - eta)^3 (mass 1)."""
    return kT * (1 + 4 * eta + 4 * eta ** 2 - 4 * eta ** 3 + eta ** 4) / (1 - eta) ** 4


def longitudinal_wave(eta, sigma=8.0, n=128, nxy=None, steps=2000, every=2, tau=1.0, eps=1e-3, smdb=True,
                      precision="fp32_local64", skip=50, floor=1e-3) -> SoundWave:
    """Periodic box n x n x n (or nxy x nxy x n) at rest with the density
    n0(eta) (1 + eps sin(2 pi z / n)): the standing sound wave's frequency and
    decay give c^2 and the longitudinal viscosity (fit_damped_cosine over the
    reads from step `skip` on, past the initial non-hydrodynamic transient, up
    to the last read whose amplitude is still above floor * B(0))."""
    import time

    import torch
    nxy = n if nxy is None else nxy
    n0 = packing_to_density(eta, sigma)
    ctx = wdlb.Context(nxy, nxy, n, False, precision, sigma, eta, tau, (0.0, 0.0, 0.0), True, smdb)
    z = np.arange(n, dtype=np.float64)
    s = np.sin(2.0 * math.pi * z / n)
    ctx.init_fields(np.repeat(n0 * (1.0 + eps * s), nxy * nxy), np.zeros(3 * nxy * nxy * n))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    times, amps = [], []
    t = 0
    while t <= steps:
        nz, _ = ctx.read_profiles()
        times.append(t)
        amps.append(2.0 / n * float((nz / n0 - 1.0) @ s))
        if t == steps:
            break
        ctx.step(every)
        t += every
    ctx.sync()
    secs = time.perf_counter() - t0
    ctx.destroy()
    times, amps = np.asarray(times, dtype=np.float64), np.asarray(amps)
    above = np.nonzero(np.abs(amps) >= floor * abs(amps[0]))[0]
    sel = (times >= skip) & (times <= times[above[-1]])
    omega, gamma = fit_damped_cosine(times[sel], amps[sel])
    q = 2.0 * math.pi / n
    return SoundWave((omega * omega + gamma * gamma) / (q * q), 2.0 * gamma / (q * q), omega, gamma, times, amps,
                     secs)
