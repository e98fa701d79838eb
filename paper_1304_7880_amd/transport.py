"""Transport coefficients measured with the WDLB step (the paper's two
experiments, Sec. 5: the bulk viscosity against packing fraction from the
decay of a transverse shear wave, and the effective viscosity of a slit pore
against its width from Poiseuille flow).

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
                         smdb=True, precision="fp32", skip=0.2) -> ShearDecay:
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
                             max_steps=200000, smdb=True, precision="fp32") -> SlitFlow:
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
