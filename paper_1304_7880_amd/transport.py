"""Transport coefficients measured with the WDLB step: the paper's two
experiments (Sec. 5: the bulk viscosity against packing fraction from the
decay of a transverse shear wave, and the effective viscosity of a slit pore
against its width from Poiseuille flow), the longitudinal wave of the
small-gradient theory (Sec. 4: sound speed from the Carnahan-Starling
equation of state, sound attenuation from the shear and bulk viscosities),
the collisional parts of the thermal conductivity of Sec. 4 from the
thermal fields at a long temperature wave, and the whole conductivity from
the decay of that wave under the energy balance at rest.

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


@dataclass
class ThermalConductivity:
    eta: float
    sigma: float
    T0: float
    n0: float
    lam_coll: float          # collisional conductivity: Q = lam_coll d2T/dz2 at q -> 0
    lam_coll_sec4: float     # (2/3) sqrt(pi T) g n^2 sigma^4 (Sec. 4, eq. thermalcond)
    b_coef: float            # heat-flux correction field: B_z = -b_coef dT/dz at q -> 0
    b_coef_sec4: float       # (8 pi/3) T n^2 g sigma^3, the angular integral of eq. campos
    shell_r1: float          # <|e|>/sigma of the lattice shell
    shell_r2: float          # <|e|^2>/sigma^2 of the lattice shell
    qs: tuple                # the two wave numbers
    lam_coll_q: tuple        # lam_coll at each
    b_coef_q: tuple          # b_coef at each

    def lam_total(self, omega0, cross=2.0):
        """kinetic (5/2) n T / omega0 (eq. qexplicit) + cross b_coef/(cross omega0)
        + collisional; cross = 2 follows eq. qexplicit (delta q = B/(2 omega0)),
        cross = 4 eq. c1exp22 (the two differ by a factor 2)."""
        return 2.5 * self.n0 * self.T0 / omega0 + self.b_coef / (cross * omega0) + self.lam_coll


def lattice_shell(sigma):
    """Offsets e of the lattice contact shell, sigma - 1/2 <= |e| < sigma + 1/2."""
    R = int(math.ceil(sigma + 0.5)) + 1
    r = np.arange(-R, R + 1)
    e = np.stack(np.meshgrid(r, r, r, indexing="ij"), -1).reshape(-1, 3).astype(np.float64)
    d2 = (e * e).sum(1)
    return e[(d2 >= (sigma - 0.5) ** 2) & (d2 < (sigma + 0.5) ** 2)]


def long_wave_limit(qs, values):
    """value(q) = v0 + c q^2 + O(q^4): the extrapolation to q = 0 from two wave numbers."""
    (q1, q2), (v1, v2) = qs, values
    return (q1 * q1 * v2 - q2 * q2 * v1) / (q1 * q1 - q2 * q2)


def thermal_conductivity(eta, sigma=8.0, lengths=(128, 256), eps=1e-4, T0=1.0 / 3.0, nxy=4,
                         precision="fp64") -> ThermalConductivity:
    """A temperature wave T = T0 (1 + eps sin(q z)) in a periodic nxy x nxy x L
    box at rest and uniform density n0(eta), for each L of lengths (q = 2 pi/L):
    the thermal fields of the library (wdlb_thermal_fields); the sin(qz)
    harmonic of Q gives lam_coll(q) = -Q_q / (T0 eps q^2), the cos(qz) harmonic
    of B_z gives b_coef(q) = -B_q / (T0 eps q); both extrapolated to q = 0."""
    n0 = packing_to_density(eta, sigma)
    qs, lam, bco = [], [], []
    for L in lengths:
        ctx = wdlb.Context(nxy, nxy, L, False, precision, sigma, eta, 1.0, (0.0, 0.0, 0.0))
        z = np.arange(L, dtype=np.float64)
        q = 2.0 * math.pi / L
        m = nxy * nxy
        T = np.repeat(T0 * (1.0 + eps * np.sin(q * z)), m)
        Q, B, _ = ctx.thermal_fields(np.full(L * m, n0), np.zeros(3 * L * m), T)
        ctx.destroy()
        N = L * m
        s, c = np.repeat(np.sin(q * z), m), np.repeat(np.cos(q * z), m)
        Qq = float(Q @ s) / float(s @ s)
        Bq = float(B[2 * N:] @ c) / float(c @ c)
        qs.append(q)
        lam.append(-Qq / (T0 * eps * q * q))
        bco.append(-Bq / (T0 * eps * q))
    g = (1.0 - eta / 2.0) / (1.0 - eta) ** 3
    e = lattice_shell(sigma)
    d = np.sqrt((e * e).sum(1))
    return ThermalConductivity(eta, sigma, T0, n0, long_wave_limit(qs, lam),
                               2.0 / 3.0 * math.sqrt(math.pi * T0) * g * n0 * n0 * sigma ** 4,
                               long_wave_limit(qs, bco), 8.0 * math.pi / 3.0 * T0 * n0 * n0 * g * sigma ** 3,
                               float(d.mean()) / sigma, float((d * d).mean()) / sigma ** 2, tuple(qs), tuple(lam),
                               tuple(bco))


@dataclass
class ConductionDecay:
    eta: float
    qs: tuple                # wave numbers 2 pi / L
    lam_q: tuple             # -(3 n / 2) r / q^2 with r the measured per-step rate of the wave
    lam: float               # extrapolated to q = 0
    lam_sec4: float          # (5/2) n T / omega0 + (8 pi/3) T n^2 g sigma^3 r1 / (2 omega0)
                             # + (2/3) sqrt(pi T) g n^2 sigma^4 r2 (Sec. 4, with the shell's moments)
    decay: tuple             # A(steps) / A(0) of each wave


def thermal_conduction_decay(eta, sigma=8.0, lengths=(128, 256), eps=1e-4, T0=1.0 / 3.0, tau=1.0, dt=0.1,
                             steps=200, nxy=4, precision="fp64") -> ConductionDecay:
    """A temperature wave T0 (1 + eps sin(q z)) in a periodic nxy x nxy x L box
    at rest and uniform density, advanced by the energy balance at rest
    (wdlb_conduction_at_rest, steps forward-Euler steps of dt); the per-step
    rate r of its amplitude gives lambda(q) = -(3 n / 2) r / q^2, extrapolated
    to q = 0 from the lengths."""
    n0 = packing_to_density(eta, sigma)
    omega0 = 1.0 / tau
    qs, lam, dec = [], [], []
    for L in lengths:
        ctx = wdlb.Context(nxy, nxy, L, False, precision, sigma, eta, tau, (0.0, 0.0, 0.0))
        z = np.arange(L, dtype=np.float64)
        q = 2.0 * math.pi / L
        m = nxy * nxy
        s = np.repeat(np.sin(q * z), m)
        T = T0 * (1.0 + eps * s)
        Tk = ctx.conduction_at_rest(np.full(L * m, n0), T, omega0, dt, steps)
        ctx.destroy()
        a0, ak = float((T - T0) @ s), float((Tk - T0) @ s)
        r = ((ak / a0) ** (1.0 / steps) - 1.0) / dt
        qs.append(q)
        lam.append(-1.5 * n0 * r / (q * q))
        dec.append(ak / a0)
    g = (1.0 - eta / 2.0) / (1.0 - eta) ** 3
    d = np.sqrt((lattice_shell(sigma) ** 2).sum(1))
    r1, r2 = float(d.mean()) / sigma, float((d * d).mean()) / sigma ** 2
    sec4 = (2.5 * n0 * T0 / omega0 + 8.0 * math.pi / 3.0 * T0 * n0 * n0 * g * sigma ** 3 * r1 / (2.0 * omega0)
            + 2.0 / 3.0 * math.sqrt(math.pi * T0) * g * n0 * n0 * sigma ** 4 * r2)
    return ConductionDecay(eta, tuple(qs), tuple(lam), long_wave_limit(qs, lam), sec4, tuple(dec))


@dataclass
class HeatMode:
    eta: float
    q: float                 # 2 pi / L
    rate: float              # measured per-step decay rate of the temperature wave at constant pressure
    rate_rest: float         # per-step rate of the same wave in the fluid at rest (conduction at rest)
    gamma: float             # c_ad^2 / c_T^2 of the Carnahan-Starling fluid
    ratio: float             # rate / (rate_rest / gamma): 1 when the heat mode decays at lambda q^2 / (n c_p)
    lam_eff: float           # rate n c_p / q^2, c_p = (3/2) gamma: the conductivity the coupled flow shows


def heat_mode(eta, sigma=8.0, L=128, tau=1.0, eps=1e-3, steps=600, every=5, skip=100, nsub=4, nxy=4,
              precision="fp64") -> HeatMode:
    """The heat mode of the coupled thermal flow (wdlb_step_thermal): a
    temperature wave kT (1 + eps sin(q z)) at constant pressure (dn/n =
    -(Z / d(nZ)/dn) dT/T, at rest) in a periodic nxy x nxy x L box; its
    amplitude's decay rate over [skip, steps] against the rate of the same
    wave at rest and uniform density (wdlb_conduction_at_rest, 100 steps of
    dt = 0.1) divided by gamma = c_ad^2 / c_T^2, the hydrodynamic heat-mode
    rate lambda q^2 / (n c_p)."""
    KT = 1.0 / 3.0
    n0 = packing_to_density(eta, sigma)
    Z = (1 + eta + eta ** 2 - eta ** 3) / (1 - eta) ** 3
    cT2 = carnahan_starling_c2(eta)
    gamma = (cT2 + 2.0 / 3.0 * KT * Z * Z) / cT2
    q = 2.0 * math.pi / L
    z = np.arange(L, dtype=np.float64)
    s = np.sin(q * z)
    m = nxy * nxy
    sr = np.repeat(s, m)
    ctx = wdlb.Context(nxy, nxy, L, False, precision, sigma, eta, tau, (0.0, 0.0, 0.0))
    T = KT * (1.0 + eps * sr)
    dt, k = 0.1, 100
    Tk = ctx.conduction_at_rest(np.full(L * m, n0), T, 1.0 / tau, dt, k)
    rate_rest = -((float((Tk - KT) @ sr) / float((T - KT) @ sr)) ** (1.0 / k) - 1.0) / dt
    ctx.init_thermal(np.repeat(n0 * (1.0 - Z / (cT2 / KT) * eps * s), m), np.zeros(3 * L * m), T)
    ts, amps = [], []
    for t in range(0, steps + 1, every):
        ts.append(t)
        amps.append(float((ctx.read_temperature() - KT) @ sr))
        ctx.step_thermal(every, nsub)
    ctx.destroy()
    ts, amps = np.array(ts, dtype=np.float64), np.array(amps)
    sel = ts >= skip
    rate = -float(np.polyfit(ts[sel], np.log(amps[sel]), 1)[0])
    return HeatMode(eta, q, rate, rate_rest, gamma, rate / (rate_rest / gamma), rate * n0 * 1.5 * gamma / (q * q))
