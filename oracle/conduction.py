"""FP64 oracle of the energy balance at rest (test infrastructure only: used
by tests/ and nothing in the product path).

Sec. 2's energy balance (eq. energyequation) for a fluid at rest (u = 0) with
a fixed density n(r), the setting in which Sec. 4 derives the thermal
conductivity (eq. thermalcond); k_B = m = 1:

    (3/2) n dT/dt = - div q + Q,
    q = -(5/2) (n T / omega0) grad T + delta q,    delta q = B / (2 omega0)

with the heat flux of eq. qexplicit (its BGK part and its correction from B),
and B and Q of Sec. 3 (eqs. campos, campob1) at u = 0, taken from ref.thermal.

Discretisation (a reading of this project; the paper gives none for the
thermal case): the divergence is the sum over the six faces between a node
and its neighbours r +- e_i of the flux through each face, the kinetic flux
-lambda_f (T(r + e_i) - T(r)) with lambda_f = (5 / (2 omega0)) times the mean
of n T at the two nodes, and the correction flux the mean of delta q_i at the
two nodes; no flux crosses a wall (adiabatic walls at z = -1/2 and nz - 1/2).
Time: forward Euler, T <- T + dt * dT/dt.
"""
from __future__ import annotations

import numpy as np

from . import ref


def rate(cfg: ref.Config, rho, T, omega0, nb=None):
    """dT/dt (N values) of the energy balance at rest for density rho and
    temperature T (N values each, x fastest)."""
    nx, ny, nz, N = cfg.nx, cfg.ny, cfg.nz, cfg.N
    rho = np.asarray(rho, dtype=np.float64).ravel()
    T = np.asarray(T, dtype=np.float64).ravel()
    if nb is None:
        nb = ref.nbar(cfg, rho)
    Q, B, _ = ref.thermal(cfg, rho, nb, np.zeros(3 * N), T)
    n3, T3 = rho.reshape(nz, ny, nx), T.reshape(nz, ny, nx)
    dq = B.reshape(3, nz, ny, nx) / (2.0 * omega0)     # delta q = B / (2 omega0), eq. qexplicit
    nT = n3 * T3
    div = np.zeros((nz, ny, nx))
    for comp, axis in ((0, 2), (1, 1), (2, 0)):          # x, y, z components along array axes 2, 1, 0
        T_up = np.roll(T3, -1, axis)                      # T(r + e_i), periodic wrap
        nT_up = np.roll(nT, -1, axis)
        lam_f = 5.0 / (2.0 * omega0) * 0.5 * (nT + nT_up)
        flux = -lam_f * (T_up - T3) + 0.5 * (dq[comp] + np.roll(dq[comp], -1, axis))   # through r + e_i / 2
        if axis == 0 and cfg.walls_z:
            flux[nz - 1] = 0.0                            # the face at the upper wall
        div += flux - np.roll(flux, 1, axis)              # with walls, the rolled-in face is the lower wall's
    return (-div.ravel() + Q) / (1.5 * rho)


def steps(cfg: ref.Config, rho, T, omega0, dt, nsteps):
    """T after nsteps forward-Euler steps of length dt at fixed density."""
    rho = np.asarray(rho, dtype=np.float64).ravel()
    nb = ref.nbar(cfg, rho)
    T = np.array(T, dtype=np.float64).ravel()
    for _ in range(nsteps):
        T = T + dt * rate(cfg, rho, T, omega0, nb)
    return T
