"""1-D z-column oracle of the WDLB step (test infrastructure only).

For states that do not depend on x and y (a slit pore started from a uniform
plane, a transverse shear wave along z), every field depends on z alone and
the 3-D shell and ball sums of the WDLB step collapse onto groups of offsets
with the same e_z.  With G depending only on e_z, the sum over a group needs
only the group's moments

    m1[k] = sum_{e in S, e_z = k} e/|e|,   m2[k] = sum_{e in S, e_z = k} (e/|e|)(e/|e|)^T,
    nb[k] = #{e in B, e_z = k}.

This module implements the same step as the 3-D oracle (Sec. 5, the
five-step LB algorithm; forces of Sec. 3: mean-field force, viscous force,
eq. campod for A_ij; collision of eq. SMDB with the source of eq. eq:dufty2)
by that different route, in numpy FP64, and shares no code with it.  The
3-D oracle must agree with it to round-off on x,y-homogeneous states, and it
is cheap enough to run the long homogeneous workloads in full.

Readings are the same as the 3-D oracle: D3Q19, kT = 1/3, trapezoidal
forcing with u = (j + F/2)/rho, Carnahan-Starling g at the midpoint density,
F^v and A_ij formed with u1 = j/rho + (g + F^mf)/2, half-way bounce-back
walls at z = -1/2 and nz - 1/2.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

KT = 1.0 / 3.0

# D3Q19: rest, 6 axis, 12 face diagonals (own copy; textbook set)
VEL = np.array([v for v in itertools.product((-1, 0, 1), repeat=3) if sum(abs(c) for c in v) <= 2],
               dtype=np.int64)
WGT = np.array([{0: 1 / 3, 1: 1 / 18, 2: 1 / 36}[int(np.abs(v).sum())] for v in VEL])
OPP = np.array([int(np.where((VEL == -v).all(1))[0][0]) for v in VEL])


def g_cs(eta):
    return (1.0 - 0.5 * eta) / (1.0 - eta) ** 3


def _lattice_points(R):
    r = np.arange(-R, R + 1)
    return np.array(np.meshgrid(r, r, r, indexing="ij")).reshape(3, -1).T


class Column:
    """x,y-homogeneous WDLB state: the populations f[19, nz]."""

    def __init__(self, nz, sigma=4.0, tau=1.0, g=(0.0, 0.0, 0.0), walls=True, nonlocal_=True, smdb=True):
        self.nz, self.sigma, self.tau = int(nz), float(sigma), float(tau)
        self.g = np.asarray(g, dtype=np.float64)
        self.walls, self.nonlocal_, self.smdb = bool(walls), bool(nonlocal_), bool(smdb)
        s = self.sigma
        pts = _lattice_points(int(math.ceil(s + 0.5)) + 1)
        r2 = (pts ** 2).sum(1).astype(np.float64)
        sh = pts[(r2 >= (s - 0.5) ** 2) & (r2 < (s + 0.5) ** 2)]
        bl = pts[4.0 * r2 <= s * s]
        self.R = int(np.abs(sh).max())
        self.nshell, self.nball = len(sh), len(bl)
        ks = np.arange(-self.R, self.R + 1)
        self.ks = ks
        unit = sh / np.sqrt((sh ** 2).sum(1))[:, None]
        # group moments averaged over the four (+-x, +-y) mirror images of each
        # offset, so the parts that are odd in x or y cancel exactly
        mir = [np.array([sx, sy, 1.0]) for sx in (1.0, -1.0) for sy in (1.0, -1.0)]
        self.m1 = np.array([sum((unit[sh[:, 2] == k] * m).sum(0) for m in mir) / 4.0 for k in ks])
        self.m2 = np.array([sum(np.einsum("ni,nj->ij", unit[sh[:, 2] == k] * m, unit[sh[:, 2] == k] * m)
                                for m in mir) / 4.0 for k in ks])
        self.nb = {int(k): int((bl[:, 2] == k).sum()) for k in np.unique(bl[:, 2])}
        self.f = np.zeros((19, self.nz))

    # -- geometry ---------------------------------------------------------
    def _shift(self, a, k):
        """a(z + k) along the last axis, zero outside the slit (walls) or periodic."""
        if not self.walls:
            return np.roll(a, -k, axis=-1)
        out = np.zeros_like(a)
        n = self.nz
        if k >= 0:
            if k < n:
                out[..., : n - k] = a[..., k:]
        else:
            if -k < n:
                out[..., -k:] = a[..., : n + k]
        return out

    def _inside(self, k):
        """1 where z + k is a fluid node."""
        return self._shift(np.ones(self.nz), k)

    # -- step 1 -------------------------------------------------------------
    def init(self, n, u):
        n = np.broadcast_to(np.asarray(n, dtype=np.float64), (self.nz,)).copy()
        u = np.broadcast_to(np.asarray(u, dtype=np.float64).reshape(3, -1), (3, self.nz)).copy()
        self.f = self.feq(n, u)

    @staticmethod
    def feq(rho, u):
        cu = VEL.astype(np.float64) @ u                   # [19, nz]
        uu = (u * u).sum(0)
        return WGT[:, None] * rho[None, :] * (1 + 3 * cu + 4.5 * cu * cu - 1.5 * uu[None, :])

    # -- steps 2-4 (fields) ------------------------------------------------------
    def _groups(self, rho):
        """Per e_z group k: (index, k, G_k(z), inside mask) with G = wS g_CS(eta_mid) rho(z+k)."""
        nbar = sum(cnt * self._shift(rho, k) for k, cnt in self.nb.items()) / self.nball
        wS = 4.0 * math.pi / self.nshell
        out = []
        for idx, k in enumerate(self.ks):
            k = int(k)
            if k % 2 == 0:
                nmid = self._shift(nbar, k // 2)
            else:
                nmid = 0.5 * (self._shift(nbar, (k - 1) // 2) + self._shift(nbar, (k + 1) // 2))
            eta = math.pi * self.sigma ** 3 * nmid / 6.0
            inside = self._inside(k) > 0
            if np.any(eta[inside] >= 1.0):
                raise FloatingPointError("midpoint packing fraction reached 1")
            gam = np.where(inside, g_cs(np.where(inside, eta, 0.0)), 0.0)
            out.append((idx, k, wS * gam * self._shift(rho, k), inside))
        return out

    def fields(self, with_u1=False):
        """rho, u, F, A0 (A0 as [3, 3, nz]) of the current populations."""
        f = self.f
        rho = f.sum(0)
        if not np.all(rho > 0):
            raise FloatingPointError("non-positive density")
        j = VEL.T.astype(np.float64) @ f                   # [3, nz]
        nz = self.nz
        s2 = self.sigma ** 2
        Fmf = np.zeros((3, nz))
        Fv = np.zeros((3, nz))
        A = np.zeros((3, 3, nz))
        groups = self._groups(rho) if self.nonlocal_ else []
        for idx, k, G, inside in groups:
            Fmf += -KT * s2 * self.m1[idx][:, None] * G[None, :]
        # velocity with which the viscous force and A are formed
        u1 = j / rho[None, :] + 0.5 * (self.g[:, None] + Fmf)
        cv = 2.0 * s2 * math.sqrt(KT / math.pi)
        for idx, k, G, inside in groups:
            du = np.where(inside[None, :], self._shift(u1, k) - u1, 0.0)
            Fv += cv * np.einsum("ij,jz->iz", self.m2[idx], du) * G[None, :]
            t = self.m1[idx][None, :, None] * du[:, None, :]          # m1_j du_i
            A += -(KT / 5.0) * s2 * rho[None, None, :] * G[None, None, :] * (t + t.transpose(1, 0, 2))
        F = rho[None, :] * (self.g[:, None] + Fmf + Fv)
        u = (j + 0.5 * F) / rho[None, :]
        A0 = np.zeros((3, 3, nz))
        if self.nonlocal_ and self.smdb:
            Asym = 0.5 * (A + A.transpose(1, 0, 2))
            tr = np.trace(Asym, axis1=0, axis2=1)
            A0 = Asym - np.eye(3)[:, :, None] * tr[None, None, :] / 3.0
        if not np.all(np.isfinite(u)):
            raise FloatingPointError("non-finite velocity")
        return (rho, u, F, A0, u1) if with_u1 else (rho, u, F, A0)

    # -- one full step -------------------------------------------------------------
    def step(self, nsteps=1):
        c = VEL.astype(np.float64)
        k = 1.0 - 0.5 / self.tau
        for _ in range(int(nsteps)):
            rho, u, F, A0 = self.fields()
            feq = self.feq(rho, u)
            cu = c @ u
            guo = WGT[:, None] * (3.0 * (c @ F - (u * F).sum(0)[None, :]) + 9.0 * cu * (c @ F))
            Q = np.einsum("ai,aj->aij", c, c) - np.eye(3)[None] / 3.0
            src = 4.5 * WGT[:, None] * np.einsum("aij,ijz->az", Q, A0)
            fs = self.f - (self.f - feq) / self.tau + k * (guo + src)
            new = np.empty_like(fs)
            for a in range(19):
                cz = int(VEL[a, 2])
                if not self.walls:
                    new[a] = np.roll(fs[a], cz)
                else:
                    new[a] = fs[OPP[a]]                    # bounce-back default
                    if cz == 0:
                        new[a] = fs[a]
                    elif cz > 0:
                        new[a, 1:] = fs[a, :-1]
                    else:
                        new[a, :-1] = fs[a, 1:]
            self.f = new

    def reduce(self):
        rho, u, _, _ = self.fields()
        return rho, u[0], float((rho * u[0]).mean()), float(u[0].mean()), float(rho.sum())
