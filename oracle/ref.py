"""ctypes front end of the FP64 oracle library (test infrastructure only).

Arrays are numpy float64, structure-of-arrays with x fastest:
populations f[19, nz, ny, nx] flattened as f[a*N + i], vectors u[3*N],
tensors A[9*N] (component 3*row + col major).  See wdlb_ref.c for the
equations each call follows.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwdlb_ref.so")

NQ = 19
# D3Q19 velocity order of the oracle (rest, 6 axis, 12 diagonals).
CV = np.array([[0, 0, 0],
               [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
               [1, 1, 0], [-1, -1, 0], [1, -1, 0], [-1, 1, 0],
               [1, 0, 1], [-1, 0, -1], [1, 0, -1], [-1, 0, 1],
               [0, 1, 1], [0, -1, -1], [0, 1, -1], [0, -1, 1]], dtype=np.int64)


class _Cfg(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("walls_z", C.c_int32),
                ("sigma", C.c_double), ("tau", C.c_double), ("g", C.c_double * 3),
                ("nonlocal", C.c_int32), ("smdb", C.c_int32)]


_lib = None


def lib():
    """Load the oracle library, building it first if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from oracle.build import build
            build()
        L = C.CDLL(LIB_PATH)
        dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
        ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
        cp = C.POINTER(_Cfg)
        L.wdlb_ref_ball.argtypes = [C.c_double, C.c_void_p, C.c_int32]
        L.wdlb_ref_shell.argtypes = [C.c_double, C.c_void_p, C.c_int32]
        L.wdlb_ref_gcs.argtypes = [C.c_double]
        L.wdlb_ref_gcs.restype = C.c_double
        L.wdlb_ref_equilibrium.argtypes = [C.c_double, dp, dp]
        L.wdlb_ref_collide_node.argtypes = [dp, C.c_double, dp, dp, dp, C.c_double, dp]
        L.wdlb_ref_moments.argtypes = [cp, dp, dp, dp]
        L.wdlb_ref_nbar.argtypes = [cp, dp, dp]
        L.wdlb_ref_meanfield.argtypes = [cp, dp, dp, dp]
        L.wdlb_ref_viscous.argtypes = [cp, dp, dp, dp, dp, dp]
        L.wdlb_ref_fields.argtypes = [cp, dp, dp, dp, dp, dp, C.c_void_p]
        L.wdlb_ref_thermal.argtypes = [cp, dp, dp, dp, dp, dp, dp, dp]
        L.wdlb_ref_init.argtypes = [cp, dp, dp, dp]
        L.wdlb_ref_step.argtypes = [cp, dp, C.c_int64]
        L.wdlb_ref_init_thermal.argtypes = [cp, dp, dp, dp, dp]
        L.wdlb_ref_step_thermal.argtypes = [cp, dp, dp, C.c_int64, C.c_int32]
        L.wdlb_ref_reduce.argtypes = [cp, dp, dp, dp, dp, dp]
        L.wdlb_ref_threads.restype = C.c_int
        L.wdlb_ref_set_threads.argtypes = [C.c_int]
        del ip
        _lib = L
    return _lib


class OracleError(RuntimeError):
    pass


def _check(rc: int, what: str):
    if rc != 0:
        name = {1: "EINVAL", 2: "EUNSTABLE", 3: "ENOMEM"}.get(rc, str(rc))
        raise OracleError(f"{what}: {name}")


def ball(sigma: float) -> np.ndarray:
    n = lib().wdlb_ref_ball(sigma, None, 0)
    e = np.zeros(3 * n, dtype=np.int32)
    lib().wdlb_ref_ball(sigma, e.ctypes.data, n)
    return e.reshape(n, 3)


def shell(sigma: float) -> np.ndarray:
    n = lib().wdlb_ref_shell(sigma, None, 0)
    e = np.zeros(3 * n, dtype=np.int32)
    lib().wdlb_ref_shell(sigma, e.ctypes.data, n)
    return e.reshape(n, 3)


def gcs(eta: float) -> float:
    return lib().wdlb_ref_gcs(eta)


def equilibrium(rho: float, u) -> np.ndarray:
    out = np.zeros(NQ)
    lib().wdlb_ref_equilibrium(rho, np.ascontiguousarray(u, dtype=np.float64), out)
    return out


def collide_node(f, rho, u, F, A0, tau) -> np.ndarray:
    out = np.zeros(NQ)
    a = lambda x: np.ascontiguousarray(x, dtype=np.float64).ravel()
    lib().wdlb_ref_collide_node(a(f), rho, a(u), a(F), a(A0), tau, out)
    return out


def set_threads(n: int):
    lib().wdlb_ref_set_threads(int(n))


def threads() -> int:
    return lib().wdlb_ref_threads()


@dataclass
class Config:
    nx: int
    ny: int
    nz: int
    walls_z: bool = True
    sigma: float = 4.0
    tau: float = 1.0
    g: tuple = (0.0, 0.0, 0.0)
    nonlocal_: bool = True
    smdb: bool = True

    @property
    def N(self) -> int:
        return self.nx * self.ny * self.nz

    def c(self) -> _Cfg:
        return _Cfg(self.nx, self.ny, self.nz, int(self.walls_z), float(self.sigma), float(self.tau),
                    (C.c_double * 3)(*[float(v) for v in self.g]), int(self.nonlocal_), int(self.smdb))


@dataclass
class State:
    """Oracle state: the populations f (19*N); nothing else is carried."""
    cfg: Config
    f: np.ndarray = field(default=None)

    @classmethod
    def from_fields(cls, cfg: Config, n: np.ndarray, u: np.ndarray) -> "State":
        N = cfg.N
        f = np.zeros(NQ * N)
        n = np.ascontiguousarray(n, dtype=np.float64).ravel()
        u = np.ascontiguousarray(u, dtype=np.float64).ravel()
        assert n.size == N and u.size == 3 * N
        c = cfg.c()
        _check(lib().wdlb_ref_init(C.byref(c), n, u, f), "init")
        return cls(cfg, f)

    def step(self, nsteps: int = 1):
        c = self.cfg.c()
        _check(lib().wdlb_ref_step(C.byref(c), self.f, int(nsteps)), "step")

    def fields(self, with_u1: bool = False):
        """(rho[N], u[3N], F[3N], A0[9N]) at the current time (+ u1[3N])."""
        N = self.cfg.N
        rho, u, F, A0, u1 = np.zeros(N), np.zeros(3 * N), np.zeros(3 * N), np.zeros(9 * N), np.zeros(3 * N)
        c = self.cfg.c()
        _check(lib().wdlb_ref_fields(C.byref(c), self.f, rho, u, F, A0, u1.ctypes.data), "fields")
        return (rho, u, F, A0, u1) if with_u1 else (rho, u, F, A0)

    def reduce(self):
        """(n_z, ux_z, J_pore, u_pore, mass) at the current time."""
        rho, u, _, _ = self.fields()
        return reduce_fields(self.cfg, rho, u)

    def copy(self) -> "State":
        return State(self.cfg, self.f.copy())


def reduce_fields(cfg: Config, rho, u):
    nz = cfg.nz
    n_z, ux_z, out = np.zeros(nz), np.zeros(nz), np.zeros(3)
    c = cfg.c()
    _check(lib().wdlb_ref_reduce(C.byref(c), np.ascontiguousarray(rho), np.ascontiguousarray(u),
                                 n_z, ux_z, out), "reduce")
    return n_z, ux_z, out[0], out[1], out[2]


def moments(cfg: Config, f):
    N = cfg.N
    rho, j = np.zeros(N), np.zeros(3 * N)
    c = cfg.c()
    _check(lib().wdlb_ref_moments(C.byref(c), np.ascontiguousarray(f), rho, j), "moments")
    return rho, j


def nbar(cfg: Config, rho):
    out = np.zeros(cfg.N)
    c = cfg.c()
    _check(lib().wdlb_ref_nbar(C.byref(c), np.ascontiguousarray(rho, dtype=np.float64), out), "nbar")
    return out


def meanfield(cfg: Config, rho, nb):
    """F^mf (3N, component-major)."""
    out = np.zeros(3 * cfg.N)
    c = cfg.c()
    a = lambda x: np.ascontiguousarray(x, dtype=np.float64).ravel()
    _check(lib().wdlb_ref_meanfield(C.byref(c), a(rho), a(nb), out), "meanfield")
    return out


def viscous(cfg: Config, rho, nb, v):
    """(F^v[3N], A[9N]) formed with the velocity field v (3N)."""
    N = cfg.N
    Fv, A = np.zeros(3 * N), np.zeros(9 * N)
    c = cfg.c()
    a = lambda x: np.ascontiguousarray(x, dtype=np.float64).ravel()
    _check(lib().wdlb_ref_viscous(C.byref(c), a(rho), a(nb), a(v), Fv, A), "viscous")
    return Fv, A


def thermal(cfg: Config, rho, nb, v, T):
    """(Q[N], B[3N], F^T[3N]) of the fields rho, v (3N), T (N) (Sec. 3, eqs.
    campob1, campos, thermalforce; k_B = m = 1)."""
    N = cfg.N
    Q, B, FT = np.zeros(N), np.zeros(3 * N), np.zeros(3 * N)
    c = cfg.c()
    a = lambda x: np.ascontiguousarray(x, dtype=np.float64).ravel()
    _check(lib().wdlb_ref_thermal(C.byref(c), a(rho), a(nb), a(v), a(T), Q, B, FT), "thermal")
    return Q, B, FT


@dataclass
class ThermalState:
    """Oracle state of the coupled thermal flow (a hybrid reading: the
    paper's LB scheme is isothermal): populations f (19 N) and the node
    temperatures T (N)."""
    cfg: Config
    f: np.ndarray = field(default=None)
    T: np.ndarray = field(default=None)

    @classmethod
    def from_fields(cls, cfg: Config, n, u, T) -> "ThermalState":
        N = cfg.N
        f = np.zeros(NQ * N)
        a = lambda x: np.ascontiguousarray(x, dtype=np.float64).ravel()
        c = cfg.c()
        _check(lib().wdlb_ref_init_thermal(C.byref(c), a(n), a(u), a(T), f), "init_thermal")
        return cls(cfg, f, np.array(T, dtype=np.float64).ravel())

    def step(self, nsteps: int = 1, nsub: int = 4):
        c = self.cfg.c()
        _check(lib().wdlb_ref_step_thermal(C.byref(c), self.f, self.T, int(nsteps), int(nsub)), "step_thermal")

    def moments(self):
        return moments(self.cfg, self.f)
