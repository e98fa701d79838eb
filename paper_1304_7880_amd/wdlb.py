"""Python binding of libwdlb.so (the C ABI in include/wdlb.h).

Argument marshalling only: every step of the method runs in the HIP
kernels of the library.  PyTorch provides the device workspace and the
stream.  There is no fallback: if the library or a GPU is missing the calls
raise.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwdlb.so")

OK, E_INVAL, E_NOMEM, E_HIP, E_UNSTABLE, E_STATE, E_NOT_CONVERGED = range(7)
STATUS = {0: "OK", 1: "E_INVAL", 2: "E_NOMEM", 3: "E_HIP", 4: "E_UNSTABLE", 5: "E_STATE", 6: "E_NOT_CONVERGED"}
FP64, FP32, BF16_NEQ, FP32_LOCAL64, BF16_NEQ_LOCAL64 = 0, 1, 2, 3, 4
NKERNELS = 6
NTILES = 7
PRECISION = {"fp64": FP64, "fp32": FP32, "bf16": BF16_NEQ, "fp32_local64": FP32_LOCAL64,
             "bf16_local64": BF16_NEQ_LOCAL64}

# D3Q19 order of the library's populations (include/wdlb.h)
CV = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
               [1, 1, 0], [-1, -1, 0], [1, -1, 0], [-1, 1, 0], [1, 0, 1], [-1, 0, -1], [1, 0, -1],
               [-1, 0, 1], [0, 1, 1], [0, -1, -1], [0, 1, -1], [0, -1, 1]], dtype=np.int64)

SYMBOLS = ["wdlb_workspace_size", "wdlb_create", "wdlb_create_static", "wdlb_set_params", "wdlb_init_uniform", "wdlb_init_fields",
           "wdlb_step", "wdlb_sync", "wdlb_read_fields", "wdlb_read_fields_ex", "wdlb_read_profiles",
           "wdlb_read_flux", "wdlb_read_populations", "wdlb_thermal_fields", "wdlb_thermal_fields_device", "wdlb_conduction_at_rest",
           "wdlb_init_thermal", "wdlb_step_thermal", "wdlb_state_size", "wdlb_save_state", "wdlb_load_state",
           "wdlb_get_step", "wdlb_profile", "wdlb_profile_read", "wdlb_kernel_name", "wdlb_set_tile",
           "wdlb_get_tile", "wdlb_set_graphs", "wdlb_last_error", "wdlb_destroy",
           "wdlb_server_workspace_size", "wdlb_server_create", "wdlb_server_submit", "wdlb_server_poll",
           "wdlb_server_drain", "wdlb_server_stats_get", "wdlb_server_last_error", "wdlb_server_destroy"]


class LatticeDesc(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("walls_z", C.c_int32),
                ("precision", C.c_int32), ("stream", C.c_void_p)]


class Params(C.Structure):
    _fields_ = [("sigma", C.c_double), ("eta", C.c_double), ("tau", C.c_double), ("g", C.c_double * 3),
                ("nonlocal_", C.c_int32), ("smdb", C.c_int32)]


class ServerParams(C.Structure):
    _fields_ = [("sigma", C.c_double), ("tol", C.c_double), ("check_every", C.c_int32), ("pad", C.c_int32),
                ("max_steps", C.c_int64)]


class Request(C.Structure):
    _fields_ = [("H", C.c_int32), ("pad", C.c_int32), ("eta", C.c_double), ("gx", C.c_double), ("tau", C.c_double)]


class Result(C.Structure):
    _fields_ = [("state", C.c_int32), ("status", C.c_int32), ("H", C.c_int32), ("pad", C.c_int32),
                ("steps", C.c_int64), ("j_pore", C.c_double), ("u_pore", C.c_double), ("t_submit", C.c_double),
                ("t_admit", C.c_double), ("t_done", C.c_double)]


class ServerStats(C.Structure):
    _fields_ = [("chunks", C.c_int64), ("steps", C.c_int64), ("node_updates", C.c_double),
                ("resident", C.c_int32), ("max_resident", C.c_int32), ("queued", C.c_int32),
                ("finished", C.c_int32), ("busy_s", C.c_double)]


class WdlbError(RuntimeError):
    def __init__(self, status, msg=""):
        self.status = status
        super().__init__(f"{STATUS.get(status, status)}: {msg}")


_lib = None


def load(path: str = LIB_PATH):
    """Load libwdlb.so (after torch, so that both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with __graft_entry__.build() "
                           "or python -m paper_1304_7880_amd.build")
    import torch  # noqa: F401  (binds the library to torch's HIP runtime)
    L = C.CDLL(path)
    vp, dp = C.c_void_p, C.POINTER(C.c_double)
    L.wdlb_workspace_size.argtypes = [C.POINTER(LatticeDesc), C.POINTER(Params), C.POINTER(C.c_size_t)]
    L.wdlb_create.argtypes = [C.POINTER(LatticeDesc), C.POINTER(Params), vp, C.c_size_t, C.POINTER(vp)]
    L.wdlb_create_static.argtypes = [C.POINTER(LatticeDesc), C.POINTER(Params), C.POINTER(vp)]
    L.wdlb_set_params.argtypes = [vp, C.POINTER(Params)]
    L.wdlb_init_uniform.argtypes = [vp, dp]
    L.wdlb_init_fields.argtypes = [vp, dp, dp]
    L.wdlb_step.argtypes = [vp, C.c_int64]
    L.wdlb_sync.argtypes = [vp]
    L.wdlb_read_fields.argtypes = [vp, dp, dp]
    L.wdlb_read_fields_ex.argtypes = [vp, dp, dp, dp, dp]
    L.wdlb_read_profiles.argtypes = [vp, dp, dp]
    L.wdlb_read_flux.argtypes = [vp, dp, dp, dp]
    L.wdlb_read_populations.argtypes = [vp, dp]
    L.wdlb_thermal_fields.argtypes = [vp, dp, dp, dp, dp, dp, dp]
    L.wdlb_thermal_fields_device.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    L.wdlb_conduction_at_rest.argtypes = [vp, dp, dp, C.c_double, C.c_double, C.c_int64]
    L.wdlb_init_thermal.argtypes = [vp, dp, dp, dp, vp]
    L.wdlb_step_thermal.argtypes = [vp, vp, C.c_int64, C.c_int32]
    L.wdlb_state_size.argtypes = [vp, C.POINTER(C.c_size_t)]
    L.wdlb_save_state.argtypes = [vp, vp, C.c_size_t]
    L.wdlb_load_state.argtypes = [vp, vp, C.c_size_t]
    L.wdlb_get_step.argtypes = [vp, C.POINTER(C.c_int64)]
    L.wdlb_profile.argtypes = [vp, C.c_int32]
    L.wdlb_profile_read.argtypes = [vp, C.c_int32, dp, C.POINTER(C.c_int64)]
    L.wdlb_kernel_name.argtypes = [C.c_int32]
    L.wdlb_kernel_name.restype = C.c_char_p
    L.wdlb_set_tile.argtypes = [vp, C.c_int32]
    L.wdlb_get_tile.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    L.wdlb_set_graphs.argtypes = [vp, C.c_int32]
    L.wdlb_last_error.argtypes = [vp]
    L.wdlb_last_error.restype = C.c_char_p
    L.wdlb_destroy.argtypes = [vp]
    L.wdlb_destroy.restype = None
    L.wdlb_server_workspace_size.argtypes = [C.POINTER(LatticeDesc), C.POINTER(ServerParams), C.POINTER(C.c_size_t)]
    L.wdlb_server_create.argtypes = [C.POINTER(LatticeDesc), C.POINTER(ServerParams), vp, C.c_size_t,
                                     C.POINTER(vp)]
    L.wdlb_server_submit.argtypes = [vp, C.POINTER(Request), C.POINTER(C.c_uint64)]
    L.wdlb_server_poll.argtypes = [vp, C.c_uint64, C.POINTER(Result), dp, C.c_int32]
    L.wdlb_server_drain.argtypes = [vp]
    L.wdlb_server_stats_get.argtypes = [vp, C.POINTER(ServerStats)]
    L.wdlb_server_last_error.argtypes = [vp]
    L.wdlb_server_last_error.restype = C.c_char_p
    L.wdlb_server_destroy.argtypes = [vp]
    L.wdlb_server_destroy.restype = None
    _lib = L
    return L


def _ptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(C.c_double))


def make_desc(nx, ny, nz, walls_z=True, precision="fp32", stream=None) -> LatticeDesc:
    return LatticeDesc(int(nx), int(ny), int(nz), int(bool(walls_z)), PRECISION[precision]
                       if isinstance(precision, str) else int(precision), stream)


def make_params(sigma=4.0, eta=0.2, tau=1.0, g=(0.0, 0.0, 0.0), nonlocal_=True, smdb=True) -> Params:
    return Params(float(sigma), float(eta), float(tau), (C.c_double * 3)(*[float(v) for v in g]),
                  int(bool(nonlocal_)), int(bool(smdb)))


def workspace_size(desc: LatticeDesc, params: Params) -> int:
    n = C.c_size_t(0)
    st = load().wdlb_workspace_size(C.byref(desc), C.byref(params), C.byref(n))
    if st != OK:
        raise WdlbError(st, "workspace_size")
    return n.value


class Context:
    """One lattice on the current device; the workspace is a torch uint8 tensor."""

    def __init__(self, nx, ny, nz, walls_z=True, precision="fp32", sigma=4.0, eta=0.2, tau=1.0,
                 g=(0.0, 0.0, 0.0), nonlocal_=True, smdb=True, stream=None, device="cuda", static=False):
        """static=True: wdlb_create_static (the library's own device array as
        the workspace; nothing is allocated), else wdlb_create on a torch
        workspace."""
        import torch
        L = load()
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        self.desc = make_desc(nx, ny, nz, walls_z, precision, C.c_void_p(stream.cuda_stream))
        self.params = make_params(sigma, eta, tau, g, nonlocal_, smdb)
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.N = self.nx * self.ny * self.nz
        self.device = device
        self.T = None          # the temperature of the coupled thermal flow (device, storage real)
        h = C.c_void_p()
        if static:
            self.workspace = None
            st = L.wdlb_create_static(C.byref(self.desc), C.byref(self.params), C.byref(h))
            if st != OK:
                raise WdlbError(st, "wdlb_create_static")
        else:
            nbytes = workspace_size(self.desc, self.params)
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=device)
            st = L.wdlb_create(C.byref(self.desc), C.byref(self.params), C.c_void_p(self.workspace.data_ptr()),
                               nbytes, C.byref(h))
            if st != OK:
                raise WdlbError(st, "wdlb_create")
        self.h = h
        self._L = L

    # -- plumbing -----------------------------------------------------------
    def _chk(self, st, what):
        if st != OK:
            msg = self._L.wdlb_last_error(self.h)
            raise WdlbError(st, f"{what}: {msg.decode() if msg else ''}")

    def destroy(self):
        """Release the context and drop the reference to its workspace (the
        library synchronises the stream first, so the memory is idle)."""
        if getattr(self, "h", None):
            self._L.wdlb_destroy(self.h)
            self.h = None
        self.workspace = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    # -- the C entry points ---------------------------------------------------
    def set_params(self, sigma, eta, tau, g, nonlocal_=True, smdb=True):
        self.params = make_params(sigma, eta, tau, g, nonlocal_, smdb)
        self._chk(self._L.wdlb_set_params(self.h, C.byref(self.params)), "set_params")

    def init_uniform(self, u0=(0.0, 0.0, 0.0)):
        u = np.ascontiguousarray(u0, dtype=np.float64)
        self._chk(self._L.wdlb_init_uniform(self.h, _ptr(u)), "init_uniform")

    def init_fields(self, n, u):
        n = np.ascontiguousarray(n, dtype=np.float64).ravel()
        u = np.ascontiguousarray(u, dtype=np.float64).ravel()
        if n.size != self.N or u.size != 3 * self.N:
            raise ValueError("field sizes do not match the lattice")
        self._chk(self._L.wdlb_init_fields(self.h, _ptr(n), _ptr(u)), "init_fields")

    def step(self, nsteps=1):
        self._chk(self._L.wdlb_step(self.h, int(nsteps)), "step")

    def sync(self):
        self._chk(self._L.wdlb_sync(self.h), "sync")

    def read_fields(self, with_forces=False):
        N = self.N
        n, u = np.zeros(N), np.zeros(3 * N)
        if not with_forces:
            self._chk(self._L.wdlb_read_fields(self.h, _ptr(n), _ptr(u)), "read_fields")
            return n, u
        F, A0 = np.zeros(3 * N), np.zeros(9 * N)
        self._chk(self._L.wdlb_read_fields_ex(self.h, _ptr(n), _ptr(u), _ptr(F), _ptr(A0)), "read_fields_ex")
        return n, u, F, A0

    def read_profiles(self):
        nz_, ux = np.zeros(self.nz), np.zeros(self.nz)
        self._chk(self._L.wdlb_read_profiles(self.h, _ptr(nz_), _ptr(ux)), "read_profiles")
        return nz_, ux

    def read_flux(self):
        j, u, m = C.c_double(), C.c_double(), C.c_double()
        self._chk(self._L.wdlb_read_flux(self.h, C.byref(j), C.byref(u), C.byref(m)), "read_flux")
        return j.value, u.value, m.value

    def thermal_fields(self, n, u, T):
        """(Q[N], B[3N], F^T[3N]) of Sec. 3 (eqs. campob1, campos,
        thermalforce) at the given density n[N], velocity u[3N] and
        temperature T[N]; the state is left as it was."""
        N = self.N
        n = np.ascontiguousarray(n, dtype=np.float64).ravel()
        u = np.ascontiguousarray(u, dtype=np.float64).ravel()
        T = np.ascontiguousarray(T, dtype=np.float64).ravel()
        if n.size != N or u.size != 3 * N or T.size != N:
            raise ValueError("field sizes do not match the lattice")
        Q, B, FT = np.zeros(N), np.zeros(3 * N), np.zeros(3 * N)
        self._chk(self._L.wdlb_thermal_fields(self.h, _ptr(n), _ptr(u), _ptr(T), _ptr(Q), _ptr(B), _ptr(FT)),
                  "thermal_fields")
        return Q, B, FT

    def thermal_fields_device(self, n, u, T, Q, B, FT):
        """wdlb_thermal_fields_device on device tensors (contiguous, on the
        context's device, float64 in the FP64 mode and float32 otherwise):
        n, T, Q of N values; u, B, FT of 3N.  Asynchronous on the stream."""
        import torch
        dt = torch.float64 if self.desc.precision == FP64 else torch.float32
        N = self.N
        for name, t, size in (("n", n, N), ("u", u, 3 * N), ("T", T, N), ("Q", Q, N), ("B", B, 3 * N),
                              ("FT", FT, 3 * N)):
            if not (t.is_cuda and t.dtype == dt and t.is_contiguous() and t.numel() == size):
                raise ValueError(f"{name}: a contiguous {dt} device tensor of {size} values is required")
        self._chk(self._L.wdlb_thermal_fields_device(self.h, n.data_ptr(), u.data_ptr(), T.data_ptr(), Q.data_ptr(),
                                                     B.data_ptr(), FT.data_ptr()), "thermal_fields_device")

    def conduction_at_rest(self, n, T, omega0, dt, nsteps):
        """T after nsteps forward-Euler steps of the energy balance at rest
        (wdlb_conduction_at_rest) at the fixed density n (N values each)."""
        N = self.N
        n = np.ascontiguousarray(n, dtype=np.float64).ravel()
        T = np.array(T, dtype=np.float64).ravel()
        if n.size != N or T.size != N:
            raise ValueError("field sizes do not match the lattice")
        self._chk(self._L.wdlb_conduction_at_rest(self.h, _ptr(n), _ptr(T), float(omega0), float(dt), int(nsteps)),
                  "conduction_at_rest")
        return T

    def init_thermal(self, n, u, T):
        """wdlb_init_thermal: the state at density n[N], velocity u[3N] and
        temperature T[N]; T is held on the device in self.T (float64 in the
        FP64 mode, float32 in the FP32 ones)."""
        import torch
        N = self.N
        n = np.ascontiguousarray(n, dtype=np.float64).ravel()
        u = np.ascontiguousarray(u, dtype=np.float64).ravel()
        T = np.ascontiguousarray(T, dtype=np.float64).ravel()
        if n.size != N or u.size != 3 * N or T.size != N:
            raise ValueError("field sizes do not match the lattice")
        dt = torch.float64 if self.desc.precision == FP64 else torch.float32
        if self.T is None or self.T.dtype != dt:
            self.T = torch.empty(N, dtype=dt, device=self.device)
        self._chk(self._L.wdlb_init_thermal(self.h, _ptr(n), _ptr(u), _ptr(T), self.T.data_ptr()), "init_thermal")

    def step_thermal(self, nsteps=1, nsub=4):
        """wdlb_step_thermal: nsteps coupled steps, the conduction in nsub
        sub-steps each; asynchronous (sync() reports an instability)."""
        if self.T is None:
            raise WdlbError(E_STATE, "step_thermal: init_thermal first")
        self._chk(self._L.wdlb_step_thermal(self.h, self.T.data_ptr(), int(nsteps), int(nsub)), "step_thermal")

    def read_temperature(self):
        """T[N] of the coupled thermal flow (host, float64), after a sync."""
        if self.T is None:
            raise WdlbError(E_STATE, "read_temperature: init_thermal first")
        self.sync()
        return self.T.cpu().numpy().astype(np.float64)

    def read_populations(self):
        f = np.zeros(19 * self.N)
        self._chk(self._L.wdlb_read_populations(self.h, _ptr(f)), "read_populations")
        return f

    def state_size(self):
        n = C.c_size_t()
        self._chk(self._L.wdlb_state_size(self.h, C.byref(n)), "state_size")
        return n.value

    def save_state(self) -> bytes:
        n = self.state_size()
        buf = C.create_string_buffer(n)
        self._chk(self._L.wdlb_save_state(self.h, buf, n), "save_state")
        return buf.raw

    def load_state(self, data: bytes):
        buf = C.create_string_buffer(data, len(data))
        self._chk(self._L.wdlb_load_state(self.h, buf, len(data)), "load_state")

    def profile(self, enable=True, kernels=None):
        """Time the step kernels with HIP events: all of them, or only those
        named in kernels; enable=False stops."""
        mask = 0
        if enable:
            if kernels is None:
                mask = -1
            else:
                names = [self._L.wdlb_kernel_name(k).decode() for k in range(NKERNELS)]
                for n in kernels:
                    mask |= 1 << names.index(n)
        self._chk(self._L.wdlb_profile(self.h, mask), "profile")

    def profile_read(self):
        """{kernel name: (total ms, launches)} of the timed step kernels (synchronises)."""
        out = {}
        for k in range(NKERNELS):
            ms, n = C.c_double(), C.c_int64()
            self._chk(self._L.wdlb_profile_read(self.h, k, C.byref(ms), C.byref(n)), "profile_read")
            out[self._L.wdlb_kernel_name(k).decode()] = (ms.value, n.value)
        return out

    def set_tile(self, variant=-1):
        """Contact-shell tile variant (0 .. NTILES-1), -1 = automatic."""
        self._chk(self._L.wdlb_set_tile(self.h, int(variant)), "set_tile")

    def get_tile(self):
        """(tile variant in use, True when the compiled-shell kernels run)."""
        v, sp = C.c_int32(), C.c_int32()
        self._chk(self._L.wdlb_get_tile(self.h, C.byref(v), C.byref(sp)), "get_tile")
        return v.value, bool(sp.value)

    def set_graphs(self, enable=True):
        """Replay pairs of steps as HIP graphs (default) or launch each kernel."""
        self._chk(self._L.wdlb_set_graphs(self.h, int(bool(enable))), "set_graphs")

    def get_step(self):
        s = C.c_int64()
        self._chk(self._L.wdlb_get_step(self.h, C.byref(s)), "get_step")
        return s.value


class Server:
    """Batched slit-pore solves over resident requests (wdlb_server_*): nx x ny
    slits of any height up to nz - R stacked in one lattice of nz planes; the
    pool is a torch uint8 tensor; a worker thread in the library steps them."""

    def __init__(self, nx, ny, nz, sigma=4.0, tol=1e-8, check_every=100, max_steps=100000, device="cuda",
                 precision="fp32_local64"):
        import torch
        L = load()
        self.desc = make_desc(nx, ny, nz, True, precision, None)
        self.params = ServerParams(float(sigma), float(tol), int(check_every), 0, int(max_steps))
        n = C.c_size_t(0)
        st = L.wdlb_server_workspace_size(C.byref(self.desc), C.byref(self.params), C.byref(n))
        if st != OK:
            raise WdlbError(st, "wdlb_server_workspace_size")
        self.pool = torch.empty(n.value, dtype=torch.uint8, device=device)
        torch.cuda.synchronize()
        h = C.c_void_p()
        st = L.wdlb_server_create(C.byref(self.desc), C.byref(self.params), C.c_void_p(self.pool.data_ptr()),
                                  n.value, C.byref(h))
        if st != OK:
            raise WdlbError(st, "wdlb_server_create")
        self.h, self._L = h, L
        self.sigma = float(sigma)

    def submit(self, H, eta, gx, tau=1.0):
        rid = C.c_uint64()
        r = Request(int(H), 0, float(eta), float(gx), float(tau))
        st = self._L.wdlb_server_submit(self.h, C.byref(r), C.byref(rid))
        if st != OK:
            raise WdlbError(st, f"submit: {self._L.wdlb_server_last_error(self.h).decode()}")
        return rid.value

    def poll(self, rid, H=None):
        """(Result, u_x(z) plane means or None).  The profile buffer is sized
        from the request's own H (a first call without a buffer); H, if
        given, is only checked against it."""
        res = Result()
        st = self._L.wdlb_server_poll(self.h, int(rid), C.byref(res), None, 0)
        if st != OK:
            raise WdlbError(st, "poll")
        if res.state != 2:
            return res, None
        if H is not None and int(H) != res.H:
            raise ValueError(f"request {rid} has H = {res.H}, not {H}")
        ux = np.zeros(res.H)
        st = self._L.wdlb_server_poll(self.h, int(rid), C.byref(res), _ptr(ux), ux.size)
        if st != OK:
            raise WdlbError(st, "poll")
        return res, ux

    def drain(self):
        st = self._L.wdlb_server_drain(self.h)
        if st != OK:
            raise WdlbError(st, f"drain: {self._L.wdlb_server_last_error(self.h).decode()}")

    def stats(self):
        s = ServerStats()
        self._L.wdlb_server_stats_get(self.h, C.byref(s))
        return {k: getattr(s, k) for k, _ in ServerStats._fields_}

    def destroy(self):
        if getattr(self, "h", None):
            self._L.wdlb_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass
