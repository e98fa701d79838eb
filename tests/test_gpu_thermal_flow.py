"""GPU coupled thermal flow (wdlb_init_thermal / wdlb_step_thermal) against
the FP64 oracle (ref.ThermalState) on the same seeded n, u, T.

Bars, FP64 storage: the populations and T to 1e-11 of their largest value
after every step, and the change of T over the run to 1e-9 of its largest
change (the shell and face sums are taken in another order, and the viscous
force is recovered from the step's total force by a subtraction; FP64
round-off).  FP32 storage (both local arithmetics): the populations to 1e-5
of their largest value (FP32 storage, a few 1e-8 per step, and shell sums
that cancel to many times the rounding of their largest term; measured
<= 5.1e-7 over four steps), T to 1e-6 of itself (stored in FP32, 6e-8, and
changed each step by the work of a velocity carrying that rounding;
measured <= 1.2e-7) and its change to 2e-5 of the largest change (measured
<= 8.7e-7), the bars of the FP32 conduction at rest.
"""
import math
import sys

import numpy as np
import pytest

from oracle import ref
from paper_1304_7880_amd.transport import carnahan_starling_c2, fit_damped_cosine
from paper_1304_7880_amd.workloads import packing_to_density, random_fields, random_temperature

pytestmark = pytest.mark.gpu

KT = 1.0 / 3.0


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _ctx(nx, ny, nz, walls, prec, sigma, eta, tau, g=(0.0, 0.0, 0.0), nonlocal_=True, smdb=True):
    from paper_1304_7880_amd import wdlb
    return wdlb.Context(nx, ny, nz, walls, prec, sigma, eta, tau, g, nonlocal_, smdb)


CASES = [
    # (name, shape, walls, sigma, eta, tau, g, smdb, steps, nsub, T noise); the sub-steps keep the explicit
    # conduction stable, dt (5/3) T / (omega0 nsub) <= 1/6, except in the one-sub-step case, whose grid-scale
    # T noise grows (about 6 times a step) and is kept small for that reason
    ("walled 21x19x13 sigma=3 (several tiles, ragged)", (21, 19, 13), True, 3.0, 0.3, 0.8, (1e-4, 2e-5, 0.0), True,
     4, 4, 0.1),
    ("periodic 9x7x11 sigma=4 (stencil wraps, one sub-step)", (9, 7, 11), False, 4.0, 0.25, 1.1, (0.0, 3e-5, 1e-5),
     True, 3, 1, 1e-3),
    ("periodic 10x9x12 sigma=4", (10, 9, 12), False, 4.0, 0.25, 1.1, (0.0, 3e-5, 1e-5), True, 3, 5, 0.1),
    ("walled 17x5x23 sigma=6 no SMDB", (17, 5, 23), True, 6.0, 0.35, 0.8, (2e-5, 0.0, 0.0), False, 3, 4, 0.1),
    ("walled 70x5x12 sigma=3 (per-node tiles ragged)", (70, 5, 12), True, 3.0, 0.3, 0.9, (1e-4, 0.0, 0.0), True,
     2, 4, 0.1),
    ("walled 23x18x19 sigma=5 (table-driven shell)", (23, 18, 19), True, 5.0, 0.3, 0.9, (1e-4, 0.0, 0.0), True, 2,
     6, 0.1),
]


BARS = {"fp64": (1e-11, 1e-11, 1e-9), "fp32": (1e-5, 1e-6, 2e-5), "fp32_local64": (1e-5, 1e-6, 2e-5)}
FP32_CASES = [CASES[0], CASES[2], CASES[5],
              # the compiled shells of sigma = 6 and 8 (FP32 only), ragged tiles
              ("walled 36x10x26 sigma=6 (compiled shell)", (36, 10, 26), True, 6.0, 0.35, 0.8, (2e-5, 0.0, 0.0),
               True, 2, 4, 0.1),
              ("periodic 24x20x30 sigma=8 (compiled shell)", (24, 20, 30), False, 8.0, 0.25, 1.0, (0.0, 0.0, 0.0),
               True, 2, 5, 0.1)]


def _run_case(case, prec):
    name, (nx, ny, nz), walls, sigma, eta, tau, g, smdb, steps, nsub, noise = case
    tf, tT, tdT = BARS[prec]
    _say(f"thermal flow {name} {prec}")
    n, u = random_fields(nx, ny, nz, packing_to_density(eta, sigma), 0.05, 0.01, seed=41)
    T0 = random_temperature(nx, ny, nz, KT, noise, seed=42)
    st = ref.ThermalState.from_fields(ref.Config(nx, ny, nz, walls, sigma, tau, g, True, smdb), n, u, T0)
    ctx = _ctx(nx, ny, nz, walls, prec, sigma, eta, tau, g, True, smdb)
    ctx.init_thermal(n, u, T0)
    for k in range(steps + 1):
        f_g, T_g = ctx.read_populations(), ctx.read_temperature()
        ef, eT = _rel(f_g, st.f), _rel(T_g, st.T)
        edT = _rel(T_g - T0, st.T - T0) if k else 0.0
        _say(f"  step {k}: f {ef:.2e}  T {eT:.2e}  change of T {edT:.2e}")
        assert ef < tf and eT < tT and edT < tdT, (k, ef, eT, edT)
        if k < steps:
            st.step(1, nsub)
            ctx.step_thermal(1, nsub)
    ctx.sync()
    ctx.destroy()


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_thermal_flow_matches_oracle(case):
    _run_case(case, "fp64")


@pytest.mark.parametrize("prec", ["fp32", "fp32_local64"])
@pytest.mark.parametrize("case", FP32_CASES, ids=[c[0] for c in FP32_CASES])
def test_thermal_flow_fp32_storage_matches_oracle(case, prec):
    _run_case(case, prec)


def test_several_steps_in_one_call():
    nx, ny, nz, sigma, eta, tau = 16, 12, 14, 4.0, 0.3, 0.9
    n, u = random_fields(nx, ny, nz, packing_to_density(eta, sigma), 0.05, 0.01, seed=43)
    T0 = random_temperature(nx, ny, nz, KT, 0.1, seed=44)
    st = ref.ThermalState.from_fields(ref.Config(nx, ny, nz, True, sigma, tau), n, u, T0)
    st.step(6, 4)
    ctx = _ctx(nx, ny, nz, True, "fp64", sigma, eta, tau)
    ctx.init_thermal(n, u, T0)
    ctx.step_thermal(6, 4)
    f_g, T_g = ctx.read_populations(), ctx.read_temperature()
    ctx.destroy()
    assert _rel(f_g, st.f) < 1e-11 and _rel(T_g, st.T) < 1e-11 and _rel(T_g - T0, st.T - T0) < 1e-9


def test_isothermal_temperature_gives_the_isothermal_step():
    """At T = kT everywhere theta = 1 exactly: the populations take the
    library's isothermal step (to the round-off of recovering F^v); T itself
    then moves with the flow's work and Q, so one step is compared."""
    nx, ny, nz, sigma, eta, tau, g = 21, 13, 17, 3.0, 0.3, 0.9, (1e-4, 2e-5, 0.0)
    n, u = random_fields(nx, ny, nz, packing_to_density(eta, sigma), 0.05, 0.01, seed=45)
    a = _ctx(nx, ny, nz, True, "fp64", sigma, eta, tau, g)
    a.init_thermal(n, u, np.full(nx * ny * nz, KT))
    a.step_thermal(1, 2)
    b = _ctx(nx, ny, nz, True, "fp64", sigma, eta, tau, g)
    b.init_fields(n, u)
    b.step(1)
    fa, fb = a.read_populations(), b.read_populations()
    a.destroy()
    b.destroy()
    assert _rel(fa, fb) < 1e-14, _rel(fa, fb)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-14), ("fp32", 1e-6)])
def test_rest_state_is_a_fixed_point(prec, tol):
    nx, ny, nz, sigma = 10, 8, 12, 3.0
    N = nx * ny * nz
    ctx = _ctx(nx, ny, nz, False, prec, sigma, 0.3, 0.9)
    ctx.init_thermal(np.full(N, packing_to_density(0.3, sigma)), np.zeros(3 * N), np.full(N, 0.41))
    f0, T0 = ctx.read_populations(), ctx.read_temperature()
    ctx.step_thermal(10, 4)
    f1, T = ctx.read_populations(), ctx.read_temperature()
    ctx.destroy()
    assert np.abs(T - T0).max() < tol * 0.41 and _rel(f1, f0) < tol


def test_sound_wave_runs_at_the_adiabatic_speed():
    """The oracle's pin of the sound speed, run on the GPU path: sigma = 8,
    eta = 0.25, a density wave of 128 nodes started on the adiabat; c^2 within
    1 % of kT d(nZ)/dn + (2/3) T Z^2."""
    sigma, eta, L, eps, tau = 8.0, 0.25, 128, 1e-3, 1.0
    N = 16 * L
    n0 = packing_to_density(eta, sigma)
    z = np.arange(L, dtype=np.float64)
    s = np.sin(2 * math.pi * z / L)
    Z = (1 + eta + eta ** 2 - eta ** 3) / (1 - eta) ** 3
    ctx = _ctx(4, 4, L, False, "fp64", sigma, eta, tau)
    ctx.init_thermal(np.repeat(n0 * (1 + eps * s), 16), np.zeros(3 * N), np.repeat(KT * (1 + 2.0 / 3.0 * Z * eps * s), 16))
    times, amps = [], []
    for t in range(0, 800, 2):
        rho, _ = ctx.read_fields()
        times.append(t)
        amps.append(2.0 / L * float((rho.reshape(L, 16).mean(1) / n0 - 1) @ s))
        ctx.step_thermal(2, 4)
    ctx.destroy()
    times, amps = np.array(times, dtype=np.float64), np.array(amps)
    sel = times >= 50
    om, ga = fit_damped_cosine(times[sel], amps[sel])
    q = 2 * math.pi / L
    c2 = (om * om + ga * ga) / (q * q)
    c2_ad = carnahan_starling_c2(eta) + 2.0 / 3.0 * KT * Z * Z
    _say(f"  c^2 {c2:.6f}  adiabatic {c2_ad:.6f}  isothermal {carnahan_starling_c2(eta):.6f}")
    assert abs(c2 / c2_ad - 1) < 0.01


def test_bad_input():
    from paper_1304_7880_amd import wdlb
    nx, ny, nz, sigma = 12, 9, 10, 3.0
    N = nx * ny * nz
    n, u = random_fields(nx, ny, nz, packing_to_density(0.3, sigma), 0.05, 0.01, seed=1)
    T = random_temperature(nx, ny, nz, KT, 0.1, seed=2)
    for prec in ("bf16", "bf16_local64"):
        c = _ctx(nx, ny, nz, True, prec, sigma, 0.3, 0.9)
        with pytest.raises(wdlb.WdlbError) as e:
            c.init_thermal(n, u, T)
        assert e.value.status == wdlb.E_INVAL
        c.destroy()
    c = _ctx(nx, ny, nz, True, "fp64", sigma, 0.3, 0.9, nonlocal_=False)
    with pytest.raises(wdlb.WdlbError) as e:
        c.init_thermal(n, u, T)
    assert e.value.status == wdlb.E_INVAL
    c.destroy()
    c = _ctx(nx, ny, nz, True, "fp64", sigma, 0.3, 0.9)
    for bad in (-T, T * np.nan):
        with pytest.raises(wdlb.WdlbError) as e:
            c.init_thermal(n, u, bad)
        assert e.value.status == wdlb.E_INVAL
    c.init_thermal(n, u, T)
    for nst, nsub in ((-1, 4), (1, 0)):
        with pytest.raises(wdlb.WdlbError) as e:
            c.step_thermal(nst, nsub)
        assert e.value.status == wdlb.E_INVAL
    c.step_thermal(2, 4)
    c.sync()
    c.destroy()
    assert N == T.size


def test_negative_temperature_is_reported():
    """A temperature that is not positive at a step's start (set from the
    host into the device array) is reported by the next sync."""
    from paper_1304_7880_amd import wdlb
    nx, ny, nz, sigma = 12, 9, 10, 3.0
    n, u = random_fields(nx, ny, nz, packing_to_density(0.3, sigma), 0.05, 0.0, seed=3)
    c = _ctx(nx, ny, nz, False, "fp64", sigma, 0.3, 0.9)
    c.init_thermal(n, u, np.full(nx * ny * nz, KT))
    c.T[5] = -1.0
    c.step_thermal(1, 1)
    with pytest.raises(wdlb.WdlbError) as e:
        c.sync()
    assert e.value.status == wdlb.E_UNSTABLE and "temperature" in str(e.value)
    c.destroy()


@pytest.mark.parametrize("prec,tol_f,tol_T,tol_dT", [("fp32_local64", 1e-5, 1e-6, 2e-5), ("fp64", 1e-11, 1e-11, 1e-9)])
def test_full_slab_z_only_matches_the_column_oracle(prec, tol_f, tol_T, tol_dT):
    """The benchmark's slab (512 x 512 x 256 between walls, sigma = 10, eta =
    0.40, tau = 0.7, g_x = 5e-7, the shells the bench runs) with seeded
    fields that depend on z only (n: 5 %, u_x: 1e-3, T: 10 % plane by plane),
    three coupled steps of four sub-steps: every column of the slab keeps
    the same values, and they equal the oracle's on a 4 x 4 x 256 column of
    the same planes (the shell sums of an x,y-homogeneous state are the
    same on any width), sampled at 64 columns for the populations."""
    from paper_1304_7880_amd.workloads import SLAB_LARGE as w
    nx, ny, nz = w.nx, w.ny, w.nz
    rng = np.random.default_rng(51)
    n_z = w.n0 * (1 + 0.05 * rng.uniform(-1, 1, nz))
    ux_z = 1e-3 * rng.uniform(-1, 1, nz)
    T_z = KT * (1 + 0.1 * rng.uniform(-1, 1, nz))
    cfg = ref.Config(4, 4, nz, True, w.sigma, w.tau, w.g)
    uc = np.zeros(3 * cfg.N)
    uc[:cfg.N] = np.repeat(ux_z, 16)
    st = ref.ThermalState.from_fields(cfg, np.repeat(n_z, 16), uc, np.repeat(T_z, 16))
    st.step(3, 4)
    fo = st.f.reshape(19, nz, 16)[:, :, 0]
    To = st.T.reshape(nz, 16)[:, 0]
    _say(f"full slab z-only {prec}: oracle column done")
    N = nx * ny * nz
    u = np.zeros(3 * N)
    u[:N] = np.repeat(ux_z, nx * ny)
    ctx = _ctx(nx, ny, nz, True, prec, w.sigma, w.eta, w.tau, w.g)
    ctx.init_thermal(np.repeat(n_z, nx * ny), u, np.repeat(T_z, nx * ny))
    del u
    ctx.step_thermal(3, 4)
    Tg = ctx.read_temperature().reshape(nz, nx * ny)
    assert np.all(Tg == Tg[:, :1]), "columns differ in T"
    eT, edT = _rel(Tg[:, 0], To), _rel(Tg[:, 0] - T_z, To - T_z)
    cols = np.random.default_rng(52).choice(nx * ny, 64, replace=False)
    fg = ctx.read_populations().reshape(19, nz, nx * ny)[:, :, cols]
    ctx.destroy()
    assert np.all(fg == fg[:, :, :1]), "columns differ in f"
    ef = _rel(fg[:, :, 0], fo)
    _say(f"  f {ef:.2e}  T {eT:.2e}  change of T {edT:.2e}")
    assert ef < tol_f and eT < tol_T and edT < tol_dT, (ef, eT, edT)


def test_heat_mode_decays_at_lambda_over_n_cp():
    """The oracle's heat-mode pin on the GPU path (FP64): a temperature wave at
    constant pressure, sigma = 8, decays at the rate of the same wave at rest
    (the conduction oracle) divided by gamma = c_ad^2 / c_T^2, within 2 %."""
    from oracle import conduction
    sigma, eta, tau, L, eps = 8.0, 0.25, 1.0, 128, 1e-3
    N = 16 * L
    cfg = ref.Config(4, 4, L, False, sigma, tau)
    n0 = packing_to_density(eta, sigma)
    Z = (1 + eta + eta ** 2 - eta ** 3) / (1 - eta) ** 3
    dnZ = carnahan_starling_c2(eta) / KT
    s = np.sin(2 * math.pi * np.arange(L) / L)
    sr = np.repeat(s, 16)
    r = conduction.rate(cfg, np.full(N, n0), KT * (1 + eps * sr), 1.0 / tau)
    r_rest = -float(r @ sr) / float(sr @ sr) / (KT * eps)
    gamma = (carnahan_starling_c2(eta) + 2.0 / 3.0 * KT * Z * Z) / carnahan_starling_c2(eta)
    ctx = _ctx(4, 4, L, False, "fp64", sigma, eta, tau)
    ctx.init_thermal(np.repeat(n0 * (1 - Z / dnZ * eps * s), 16), np.zeros(3 * N), np.repeat(KT * (1 + eps * s), 16))
    ts, amps = [], []
    for t in range(0, 601, 5):
        ts.append(t)
        amps.append(float((ctx.read_temperature().reshape(L, 16).mean(1) - KT) @ s))
        ctx.step_thermal(5, 4)
    ctx.destroy()
    ts, amps = np.array(ts, dtype=np.float64), np.array(amps)
    sel = ts >= 100
    rate = -np.polyfit(ts[sel], np.log(amps[sel]), 1)[0]
    _say(f"  heat mode rate {rate:.6e}  lambda q^2/(n c_p) {r_rest / gamma:.6e}")
    assert abs(rate / (r_rest / gamma) - 1) < 0.02


def test_checkpoint_and_resume():
    """Save the state (wdlb_save_state) and T after three coupled steps, load
    both into a new context, step three more: the same populations and T as
    six steps without the interruption, bit for bit."""
    nx, ny, nz, sigma, eta, tau = 14, 12, 13, 4.0, 0.3, 0.9
    n, u = random_fields(nx, ny, nz, packing_to_density(eta, sigma), 0.05, 0.01, seed=61)
    T0 = random_temperature(nx, ny, nz, KT, 0.05, seed=62)
    a = _ctx(nx, ny, nz, True, "fp32_local64", sigma, eta, tau)
    a.init_thermal(n, u, T0)
    a.step_thermal(3, 4)
    blob, Tk = a.save_state(), a.read_temperature()
    a.step_thermal(3, 4)
    fa, Ta = a.read_populations(), a.read_temperature()
    a.destroy()
    b = _ctx(nx, ny, nz, True, "fp32_local64", sigma, eta, tau)
    b.init_thermal(n, u, T0)          # allocates b.T; the state and T are then replaced
    b.load_state(blob)
    b.T.copy_(__import__("torch").from_numpy(Tk.astype(np.float32)))
    b.step_thermal(3, 4)
    fb, Tb = b.read_populations(), b.read_temperature()
    b.destroy()
    assert np.array_equal(fa, fb) and np.array_equal(Ta, Tb)


@pytest.mark.parametrize("prec,sigma", [("fp32_local64", 6.0), ("fp32_local64", 10.0), ("fp64", 10.0)])
def test_compiled_and_table_driven_kernels_give_the_same_bits(prec, sigma):
    """The coupled step on the kernels compiled for the shell (the shells, the
    thermal sums at u = 0, with their density ring in FP32) and on the table-driven
    kernels of the same tiles: the same populations and T, bit for bit, after
    three steps on a walled lattice with ragged tiles."""
    nx, ny, nz, eta, tau = 37, 19, 2 * int(sigma) + 9, 0.3, 0.85
    n, u = random_fields(nx, ny, nz, packing_to_density(eta, sigma), 0.05, 0.01, seed=71)
    T0 = random_temperature(nx, ny, nz, KT, 0.05, seed=72)
    out = []
    for forced in (False, True):
        ctx = _ctx(nx, ny, nz, True, prec, sigma, eta, tau, (1e-4, 2e-5, 0.0))
        tile, spec = ctx.get_tile()
        if forced:
            ctx.set_tile(tile)
            assert ctx.get_tile() == (tile, False)
        else:
            assert spec
        ctx.init_thermal(n, u, T0)
        ctx.step_thermal(3, 4)
        out.append((ctx.read_populations(), ctx.read_temperature()))
        ctx.destroy()
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


def test_allocation_free_context_steps_the_same():
    """The coupled flow on a context made by wdlb_create_static (the
    library's own device array as the workspace) gives the bits of a context
    on a caller's workspace; T stays the caller's (FP32 storage, walled
    17x11x15, sigma = 3, three steps)."""
    from paper_1304_7880_amd import wdlb
    nx, ny, nz, sigma, eta, tau = 17, 11, 15, 3.0, 0.3, 0.9
    n, u = random_fields(nx, ny, nz, packing_to_density(eta, sigma), 0.05, 0.01, seed=81)
    T0 = random_temperature(nx, ny, nz, KT, 0.05, seed=82)
    out = []
    for static in (False, True):
        ctx = wdlb.Context(nx, ny, nz, True, "fp32_local64", sigma, eta, tau, (1e-4, 0.0, 0.0), static=static)
        ctx.init_thermal(n, u, T0)
        ctx.step_thermal(3, 4)
        out.append((ctx.read_populations(), ctx.read_temperature()))
        ctx.destroy()
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


@pytest.mark.parametrize("prec", ["fp64", "fp32_local64"])
def test_graph_replay_equals_eager_steps(prec):
    """Six coupled steps in one call (three graph replays of two steps, the
    graph captured for this T and nsub) against six eager steps: the same
    bits; then a call with another nsub (a new capture) and a single step
    (eager) keep them equal."""
    nx, ny, nz, sigma, eta, tau = 20, 13, 15, 4.0, 0.3, 0.9
    n, u = random_fields(nx, ny, nz, packing_to_density(eta, sigma), 0.05, 0.01, seed=91)
    T0 = random_temperature(nx, ny, nz, KT, 0.05, seed=92)
    out = []
    for graphs in (True, False):
        ctx = _ctx(nx, ny, nz, True, prec, sigma, eta, tau, (1e-4, 0.0, 0.0))
        ctx.set_graphs(graphs)
        ctx.init_thermal(n, u, T0)
        ctx.step_thermal(6, 4)
        ctx.step_thermal(2, 5)
        ctx.step_thermal(1, 4)
        out.append((ctx.read_populations(), ctx.read_temperature()))
        ctx.destroy()
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
