"""GPU thermal fields (Sec. 3: Q of eq. campob1, B_i of eq. campos, F^T of
eq. thermalforce) through the C ABI against the FP64 oracle, element by
element, on seeded random n, u, T.

Bars: FP64 1e-13 of the largest value of each field (round-off of sums over
the shell in another order; measured at most 4.4e-15).  FP32: the inputs are
rounded to FP32 first (relative 6e-8), and a temperature difference of a
tenth of T carries that rounding as ~1e-6 of itself; the shell sums of random
differences cancel to about sqrt(|S|) of their terms, so the round-off is
some 1e-6 of the largest value (measured at most 2.1e-6), held to 2e-5.
"""
import sys

import numpy as np
import pytest

from oracle import ref
from paper_1304_7880_amd.workloads import packing_to_density, random_fields, random_temperature

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _ctx(nx, ny, nz, walls, prec, sigma, eta=0.3):
    from paper_1304_7880_amd import wdlb
    return wdlb.Context(nx, ny, nz, walls, prec, sigma, eta, 1.0, (0.0, 0.0, 0.0))


CASES = [
    # (name, shape, walls, sigma, eta)
    ("walled 37x21x19 sigma=4 (32x8 tiles, ragged)", (37, 21, 19), True, 4.0, 0.3),
    ("periodic 20x18x16 sigma=3", (20, 18, 16), False, 3.0, 0.25),
    ("walled 4x4x16 sigma=4 (domain smaller than stencil)", (4, 4, 16), True, 4.0, 0.2),
    ("walled 40x12x30 sigma=6", (40, 12, 30), True, 6.0, 0.35),
    ("periodic 14x13x15 sigma=5.5 (non-integer sigma)", (14, 13, 15), False, 5.5, 0.3),
    ("walled 33x10x20 sigma=7 (table-driven density)", (33, 10, 20), True, 7.0, 0.25),
    ("walled 22x21x26 sigma=10", (22, 21, 26), True, 10.0, 0.3),
    ("walled 27x26x30 sigma=12", (27, 26, 30), True, 12.0, 0.2),
    # reach 16: the FP64 rings do not fit in LDS, the kernel reads through the caches
    ("walled 20x18x36 sigma=16 (largest sigma)", (20, 18, 36), True, 16.0, 0.2),
]


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-13), ("fp32", 2e-5), ("fp32_local64", 2e-5)])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_thermal_fields_random(case, prec, tol):
    name, (nx, ny, nz), walls, sigma, eta = case
    _say(f"thermal {name} {prec}")
    n, u = random_fields(nx, ny, nz, packing_to_density(eta, sigma), 0.05, 0.01, seed=11)
    T = random_temperature(nx, ny, nz, 1.0 / 3.0, 0.1, seed=12)
    cfg = ref.Config(nx, ny, nz, walls, sigma, 1.0)
    Q_o, B_o, FT_o = ref.thermal(cfg, n, ref.nbar(cfg, n), u, T)
    ctx = _ctx(nx, ny, nz, walls, prec, sigma, eta)
    Q_g, B_g, FT_g = ctx.thermal_fields(n, u, T)
    ctx.destroy()
    e = (_rel(Q_g, Q_o), _rel(B_g, B_o), _rel(FT_g, FT_o))
    _say(f"  Q {e[0]:.2e}  B {e[1]:.2e}  F^T {e[2]:.2e}")
    assert max(e) < tol, e


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_uniform_temperature_and_velocity_give_zero(prec):
    nx, ny, nz, sigma = 24, 17, 15, 4.0
    n, _ = random_fields(nx, ny, nz, packing_to_density(0.3, sigma), 0.05, 0.0, seed=3)
    u = np.repeat([2e-3, -1e-3, 5e-4], nx * ny * nz)
    T = np.full(nx * ny * nz, 0.4)
    ctx = _ctx(nx, ny, nz, True, prec, sigma)
    Q, B, FT = ctx.thermal_fields(n, u, T)
    ctx.destroy()
    assert not Q.any() and not B.any() and not FT.any()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_z_profile_gives_exact_zero_lateral_components(prec):
    """n, u, T that depend on z only: the x and y components of B and F^T
    are exactly zero (mirror images summed as differences)."""
    nx, ny, nz, sigma = 40, 19, 23, 6.0
    rng = np.random.default_rng(5)
    nz_prof = packing_to_density(0.3, sigma) * (1 + 0.1 * rng.uniform(-1, 1, nz))
    T_prof = (1 / 3) * (1 + 0.1 * rng.uniform(-1, 1, nz))
    ux_prof = 1e-3 * rng.uniform(-1, 1, nz)
    n = np.repeat(nz_prof, nx * ny)
    T = np.repeat(T_prof, nx * ny)
    u = np.concatenate([np.repeat(ux_prof, nx * ny), np.zeros(2 * nx * ny * nz)])
    ctx = _ctx(nx, ny, nz, True, prec, sigma)
    Q, B, FT = ctx.thermal_fields(n, u, T)
    ctx.destroy()
    N = nx * ny * nz
    assert not B[:2 * N].any() and not FT[:2 * N].any()
    assert np.abs(B[2 * N:]).max() > 0


@pytest.mark.parametrize("prec", ["fp64", "fp32_local64"])
def test_call_leaves_the_state(prec):
    """Stepping after a thermal-field call gives the same state, bit for
    bit, as stepping without it (graph replay on and off)."""
    nx, ny, nz, sigma = 21, 19, 13, 3.0
    n, u = random_fields(nx, ny, nz, packing_to_density(0.3, sigma), 0.05, 0.01, seed=7)
    T = random_temperature(nx, ny, nz, 1.0 / 3.0, 0.1, seed=8)
    outs = []
    for call in (False, True):
        for graphs in (True, False):
            ctx = _ctx(nx, ny, nz, True, prec, sigma)
            ctx.set_graphs(graphs)
            ctx.init_fields(n, u)
            ctx.step(4)
            if call:
                ctx.thermal_fields(n * 1.01, u, T)
            ctx.step(5)
            outs.append(ctx.read_fields(with_forces=True))
            ctx.destroy()
    for o in outs[1:]:
        for a, b in zip(outs[0], o):
            assert np.array_equal(a, b)


def test_thermal_fields_before_init_and_bad_input():
    from paper_1304_7880_amd import wdlb
    nx, ny, nz, sigma = 12, 9, 10, 3.0
    n, u = random_fields(nx, ny, nz, packing_to_density(0.3, sigma), 0.05, 0.01, seed=1)
    T = random_temperature(nx, ny, nz, 1.0 / 3.0, 0.1, seed=2)
    ctx = _ctx(nx, ny, nz, True, "fp64", sigma)
    Q, B, FT = ctx.thermal_fields(n, u, T)      # no init needed
    assert np.isfinite(Q).all() and np.abs(Q).max() > 0
    T_bad = T.copy()
    T_bad[5] = 0.0
    with pytest.raises(wdlb.WdlbError) as ei:
        ctx.thermal_fields(n, u, T_bad)
    assert ei.value.status == wdlb.E_INVAL
    n_bad = n.copy()
    n_bad[3] = -1.0
    with pytest.raises(wdlb.WdlbError) as ei:
        ctx.thermal_fields(n_bad, u, T)
    assert ei.value.status == wdlb.E_INVAL
    with pytest.raises(wdlb.WdlbError) as ei:      # midpoint packing fraction >= 1
        ctx.thermal_fields(n * 4.0, u, T)
    assert ei.value.status == wdlb.E_UNSTABLE
    Q2, _, _ = ctx.thermal_fields(n, u, T)
    assert np.array_equal(Q, Q2)
    ctx.destroy()


def test_full_size_slab_z_profile_against_column():
    """The 512x512x256 slit at sigma = 10 in FP32 with n, u, T that depend on
    z only: every (x, y) column equals the oracle's fields on a 4x4x256
    periodic-in-x,y lattice with the same profiles (the shell sums of a
    z-only state do not depend on the lateral extent)."""
    nx, ny, nz, sigma, eta = 512, 512, 256, 10.0, 0.4
    rng = np.random.default_rng(21)
    z = np.arange(nz)
    nz_prof = packing_to_density(eta, sigma) * (1 + 0.05 * np.sin(2 * np.pi * z / 37) + 0.02 * rng.uniform(-1, 1, nz))
    T_prof = (1 / 3) * (1 + 0.1 * np.cos(2 * np.pi * z / 51) + 0.02 * rng.uniform(-1, 1, nz))
    uz_prof = 1e-3 * np.sin(2 * np.pi * z / 64)
    ux_prof = 1e-3 * rng.uniform(-1, 1, nz)

    def fields(mx, my):
        m = mx * my
        return (np.repeat(nz_prof, m), np.concatenate([np.repeat(ux_prof, m), np.zeros(nz * m), np.repeat(uz_prof, m)]),
                np.repeat(T_prof, m))

    cfg = ref.Config(4, 4, nz, True, sigma, 1.0)
    n4, u4, T4 = fields(4, 4)
    Q_o, B_o, FT_o = ref.thermal(cfg, n4, ref.nbar(cfg, n4), u4, T4)
    col = lambda a, k: a[k * 16 * nz:(k + 1) * 16 * nz].reshape(nz, 16)[:, 0]
    _say("thermal 512x512x256 sigma=10 fp32, z-only fields")
    n, u, T = fields(nx, ny)
    ctx = _ctx(nx, ny, nz, True, "fp32", sigma, eta)
    Q, B, FT = ctx.thermal_fields(n, u, T)
    ctx.destroy()
    del n, u, T
    m = nx * ny
    Qz = Q.reshape(nz, m)
    Bz = B[2 * nz * m:].reshape(nz, m)
    Fz = FT[2 * nz * m:].reshape(nz, m)
    eq = float(np.abs(Qz - col(Q_o, 0)[:, None]).max() / np.abs(Q_o).max())
    eb = float(np.abs(Bz - col(B_o, 2)[:, None]).max() / np.abs(B_o).max())
    ef = float(np.abs(Fz - col(FT_o, 2)[:, None]).max() / np.abs(FT_o).max())
    _say(f"  Q {eq:.2e}  B_z {eb:.2e}  F^T_z {ef:.2e}")
    assert not B[:2 * nz * m].any() and not FT[:2 * nz * m].any()
    assert max(eq, eb, ef) < 2e-5


@pytest.mark.parametrize("prec,sigma,shape", [("fp32", 6.0, (40, 24, 30)), ("fp32", 10.0, (70, 20, 26)),
                                              ("fp64", 10.0, (70, 20, 26))])
def test_compiled_and_table_driven_kernels_agree_bitwise(prec, sigma, shape):
    """At a compiled shell (FP32; FP64 at sigma = 10): the compiled kernel
    (automatic choice) and the table-driven ring kernel (a forced shell tile)
    give the same bits."""
    nx, ny, nz = shape
    n, u = random_fields(nx, ny, nz, packing_to_density(0.3, sigma), 0.05, 0.01, seed=4)
    T = random_temperature(nx, ny, nz, 1.0 / 3.0, 0.1, seed=5)
    outs = []
    for forced in (False, True):
        ctx = _ctx(nx, ny, nz, True, prec, sigma)
        if forced:
            ctx.set_tile(6)
        outs.append(ctx.thermal_fields(n, u, T))
        ctx.destroy()
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


def test_step_instability_survives_a_thermal_call():
    """A step that met a packing fraction >= 1 is still reported by the next
    synchronising call after a (successful) thermal-field evaluation."""
    from paper_1304_7880_amd import wdlb
    nx, ny, nz, sigma = 8, 8, 8, 4.0
    ctx = _ctx(nx, ny, nz, True, "fp32", sigma)
    ctx.init_fields(np.full(nx * ny * nz, packing_to_density(1.2, sigma)), np.zeros(3 * nx * ny * nz))
    ctx.step(1)
    n, u = random_fields(nx, ny, nz, packing_to_density(0.3, sigma), 0.05, 0.01, seed=9)
    Q, _, _ = ctx.thermal_fields(n, u, random_temperature(nx, ny, nz, 1.0 / 3.0, 0.1, seed=10))
    assert np.isfinite(Q).all()
    with pytest.raises(wdlb.WdlbError) as e:
        ctx.sync()
    assert e.value.status == wdlb.E_UNSTABLE
    ctx.destroy()


@pytest.mark.parametrize("prec,tol", [("bf16", 2e-5), ("bf16_local64", 2e-5)])
def test_thermal_fields_bf16_storage_modes(prec, tol):
    """The BF16 storage modes keep FP32 per-step arrays: the thermal fields
    are those of FP32."""
    nx, ny, nz, sigma, walls = 37, 21, 19, 4.0, True
    n, u = random_fields(nx, ny, nz, packing_to_density(0.3, sigma), 0.05, 0.01, seed=11)
    T = random_temperature(nx, ny, nz, 1.0 / 3.0, 0.1, seed=12)
    cfg = ref.Config(nx, ny, nz, walls, sigma, 1.0)
    Q_o, B_o, FT_o = ref.thermal(cfg, n, ref.nbar(cfg, n), u, T)
    ctx = _ctx(nx, ny, nz, walls, prec, sigma)
    Q_g, B_g, FT_g = ctx.thermal_fields(n, u, T)
    ctx.destroy()
    e = (_rel(Q_g, Q_o), _rel(B_g, B_o), _rel(FT_g, FT_o))
    assert max(e) < tol, e


@pytest.mark.parametrize("prec", ["fp64", "fp32_local64"])
def test_device_entry_point_equals_host_entry_point(prec):
    """wdlb_thermal_fields_device on device tensors gives the host call's
    values bit for bit (inputs rounded to the storage real first on both
    sides), twice in a row, the second on other fields; a packing fraction
    >= 1 is reported by the next sync."""
    import torch
    from paper_1304_7880_amd import wdlb
    nx, ny, nz, sigma = 37, 21, 19, 6.0
    dt = torch.float64 if prec == "fp64" else torch.float32
    ctx = _ctx(nx, ny, nz, True, prec, sigma)
    N = nx * ny * nz
    for seed in (3, 4):
        n, u = random_fields(nx, ny, nz, packing_to_density(0.3, sigma), 0.05, 0.01, seed=seed)
        T = random_temperature(nx, ny, nz, 1.0 / 3.0, 0.1, seed=seed + 10)
        dn, du, dT = (torch.tensor(a, dtype=dt, device="cuda") for a in (n, u, T))
        Q, B, FT = (torch.empty(k * N, dtype=dt, device="cuda") for k in (1, 3, 3))
        ctx.thermal_fields_device(dn, du, dT, Q, B, FT)
        ctx.sync()
        # the host call on the same (rounded) inputs
        hQ, hB, hFT = ctx.thermal_fields(dn.cpu().double().numpy(), du.cpu().double().numpy(),
                                         dT.cpu().double().numpy())
        assert np.array_equal(Q.cpu().double().numpy(), hQ)
        assert np.array_equal(B.cpu().double().numpy(), hB)
        assert np.array_equal(FT.cpu().double().numpy(), hFT)
    dn4 = torch.full((N,), packing_to_density(1.2, sigma), dtype=dt, device="cuda")
    ctx.thermal_fields_device(dn4, du, dT, Q, B, FT)
    with pytest.raises(wdlb.WdlbError) as e:
        ctx.sync()
    assert e.value.status == wdlb.E_UNSTABLE
    ctx.destroy()
