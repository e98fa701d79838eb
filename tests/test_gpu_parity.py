"""GPU (HIP, gfx950) against the FP64 oracle, element by element.

Every case runs the library through its C ABI and the oracle on the same
seeded inputs.  FP64 on the GPU must agree to round-off.  FP32 must agree
within 1e-5 relative on the flow (u_x(z) and the pore-averaged flux) of the
slit workloads.  On random fields the shell sums cancel: with 5 % density
noise the mean-field force is about 300 times smaller than the sum of the
magnitudes of its |S| terms, so FP32 round-off there is ~300 x 6e-8 of the
largest force; the random-field FP32 tolerances (1e-4 on rho, u, f; 1e-3 on
F and A0, relative to the largest value) are that round-off, not a looser
physics target.
"""
import math
import sys

import numpy as np
import pytest

from oracle import ref
from paper_1304_7880_amd.workloads import (SLAB_64, SLAB_SMALL, initial_fields, packing_to_density,
                                           random_fields)

pytestmark = pytest.mark.gpu


def _ctx(nx, ny, nz, walls, prec, sigma, eta, tau, g, nonlocal_=True, smdb=True):
    from paper_1304_7880_amd import wdlb
    return wdlb.Context(nx, ny, nz, walls, prec, sigma, eta, tau, g, nonlocal_, smdb)


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


CASES = [
    # (name, shape, walls, sigma, eta, tau, g, steps)
    ("walled 21x19x13 sigma=3 (several tiles, ragged)", (21, 19, 13), True, 3.0, 0.3, 0.8, (1e-4, 2e-5, 0.0), 4),
    ("periodic 9x7x11 sigma=4 (stencil wraps)", (9, 7, 11), False, 4.0, 0.25, 1.1, (0.0, 3e-5, 1e-5), 3),
    ("walled 4x4x16 sigma=4 (domain smaller than stencil)", (4, 4, 16), True, 4.0, 0.2, 1.0, (1e-4, 0, 0), 5),
    ("walled 17x5x23 sigma=6", (17, 5, 23), True, 6.0, 0.35, 0.8, (2e-5, 0, 0), 3),
    # 12 wide: the density kernel on the narrow 16x16x2 tiles (table-driven at sigma = 8)
    ("walled 12x9x21 sigma=8", (12, 9, 21), True, 8.0, 0.3, 0.9, (1e-4, 0, 0), 2),
    # 16 wide in x: the narrow 16x16x2 tiles (compiled for sigma = 4 in fp32)
    ("walled 16x16x14 sigma=4 (narrow tiles)", (16, 16, 14), True, 4.0, 0.3, 1.0, (2e-5, 0, 0), 3),
    # the largest compiled shell (reach 11) against the oracle's fields
    ("walled 22x21x26 sigma=10", (22, 21, 26), True, 10.0, 0.3, 0.9, (1e-4, 0, 0), 2),
    # 64x4 tiles of the per-node kernels, ragged in x (70 = 64 + 6) and y (5 = 4 + 1)
    ("walled 70x5x12 sigma=3 (per-node tiles ragged)", (70, 5, 12), True, 3.0, 0.3, 0.9, (1e-4, 2e-5, 0), 3),
    # shells with no compiled kernels: the table-driven shell and ball sums
    ("walled 23x18x19 sigma=5 (table-driven shell)", (23, 18, 19), True, 5.0, 0.3, 0.9, (1e-4, 0, 0), 2),
    ("periodic 14x13x15 sigma=5.5 (non-integer sigma)", (14, 13, 15), False, 5.5, 0.3, 0.9, (0, 2e-5, 1e-5), 2),
    ("walled 33x10x20 sigma=7 (table-driven shell)", (33, 10, 20), True, 7.0, 0.25, 1.0, (1e-4, 0, 0), 2),
    ("walled 27x26x30 sigma=12 (reach 12, beyond the compiled shells)", (27, 26, 30), True, 12.0, 0.2, 1.0,
     (1e-4, 0, 0), 1),
]


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-11), ("fp32", 1e-4)])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_random_fields_few_steps(case, prec, tol):
    name, (nx, ny, nz), walls, sigma, eta, tau, g, steps = case
    _say(f"case {name} {prec}")
    n0 = packing_to_density(eta, sigma)
    n, u = random_fields(nx, ny, nz, n0, 0.05, 0.01, seed=7)
    cfg = ref.Config(nx, ny, nz, walls, sigma, tau, g)
    st = ref.State.from_fields(cfg, n, u)
    ctx = _ctx(nx, ny, nz, walls, prec, sigma, eta, tau, g)
    ctx.init_fields(n, u)
    for k in range(steps + 1):
        rho_o, u_o, F_o, A_o = st.fields()
        rho_g, u_g, F_g, A_g = ctx.read_fields(with_forces=True)
        assert _rel(rho_g, rho_o) < tol, ("rho", k)
        assert _rel(u_g, u_o) < tol, ("u", k)
        assert _rel(F_g, F_o) < 10 * tol, ("F", k)
        assert _rel(A_g, A_o) < 10 * tol, ("A0", k)
        f_g = ctx.read_populations()
        assert _rel(f_g, st.f) < tol, ("f", k)
        if k < steps:
            st.step(1)
            ctx.step(1)
    ctx.sync()
    ctx.destroy()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-11), ("fp32", 1e-4)])
@pytest.mark.parametrize("variant", range(7))
def test_shell_tile_variants(variant, prec, tol):
    """Every contact-shell tile variant (LDS rings of 32x8x2, 32x16x1 and
    16x16x2, and the 16x16x1 and 32x8x2 tiles reading gamma through the
    caches), forced on a walled 40x20x13 lattice that leaves ragged tiles in
    x, y and z."""
    from paper_1304_7880_amd import wdlb
    nx, ny, nz, sigma, eta, tau, g = 40, 20, 13, 4.0, 0.3, 0.9, (1e-4, -3e-5, 0.0)
    _say(f"tile variant {variant} {prec}")
    n0 = packing_to_density(eta, sigma)
    n, u = random_fields(nx, ny, nz, n0, 0.05, 0.01, seed=11)
    st = ref.State.from_fields(ref.Config(nx, ny, nz, True, sigma, tau, g), n, u)
    ctx = _ctx(nx, ny, nz, True, prec, sigma, eta, tau, g)
    ctx.set_tile(variant)
    assert ctx.get_tile() == (variant, False)
    ctx.init_fields(n, u)
    for k in range(3):
        rho_o, u_o, F_o, A_o = st.fields()
        rho_g, u_g, F_g, A_g = ctx.read_fields(with_forces=True)
        assert _rel(rho_g, rho_o) < tol, ("rho", k)
        assert _rel(u_g, u_o) < tol, ("u", k)
        assert _rel(F_g, F_o) < 10 * tol, ("F", k)
        assert _rel(A_g, A_o) < 10 * tol, ("A0", k)
        st.step(1)
        ctx.step(1)
    ctx.set_tile(-1)
    ctx.destroy()


def test_shell_tile_that_does_not_fit_is_refused():
    """sigma = 16 in FP64: the 32x8x2 LDS rings exceed 160 KB; forcing that
    variant fails and leaves the automatic choice in place."""
    from paper_1304_7880_amd import wdlb
    ctx = _ctx(8, 8, 40, True, "fp64", 16.0, 0.2, 1.0, (0, 0, 0))
    auto = ctx.get_tile()
    with pytest.raises(wdlb.WdlbError):
        ctx.set_tile(0)
    assert ctx.get_tile() == auto
    ctx.destroy()


SPECIALISED = [3.0, 4.0, 6.0, 8.0, 10.0]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("sigma", SPECIALISED)
def test_compiled_shell_equals_table_driven(sigma, prec):
    """The kernels compiled for one shell and the table-driven kernels on the
    same tile sum the same terms in the same order: identical results, bit
    for bit, on a walled lattice with ragged tiles."""
    from paper_1304_7880_amd import wdlb
    nx, ny, nz, eta, tau, g = 37, 19, 2 * int(sigma) + 9, 0.3, 0.85, (1e-4, 2e-5, -1e-5)
    _say(f"compiled shell sigma={sigma} {prec}")
    n0 = packing_to_density(eta, sigma)
    n, u = random_fields(nx, ny, nz, n0, 0.05, 0.01, seed=5)
    out = []
    for forced in (False, True):
        ctx = _ctx(nx, ny, nz, True, prec, sigma, eta, tau, g)
        tile, spec = ctx.get_tile()
        if forced:
            ctx.set_tile(tile)
            assert ctx.get_tile() == (tile, False)
        else:
            # FP32 at sigma >= 8 and FP64 at sigma = 10: the compiled viscous
            # kernel on the tile that reads gamma through the caches
            assert spec, (tile, spec)
            if sigma == 10.0 or (sigma == 8.0 and prec == "fp32"):
                assert tile == 6, tile
        ctx.init_fields(n, u)
        ctx.step(3)
        out.append(ctx.read_fields(with_forces=True))
        ctx.destroy()
    for k, name in enumerate(("rho", "u", "F", "A0")):
        assert np.array_equal(out[0][k], out[1][k]), (name, _rel(out[0][k], out[1][k]))


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32_local64", 1e-5), ("fp32", 1e-4)])
def test_small_slab_full_run(prec, tol):
    """The 4x4x16 slit (sigma = 4, eta = 0.2, tau = 1, g_x = 1e-6), 2000 steps:
    n(z), u_x(z) and the pore-averaged flux against the oracle.  FP32 storage
    with FP64 local arithmetic meets 1e-5; FP32 local arithmetic (measured
    6e-5 on u_x(z), 1e-5 on the flux) is held to 1e-4."""
    w = SLAB_SMALL
    _say(f"slab {w.name} {prec}")
    n, u = initial_fields(w)
    cfg = ref.Config(w.nx, w.ny, w.nz, w.walls_z, w.sigma, w.tau, w.g)
    st = ref.State.from_fields(cfg, n, u)
    st.step(w.steps)
    nz_o, ux_o, J_o, up_o, M_o = st.reduce()
    ctx = _ctx(w.nx, w.ny, w.nz, True, prec, w.sigma, w.eta, w.tau, w.g)
    ctx.init_fields(n, u)
    ctx.step(w.steps)
    ctx.sync()
    nz_g, ux_g = ctx.read_profiles()
    J_g, up_g, M_g = ctx.read_flux()
    _say(f"  u_x(z) rel err {_rel(ux_g, ux_o):.3e}  J rel err {abs(J_g - J_o) / abs(J_o):.3e}")
    assert _rel(ux_g, ux_o) < tol
    assert abs(J_g - J_o) < tol * abs(J_o)
    assert abs(up_g - up_o) < tol * abs(up_o)
    assert _rel(nz_g, nz_o) < tol
    assert abs(M_g - M_o) < 1e-6 * M_o
    ctx.destroy()


def test_plain_bgk_poiseuille_closed_form():
    """nonlocal = 0: forced BGK between walls reaches the exact profile
    g/(2 nu) (z_w^2 - z^2) + g (4 l^2 - 3)/(4 l)."""
    H, g, tau = 16, 1e-5, 1.3
    ctx = _ctx(8, 8, H, True, "fp32", 4.0, 0.2, tau, (g, 0, 0), nonlocal_=False)
    ctx.init_fields(np.ones(8 * 8 * H), np.zeros(3 * 8 * 8 * H))
    nu = (tau - 0.5) / 3
    ctx.step(int(40 * H * H / (nu * math.pi ** 2)))
    _, ux = ctx.read_profiles()
    z = np.arange(H) - (H - 1) / 2
    lam = 2 * tau - 1
    pred = g / (2 * nu) * ((H / 2) ** 2 - z ** 2) + g * (4 * lam ** 2 - 3) / (4 * lam)
    _say(f"  poiseuille rel err {_rel(ux, pred):.3e}")
    # FP32 storage of u limits a steady state to about eps_32 times the
    # slowest relaxation time in steps (H^2/(pi^2 nu) = 73 here): ~5e-6
    assert _rel(ux, pred) < 2e-5
    ctx.destroy()


def test_mass_conservation_and_uniform_fixed_point():
    nx, ny, nz = 12, 10, 9
    ctx = _ctx(nx, ny, nz, False, "fp64", 3.0, 0.3, 0.9, (0, 0, 0))
    ctx.init_uniform((1e-3, -2e-3, 5e-4))
    f0 = ctx.read_populations()
    ctx.step(5)
    f1 = ctx.read_populations()
    assert _rel(f1, f0) < 1e-14
    n, u = random_fields(nx, ny, nz, packing_to_density(0.3, 3.0), 0.05, 0.01, seed=1)
    ctx2 = _ctx(nx, ny, nz, True, "fp32", 3.0, 0.3, 0.9, (1e-4, 0, 0))
    ctx2.init_fields(n, u)
    M0 = ctx2.read_flux()[2]
    ctx2.step(50)
    M1 = ctx2.read_flux()[2]
    assert abs(M1 - M0) < 1e-5 * M0
    ctx.destroy()
    ctx2.destroy()


def test_checkpoint_resume_and_determinism():
    nx, ny, nz = 16, 12, 10
    n, u = random_fields(nx, ny, nz, packing_to_density(0.3, 4.0), 0.05, 0.01, seed=5)
    a = _ctx(nx, ny, nz, True, "fp32", 4.0, 0.3, 1.0, (1e-5, 0, 0))
    a.init_fields(n, u)
    a.step(7)
    snap = a.save_state()
    a.step(9)
    fa = a.read_populations()
    b = _ctx(nx, ny, nz, True, "fp32", 4.0, 0.3, 1.0, (1e-5, 0, 0))
    b.load_state(snap)
    assert b.get_step() == 7
    b.step(9)
    fb = b.read_populations()
    assert np.array_equal(fa, fb)
    c = _ctx(nx, ny, nz, True, "fp32", 4.0, 0.3, 1.0, (1e-5, 0, 0))
    c.init_fields(n, u)
    c.step(16)
    assert np.array_equal(c.read_populations(), fa)
    for x in (a, b, c):
        x.destroy()


def test_new_context_has_no_pending_instability():
    """A context created on reused device memory (the torch allocator hands
    back the block of an unstable context just destroyed) reports nothing
    before its first step."""
    nx, ny, nz = 8, 8, 8
    ctx = _ctx(nx, ny, nz, True, "fp32", 4.0, 0.3, 1.0, (0, 0, 0))
    ctx.init_fields(np.full(nx * ny * nz, packing_to_density(1.2, 4.0)), np.zeros(3 * nx * ny * nz))
    ctx.step(1)
    ctx.destroy()
    ctx2 = _ctx(nx, ny, nz, True, "fp32", 4.0, 0.3, 1.0, (0, 0, 0))
    ctx2.sync()
    ctx2.destroy()


def test_instability_is_reported():
    from paper_1304_7880_amd import wdlb
    nx, ny, nz = 8, 8, 8
    ctx = _ctx(nx, ny, nz, True, "fp32", 4.0, 0.3, 1.0, (0, 0, 0))
    n = np.full(nx * ny * nz, packing_to_density(0.3, 4.0))
    n[100] = np.nan
    ctx.init_fields(n, np.zeros(3 * n.size))
    ctx.step(2)
    with pytest.raises(wdlb.WdlbError) as e:
        ctx.sync()
    assert e.value.status == wdlb.E_UNSTABLE
    # a packing fraction above 1 at the midpoints
    ctx2 = _ctx(nx, ny, nz, True, "fp32", 4.0, 0.3, 1.0, (0, 0, 0))
    ctx2.init_fields(np.full(n.size, packing_to_density(1.2, 4.0)), np.zeros(3 * n.size))
    ctx2.step(1)
    with pytest.raises(wdlb.WdlbError) as e:
        ctx2.sync()
    assert e.value.status == wdlb.E_UNSTABLE
    ctx.destroy()
    ctx2.destroy()


def test_slab64_full_size_first_steps():
    """The 64^3 slit (sigma = 6, eta = 0.35, tau = 0.8, +-1 % noise) at full
    size in FP32 against the oracle for the first steps."""
    w = SLAB_64
    steps = 3
    _say(f"slab64 {steps} steps")
    n, u = initial_fields(w)
    cfg = ref.Config(w.nx, w.ny, w.nz, True, w.sigma, w.tau, w.g)
    st = ref.State.from_fields(cfg, n, u)
    st.step(steps)
    rho_o, u_o, F_o, A_o = st.fields()
    nz_o, ux_o, J_o, _, _ = ref.reduce_fields(cfg, rho_o, u_o)
    ctx = _ctx(w.nx, w.ny, w.nz, True, "fp32", w.sigma, w.eta, w.tau, w.g)
    ctx.init_fields(n, u)
    ctx.step(steps)
    rho_g, u_g, F_g, A_g = ctx.read_fields(with_forces=True)
    _say(f"  rho {_rel(rho_g, rho_o):.2e} u {_rel(u_g, u_o):.2e} F {_rel(F_g, F_o):.2e} A {_rel(A_g, A_o):.2e}")
    assert _rel(rho_g, rho_o) < 1e-5
    assert _rel(u_g, u_o) < 1e-5
    assert _rel(F_g, F_o) < 1e-4
    assert _rel(A_g, A_o) < 1e-4
    nz_g, ux_g = ctx.read_profiles()
    # after 3 steps the plane means are ~1e-3 of the node velocities (the
    # noise-driven flow averages out), so compare them on the node scale
    assert np.abs(ux_g - ux_o).max() < 1e-5 * np.abs(u_o).max()
    assert _rel(nz_g, nz_o) < 1e-6
    ctx.destroy()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_narrow_tiles_compiled_equals_table_driven(prec):
    """A lattice 16 wide takes the 16x16x2 tiles; at sigma = 4 in fp32 it runs
    the compiled shell and ball, which must equal the table-driven kernels on
    the same tile bit for bit."""
    nx, ny, nz, sigma, eta, tau, g = 16, 16, 23, 4.0, 0.25, 1.0, (1e-5, 0.0, 0.0)
    n, u = random_fields(nx, ny, nz, packing_to_density(eta, sigma), 0.05, 0.01, seed=9)
    out = []
    for forced in (False, True):
        ctx = _ctx(nx, ny, nz, True, prec, sigma, eta, tau, g)
        tile, spec = ctx.get_tile()
        assert tile == 5
        if forced:
            ctx.set_tile(5)
            assert ctx.get_tile() == (5, False)
        else:
            assert spec == (prec == "fp32")
        ctx.init_fields(n, u)
        ctx.step(3)
        out.append(ctx.read_fields(with_forces=True))
        ctx.destroy()
    for k, name in enumerate(("rho", "u", "F", "A0")):
        assert np.array_equal(out[0][k], out[1][k]), (name, _rel(out[0][k], out[1][k]))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_graph_replay_equals_eager_steps(prec):
    """wdlb_step replays two-step HIP graphs; several replays, with eager work
    (reads, odd step counts) between them, must give exactly the fields of
    launch-by-launch stepping after every chunk."""
    nx, ny, nz, sigma, eta, tau, g = 40, 20, 13, 4.0, 0.3, 0.9, (1e-4, -3e-5, 0.0)
    n, u = random_fields(nx, ny, nz, packing_to_density(eta, sigma), 0.05, 0.01, seed=21)
    ctxs = []
    for graphs in (True, False):
        ctx = _ctx(nx, ny, nz, True, prec, sigma, eta, tau, g)
        ctx.set_graphs(graphs)
        ctx.init_fields(n, u)
        ctxs.append(ctx)
    for chunk in (4, 5, 1, 8, 2):
        outs = []
        for ctx in ctxs:
            ctx.step(chunk)
            outs.append(ctx.read_fields(with_forces=True))
        for k, name in enumerate(("rho", "u", "F", "A0")):
            assert np.array_equal(outs[0][k], outs[1][k]), (chunk, name)
    assert ctxs[0].get_step() == ctxs[1].get_step() == 20
    for ctx in ctxs:
        ctx.destroy()


@pytest.mark.parametrize("prec", ["fp32"])
def test_kernel_timing_changes_no_result(prec):
    """Timing every kernel with HIP events (wdlb_profile) runs the step launch
    by launch with events between the kernels: the fields must be exactly those
    of an untimed context, and every kernel must report a positive mean time."""
    nx, ny, nz, sigma, eta, tau, g = 64, 16, 18, 6.0, 0.3, 0.9, (1e-4, 0.0, 0.0)
    _say(f"timed vs untimed {nx}x{ny}x{nz} sigma={sigma} {prec}")
    n, u = random_fields(nx, ny, nz, packing_to_density(eta, sigma), 0.05, 0.01, seed=33)
    ctxs = []
    for timed in (True, False):
        ctx = _ctx(nx, ny, nz, True, prec, sigma, eta, tau, g)
        ctx.init_fields(n, u)
        if timed:
            ctx.profile(True)
        ctxs.append(ctx)
    for ctx in ctxs:
        ctx.step(7)
    times = ctxs[0].profile_read()
    ctxs[0].profile(False)
    outs = [ctx.read_fields(with_forces=True) for ctx in ctxs]
    for k, name in enumerate(("rho", "u", "F", "A0")):
        assert np.array_equal(outs[0][k], outs[1][k]), name
    assert set(times) == {"k_moments", "k_density", "k_meanfield", "k_shell", "k_collide", "k_thermal"}
    for name, (ms, count) in times.items():
        if name == "k_thermal":     # not a step kernel
            assert count == 0 and ms == 0, (name, ms, count)
            continue
        assert count == 7 and ms > 0, (name, ms, count)
    for ctx in ctxs:
        ctx.destroy()
