"""GPU energy balance at rest (wdlb_conduction_at_rest) against the FP64
oracle (oracle/conduction.py) on the same seeded n and T.

Bars: FP64: T to 1e-13 of its largest value and the change of T over the
run to 1e-12 of the largest change (sums over the shell in another order;
measured 1.6e-16 and 1.6e-15).  FP32: T is stored in FP32 (6e-8 relative)
and every step re-rounds it, so over 20 steps of dt = 0.05 T carries a few
1e-7 of itself and its change (about a tenth of T) a few 1e-6 of itself
(measured 1.8e-7 and 1.8e-6); the bars are 1e-6 and 2e-5.
"""
import math
import sys

import numpy as np
import pytest

from oracle import conduction, ref
from paper_1304_7880_amd.workloads import packing_to_density, random_fields, random_temperature

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _ctx(nx, ny, nz, walls, prec, sigma, eta=0.3):
    from paper_1304_7880_amd import wdlb
    return wdlb.Context(nx, ny, nz, walls, prec, sigma, eta, 1.0, (0.0, 0.0, 0.0))


CASES = [
    ("walled 21x13x17 sigma=3", (21, 13, 17), True, 3.0, 0.3),
    ("periodic 14x12x16 sigma=4", (14, 12, 16), False, 4.0, 0.25),
    ("walled 36x10x26 sigma=6 (compiled shell, ragged tiles)", (36, 10, 26), True, 6.0, 0.35),
]


@pytest.mark.parametrize("prec,tol_T,tol_dT", [("fp64", 1e-13, 1e-12), ("fp32", 1e-6, 2e-5)])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_conduction_matches_oracle(case, prec, tol_T, tol_dT):
    name, (nx, ny, nz), walls, sigma, eta = case
    _say(f"conduction {name} {prec}")
    n, _ = random_fields(nx, ny, nz, packing_to_density(eta, sigma), 0.05, 0.0, seed=21)
    T = random_temperature(nx, ny, nz, 1.0 / 3.0, 0.1, seed=22)
    cfg = ref.Config(nx, ny, nz, walls, sigma, 1.0)
    omega0, dt, k = 1.0 / 0.8, 0.05, 20
    To = conduction.steps(cfg, n, T, omega0, dt, k)
    ctx = _ctx(nx, ny, nz, walls, prec, sigma, eta)
    Tg = ctx.conduction_at_rest(n, T, omega0, dt, k)
    ctx.destroy()
    eT = float(np.abs(Tg - To).max() / np.abs(To).max())
    edT = float(np.abs((Tg - T) - (To - T)).max() / np.abs(To - T).max())
    _say(f"  T {eT:.2e}  change of T {edT:.2e} (largest change {np.abs(To - T).max():.2e})")
    assert eT < tol_T and edT < tol_dT, (eT, edT)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_uniform_temperature_stays_uniform(prec):
    nx, ny, nz, sigma = 20, 9, 15, 4.0
    n, _ = random_fields(nx, ny, nz, packing_to_density(0.3, sigma), 0.05, 0.0, seed=3)
    ctx = _ctx(nx, ny, nz, True, prec, sigma)
    T = ctx.conduction_at_rest(n, np.full(nx * ny * nz, 0.35), 1.0, 0.1, 5)
    ctx.destroy()
    assert np.all(T == np.float32(0.35) if prec == "fp32" else T == 0.35)


def test_temperature_wave_decays_at_the_oracle_rate():
    """A temperature wave in the sigma = 8 fluid at rest (FP64, 100 steps of
    dt = 0.1): its amplitude falls by (1 + dt r_q) per step, r_q the oracle's
    instantaneous rate of that harmonic, to 1e-8."""
    sigma, eta, L, eps, T0, omega0, dt, k = 8.0, 0.25, 128, 1e-4, 1.0 / 3.0, 1.0, 0.1, 100
    n0 = packing_to_density(eta, sigma)
    cfg = ref.Config(4, 4, L, False, sigma, 1.0)
    z = np.arange(L, dtype=np.float64)
    q = 2 * math.pi / L
    T = np.repeat(T0 * (1 + eps * np.sin(q * z)), 16)
    s = np.repeat(np.sin(q * z), 16)
    amp = lambda f: float((f - T0) @ s) / float(s @ s)
    r_q = float(conduction.rate(cfg, np.full(cfg.N, n0), T, omega0) @ s) / float(s @ s) / amp(T)
    ctx = _ctx(4, 4, L, False, "fp64", sigma, eta)
    Tk = ctx.conduction_at_rest(np.full(cfg.N, n0), T, omega0, dt, k)
    ctx.destroy()
    pred = amp(T) * (1 + dt * r_q) ** k
    _say(f"  amplitude {amp(Tk):.10e} predicted {pred:.10e} (decay {amp(Tk) / amp(T):.6f})")
    assert abs(amp(Tk) / pred - 1) < 1e-8


def test_bad_input_and_state_untouched():
    from paper_1304_7880_amd import wdlb
    nx, ny, nz, sigma = 12, 9, 10, 3.0
    n, u = random_fields(nx, ny, nz, packing_to_density(0.3, sigma), 0.05, 0.01, seed=1)
    T = random_temperature(nx, ny, nz, 1.0 / 3.0, 0.1, seed=2)
    outs = []
    for call in (False, True):
        ctx = _ctx(nx, ny, nz, True, "fp64", sigma)
        ctx.init_fields(n, u)
        ctx.step(3)
        if call:
            ctx.conduction_at_rest(n, T, 1.0, 0.05, 4)
            for bad in ((n, T, 0.0, 0.05, 1), (n, T, 1.0, -1.0, 1), (n, T, 1.0, 0.05, -1), (n * 0, T, 1.0, 0.05, 1),
                        (n, -T, 1.0, 0.05, 1)):
                with pytest.raises(wdlb.WdlbError) as e:
                    ctx.conduction_at_rest(*bad)
                assert e.value.status == wdlb.E_INVAL
            with pytest.raises(wdlb.WdlbError) as e:        # midpoint packing fraction >= 1
                ctx.conduction_at_rest(n * 4.0, T, 1.0, 0.05, 1)
            assert e.value.status == wdlb.E_UNSTABLE
        ctx.step(3)
        outs.append(ctx.read_fields(with_forces=True))
        ctx.destroy()
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("prec,tol_T,tol_dT", [("fp32_local64", 1e-6, 2e-5)])
def test_benchmark_slit_40_steps(prec, tol_T, tol_dT):
    """The benchmark slit's geometry (64^3 between walls, sigma = 6, eta =
    0.35, its seeded density noise) with a seeded 10 % temperature field,
    40 steps of dt = 0.05 at omega0 = 1/0.8, against the oracle run on the
    same input."""
    from paper_1304_7880_amd.workloads import SLAB_64, initial_fields
    w = SLAB_64
    n, _ = initial_fields(w)
    T = random_temperature(w.nx, w.ny, w.nz, 1.0 / 3.0, 0.1, seed=31)
    cfg = ref.Config(w.nx, w.ny, w.nz, True, w.sigma, w.tau)
    _say(f"conduction {w.name} {prec} 40 steps")
    To = conduction.steps(cfg, n, T, 1.0 / w.tau, 0.05, 40)
    ctx = _ctx(w.nx, w.ny, w.nz, True, prec, w.sigma, w.eta)
    Tg = ctx.conduction_at_rest(n, T, 1.0 / w.tau, 0.05, 40)
    ctx.destroy()
    eT = float(np.abs(Tg - To).max() / np.abs(To).max())
    edT = float(np.abs((Tg - T) - (To - T)).max() / np.abs(To - T).max())
    _say(f"  T {eT:.2e}  change of T {edT:.2e} (largest change {np.abs(To - T).max():.2e})")
    assert eT < tol_T and edT < tol_dT, (eT, edT)
