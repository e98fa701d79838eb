"""Full-size GPU runs against the FP64 column oracle (fixtures in tests/golden/,
written by tests/golden/make_column_refs.py from oracle/column1d.py).

The 64x64x256 slit at sigma = 10 (the sub-run of the 512x512x256 slab: the
state does not depend on x and y, so the sub-run has the full run's
z-profile) runs its full 10000 steps in FP32 and in the BF16 mode; the
128^3 shear wave at sigma = 8 runs 1000 steps in FP32.  Bars: FP32 1e-5 and
BF16 1e-3 relative on u_x(z) (relative to its largest value) and on the
pore-averaged flux.
"""
import json
import os
import sys

import numpy as np
import pytest

from paper_1304_7880_amd.workloads import BULK_128, SLAB_LARGE_SUB, initial_fields

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def _golden(name):
    with open(os.path.join(HERE, "golden", name)) as f:
        return json.load(f)


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-5), ("bf16", 1e-3)])
def test_large_slab_subrun_full_length(prec, tol):
    from paper_1304_7880_amd import wdlb
    ref = _golden("slab_large_sub_10000.json")
    w = SLAB_LARGE_SUB
    assert (w.nx, w.ny, w.nz, w.sigma, w.eta, w.tau) == (ref["nx"], ref["ny"], ref["nz"], ref["sigma"], ref["eta"],
                                                          ref["tau"])
    _say(f"slab {w.name} {prec} {ref['steps']} steps")
    ctx = wdlb.Context(w.nx, w.ny, w.nz, True, prec, w.sigma, w.eta, w.tau, w.g)
    ctx.init_uniform((0.0, 0.0, 0.0))
    ctx.step(ref["steps"])
    ctx.sync()
    n_g, ux_g = ctx.read_profiles()
    J_g, _, _ = ctx.read_flux()
    ctx.destroy()
    ux_o, n_o, J_o = np.array(ref["ux_z"]), np.array(ref["n_z"]), ref["j_pore"]
    e_u = float(np.abs(ux_g - ux_o).max() / np.abs(ux_o).max())
    e_J = abs(J_g - J_o) / abs(J_o)
    e_n = float(np.abs(n_g - n_o).max() / np.abs(n_o).max())
    _say(f"  u_x(z) rel {e_u:.3e}  J rel {e_J:.3e}  n(z) rel {e_n:.3e}")
    assert e_u < tol
    assert e_J < tol
    assert e_n < tol


def test_bulk_shear_wave_full_size():
    from paper_1304_7880_amd import wdlb
    ref = _golden("bulk128_shear_eta025_1000.json")
    w = BULK_128.with_(eta=ref["eta"])
    _say(f"bulk {w.name} eta={w.eta} fp32 {ref['steps']} steps")
    ctx = wdlb.Context(w.nx, w.ny, w.nz, False, "fp32", w.sigma, w.eta, w.tau, w.g)
    n, u = initial_fields(w)
    ctx.init_fields(n, u)
    ctx.step(ref["steps"])
    ctx.sync()
    n_g, ux_g = ctx.read_profiles()
    ctx.destroy()
    ux_o, n_o = np.array(ref["ux_z"]), np.array(ref["n_z"])
    e_u = float(np.abs(ux_g - ux_o).max() / np.abs(ux_o).max())
    e_n = float(np.abs(n_g - n_o).max() / np.abs(n_o).max())
    _say(f"  u_x(z) rel {e_u:.3e}  n(z) rel {e_n:.3e}")
    assert e_u < 1e-5
    assert e_n < 1e-5


def test_slab64_full_length_against_column_oracle():
    """The benchmark slit (64^3, sigma = 6, seeded +-1 % density noise) after
    its full 20000 steps: the noise has decayed over ~17 viscous times and the
    flow is that of the x,y-homogeneous slit started from the plane means of
    the same density (column oracle).  Bar: 1e-5 on u_x(z) and the flux."""
    from paper_1304_7880_amd import wdlb
    from paper_1304_7880_amd.workloads import SLAB_64
    ref = _golden("slab64_20000.json")
    w = SLAB_64
    _say(f"slab {w.name} fp32 {ref['steps']} steps")
    ctx = wdlb.Context(w.nx, w.ny, w.nz, True, "fp32", w.sigma, w.eta, w.tau, w.g)
    n, u = initial_fields(w)
    ctx.init_fields(n, u)
    ctx.step(ref["steps"])
    ctx.sync()
    n_g, ux_g = ctx.read_profiles()
    J_g, _, _ = ctx.read_flux()
    ctx.destroy()
    ux_o, J_o = np.array(ref["ux_z"]), ref["j_pore"]
    e_u = float(np.abs(ux_g - ux_o).max() / np.abs(ux_o).max())
    e_J = abs(J_g - J_o) / abs(J_o)
    _say(f"  u_x(z) rel {e_u:.3e}  J rel {e_J:.3e}")
    assert e_u < 1e-5
    assert e_J < 1e-5
