"""The column-oracle fixtures match the workload definitions and obey the
symmetries of their set-ups (CPU only)."""
import json
import os

import numpy as np

from paper_1304_7880_amd.workloads import BULK_128, SLAB_LARGE_SUB

HERE = os.path.dirname(os.path.abspath(__file__))


def _golden(name):
    with open(os.path.join(HERE, "golden", name)) as f:
        return json.load(f)


def test_slab_fixture_matches_workload_and_mirror_symmetry():
    ref = _golden("slab_large_sub_10000.json")
    w = SLAB_LARGE_SUB
    assert (ref["nx"], ref["ny"], ref["nz"], ref["sigma"], ref["eta"], ref["tau"]) == \
        (w.nx, w.ny, w.nz, w.sigma, w.eta, w.tau)
    assert tuple(ref["g"]) == tuple(w.g) and ref["walls_z"]
    ux, n = np.array(ref["ux_z"]), np.array(ref["n_z"])
    # walls at both ends: profiles symmetric about the mid-plane (to the
    # rounding of 10000 FP64 steps), flow along +x
    assert np.abs(ux - ux[::-1]).max() < 1e-10 * np.abs(ux).max()
    assert np.abs(n - n[::-1]).max() < 1e-10 * n.max()
    assert ux.min() > 0 and ref["j_pore"] > 0
    # mass per plane averages to the initial density
    assert abs(n.mean() - w.n0) < 1e-12 * w.n0


def test_shear_fixture_matches_workload_and_symmetry():
    ref = _golden("bulk128_shear_eta025_1000.json")
    w = BULK_128
    assert (ref["nx"], ref["nz"], ref["sigma"], ref["tau"], ref["shear_amp"]) == \
        (w.nx, w.nz, w.sigma, w.tau, w.shear_amp)
    ux = np.array(ref["ux_z"])
    z = np.arange(w.nz)
    # a decaying sine keeps its shape: u_x(z) = A sin(2 pi z / nz) with 0 < A < a
    s = np.sin(2 * np.pi * z / w.nz)
    A = float(ux @ s / (s @ s))
    assert 0 < A < w.shear_amp
    assert np.abs(ux - A * s).max() < 1e-9 * A


def test_slab64_fixture_matches_workload_and_mass():
    from paper_1304_7880_amd.workloads import SLAB_64, initial_fields
    ref = _golden("slab64_20000.json")
    w = SLAB_64
    assert (ref["nx"], ref["ny"], ref["nz"], ref["sigma"], ref["eta"], ref["tau"], ref["steps"]) == \
        (w.nx, w.ny, w.nz, w.sigma, w.eta, w.tau, w.steps)
    n, _ = initial_fields(w)
    # the column started from the plane means of the seeded density: same mass
    assert abs(np.sum(ref["n_z"]) * w.nx * w.ny - n.sum()) < 1e-10 * n.sum()
    assert ref["j_pore"] > 0
