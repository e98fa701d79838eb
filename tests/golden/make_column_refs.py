"""Write the column-oracle fixtures used by the full-size GPU parity tests.

    python tests/golden/make_column_refs.py

Every stored value comes from oracle/column1d.py (the FP64 1-D z-column
oracle, exact for states that do not depend on x and y; pinned against the
3-D oracle by tests/test_oracle_pins.py).  Inputs come from the seeded
workload module only.  The fixtures are small JSON files:

  slab_large_sub_10000.json  64x64x256 slit, sigma=10, eta=0.40, tau=0.7,
                             g_x=5e-7, uniform start, 10000 steps
  bulk128_shear_eta025_1000.json
                             128^3 periodic cube, sigma=8, eta=0.25, tau=1,
                             u_x = 1e-4 sin(2 pi z/128), 1000 steps
  bulk128_shear_eta005_5000.json, bulk128_shear_eta035_5000.json
                             the same cube at eta = 0.05 and 0.35 over the
                             full 5000 steps of the viscosity measurement
  slab64_20000.json          the 64^3 slit (sigma=6, eta=0.35, tau=0.8,
                             g_x=1e-6) after its full 20000 steps, as the
                             x,y-homogeneous slit started from the plane
                             means of the seeded density: after ~17 viscous times the +-1 % noise
                             of the 3-D start has decayed
"""
import json
import math
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.column1d import Column  # noqa: E402
from paper_1304_7880_amd.workloads import BULK_128, SLAB_64, SLAB_LARGE_SUB, initial_fields  # noqa: E402


def run(w, steps, n_start=None, amp_every=0):
    """The column oracle over `steps` steps; with amp_every, also the shear
    amplitude A(t) = (2/nz) sum_z u_x(z) sin(2 pi z/nz) every amp_every steps
    (from t = 0)."""
    col = Column(w.nz, sigma=w.sigma, tau=w.tau, g=w.g, walls=w.walls_z)
    z = np.arange(w.nz, dtype=np.float64)
    u = np.zeros((3, w.nz))
    u[0] = w.shear_amp * np.sin(2.0 * math.pi * z / w.nz)
    col.init(np.full(w.nz, w.n0 if n_start is None else n_start), u)
    amp = []
    if amp_every:
        s = np.sin(2.0 * math.pi * z / w.nz)
        for t in range(0, steps + 1, amp_every):
            if t:
                col.step(amp_every)
            amp.append(float(2.0 / w.nz * (col.fields()[1][0] * s).sum()))
    else:
        col.step(steps)
    rho, ux, J, upore, mass = col.reduce()
    out = {"workload": w.name, "nx": w.nx, "ny": w.ny, "nz": w.nz, "walls_z": w.walls_z, "sigma": w.sigma,
           "eta": w.eta, "tau": w.tau, "g": list(w.g), "shear_amp": w.shear_amp, "steps": steps,
           "n_z": rho.tolist(), "ux_z": ux.tolist(), "j_pore": J, "u_pore": upore,
           "generated_by": "tests/golden/make_column_refs.py with oracle/column1d.py (FP64)"}
    if amp_every:
        out["amp_every"] = amp_every
        out["amp"] = amp
    return out


def main():
    cases = [("slab_large_sub_10000.json", SLAB_LARGE_SUB, 10000, 0),
             ("bulk128_shear_eta025_1000.json", BULK_128.with_(eta=0.25), 1000, 0),
             ("bulk128_shear_eta005_5000.json", BULK_128.with_(eta=0.05), 5000, 10),
             ("bulk128_shear_eta035_5000.json", BULK_128.with_(eta=0.35), 5000, 10)]
    for name, w, steps, every in cases:
        out = run(w, steps, amp_every=every)
        with open(os.path.join(HERE, name), "w") as f:
            json.dump(out, f, indent=0)
        print(name, "J", out["j_pore"], flush=True)
    # the 64^3 slit: plane means of the seeded start give the column's start
    w = SLAB_64
    n, _ = initial_fields(w)
    n_z = n.reshape(w.nz, w.ny * w.nx).mean(axis=1)
    out = run(w, w.steps, n_start=n_z)
    out["start"] = "plane means of the seeded 3-D density"
    with open(os.path.join(HERE, "slab64_20000.json"), "w") as f:
        json.dump(out, f, indent=0)
    print("slab64_20000.json", "J", out["j_pore"], flush=True)


if __name__ == "__main__":
    main()
