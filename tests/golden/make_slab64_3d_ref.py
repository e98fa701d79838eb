"""Write the 3-D oracle fixture of the seeded 64^3 slit (same input as the GPU run).

    python tests/golden/make_slab64_3d_ref.py [--threads T] [--state PATH]

The 64x64x64 slit pore (H = 64, sigma = 6, eta = 0.35, tau = 0.8,
g_x = 1e-6) starts from the seeded density n0 (1 + 0.01 xi) of the workload
module, u = 0, and is stepped by the FP64 3-D oracle (oracle/wdlb_ref.c
through oracle/ref.py) with nothing else in between.  At each checkpoint the
plane means n(z), u_x(z) and the pore averages J_pore, u_pore and the mass
are stored (oracle reduction, FP64), together with a few single-node values
so that the noisy 3-D state itself is pinned, not only its plane means.

The oracle takes about 3 s per step on 8 host threads here, so the fixture
stops at 2000 steps (about 1.7 viscous times H^2/nu of this slit); the
20000-step end state is covered by the column-oracle fixture.  --state
names a file where the populations are saved after every checkpoint, so an
interrupted run resumes from the last one.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import ref  # noqa: E402
from paper_1304_7880_amd.workloads import SLAB_64, initial_fields  # noqa: E402

CHECKPOINTS = (100, 500, 1000, 2000)
# nodes (x, y, z) whose density and velocity are stored at each checkpoint:
# next to each wall, mid-pore, and at tile-ragged positions
PROBES = ((0, 0, 0), (17, 41, 0), (63, 63, 63), (5, 60, 1), (31, 32, 32), (40, 7, 20), (12, 50, 62))
OUT = os.path.join(HERE, "slab64_3d_oracle.json")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--state", default=None, help="resume file for the populations (npz)")
    args = ap.parse_args()
    if args.threads:
        ref.set_threads(args.threads)
    w = SLAB_64
    cfg = ref.Config(w.nx, w.ny, w.nz, w.walls_z, w.sigma, w.tau, w.g)
    out = {"workload": w.name, "nx": w.nx, "ny": w.ny, "nz": w.nz, "walls_z": w.walls_z, "sigma": w.sigma,
           "eta": w.eta, "tau": w.tau, "g": list(w.g), "noise": w.noise, "seed": w.seed, "probes": PROBES,
           "checkpoints": [],
           "generated_by": "tests/golden/make_slab64_3d_ref.py with oracle/wdlb_ref.c (FP64, 3-D)"}
    step = 0
    if args.state and os.path.exists(args.state):
        z = np.load(args.state)
        st = ref.State(cfg, z["f"].copy())
        step = int(z["step"])
        if os.path.exists(OUT):
            prev = json.load(open(OUT))
            out["checkpoints"] = [c for c in prev["checkpoints"] if c["steps"] <= step]
        print(f"resumed at step {step}", flush=True)
    else:
        n, u = initial_fields(w)
        st = ref.State.from_fields(cfg, n, u)
    N = w.N
    for target in CHECKPOINTS:
        if target <= step:
            continue
        t0 = time.time()
        while step < target:
            k = min(50, target - step)
            st.step(k)
            step += k
            print(f"step {step} ({time.time() - t0:.0f} s into this checkpoint)", flush=True)
        rho, u, _, _ = st.fields()
        n_z, ux_z, J, upore, mass = ref.reduce_fields(cfg, rho, u)
        probes = []
        for (x, y, z) in PROBES:
            i = (z * w.ny + y) * w.nx + x
            probes.append([float(rho[i]), float(u[i]), float(u[N + i]), float(u[2 * N + i])])
        out["checkpoints"].append({"steps": step, "n_z": n_z.tolist(), "ux_z": ux_z.tolist(), "j_pore": J,
                                   "u_pore": upore, "mass": mass, "probe_rho_u": probes})
        with open(OUT + ".tmp", "w") as f:
            json.dump(out, f, indent=0)
        os.replace(OUT + ".tmp", OUT)
        if args.state:
            np.savez(args.state + ".tmp.npz", f=st.f, step=step)
            os.replace(args.state + ".tmp.npz", args.state)
        print(f"checkpoint {step}: J {J:.10e}", flush=True)


if __name__ == "__main__":
    main()
