"""Benchmark of the WDLB time step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--serving N]

Workload (the headline): the 512x512x256 slit pore (H = 256) with
sigma = 10, eta = 0.40, tau = 0.7, g_x = 5e-7, uniform start, populations
stored in FP32 with the local kernels (pull, moments, collision) in FP64
arithmetic, the stencil sums in FP32 and the reductions in FP64 (the mode
that meets the 1e-5 accuracy bar).  Inputs are synthetic and resident on
the device before the timed region starts.

A step is one full WDLB step: moments, weighted density and contact values,
mean-field shell sum, viscous/SMDB shell sum, and the forced collision with
the stream.  value = fluid nodes x steps / device time of the timed steps
(MLUPS).  The dominant kernel (the viscous/SMDB shell sum) is timed with HIP
events on the library's stream during the same run and priced against the
chip's FP32 vector peak; HBM bytes per launch come from the rocprofv3
counter summary in profiles/ while it matches the device sources.  Beside
the headline: the same slab in the other storage modes, the 64x64x64 slit,
the serving trace through the batched server and the plain loop, and the
FP64 CPU oracle timed on a bounded sample on the host.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_VECTOR_TFLOPS = 157.3     # MI355X FP32 vector peak (256 CU x 4 SIMD x 64 flop/clk x 2.4 GHz)
PEAK_FP64_VECTOR_TFLOPS = 78.6      # MI355X FP64 vector peak
PEAK_HBM_GBS = 8000.0


def shell_size(sigma: float) -> int:
    R = int(math.ceil(sigma + 0.5)) + 1
    lo, hi = (sigma - 0.5) ** 2, (sigma + 0.5) ** 2
    return sum(1 for x in range(-R, R + 1) for y in range(-R, R + 1) for z in range(-R, R + 1)
               if lo <= x * x + y * y + z * z < hi)


def shell_flops_per_node(sigma: float) -> float:
    """Algorithmic FP32 flops of the viscous/SMDB contact-shell sum per node:
    36 per shell offset (du: 3, G: 1, W = G du: 3, k (k.W): 11, sym(k x W): 18)."""
    return 36.0 * shell_size(sigma)


def device_source_hash() -> str:
    """sha256 (16 hex) of the device sources with comments and blank space
    removed, to tie counter data to the code they were taken on."""
    import hashlib
    import re
    h = hashlib.sha256()
    for name in ("d3q19.hpp", "shell.hpp", "kernels.hpp"):
        src = open(os.path.join(ROOT, "paper_1304_7880_amd", "csrc", name)).read()
        src = re.sub(r"//[^\n]*", "", src)
        h.update(" ".join(src.split()).encode())
    return h.hexdigest()[:16]


PROFILES = {"slab64": os.path.join(ROOT, "profiles", "step_kernels_slab64.md"),
            "slab512": os.path.join(ROOT, "profiles", "step_kernels_slab512x512x256.md")}


def profile_figures(profile):
    """(calibrated HBM bytes per launch, rocprofv3 mean duration in ms) of each
    step kernel, from the rocprofv3 runs summarised in the profile file; both
    empty if the device code changed since they were taken."""
    if not os.path.exists(profile):
        return {}, {}
    kv, traffic, dur = {}, {}, {}
    for line in open(profile):
        if ":" not in line:
            continue
        key, val = line.split(":", 1)
        key, val = key.strip(), val.strip()
        if key == "device_source_sha256_16":
            kv[key] = val
        elif key.startswith("traffic_bytes_per_launch "):
            traffic[key.split()[1]] = float(val)
        elif key.startswith("rocprof_mean_ms "):
            dur[key.split()[1]] = float(val)
    if kv.get("device_source_sha256_16") != device_source_hash():
        return {}, {}
    return traffic, dur


def cpu_baseline(w, budget_s: float = 12.0, single_nxy: int = 16):
    """The FP64 oracle on a bounded sample of the workload, from its initial
    state: whole steps of the x,y sub-lattice w (all host threads, OpenMP over
    z-planes) until budget_s has elapsed, then one step of a single_nxy^2 x nz
    column of it on one thread.  Same sigma and nz, so the work per node is
    that of the full workload."""
    from oracle import ref
    from paper_1304_7880_amd.workloads import initial_fields
    n, u = initial_fields(w)
    cfg = ref.Config(w.nx, w.ny, w.nz, w.walls_z, w.sigma, w.tau, w.g)
    st = ref.State.from_fields(cfg, n, u)
    steps, t0 = 0, time.perf_counter()
    while True:
        st.step(1)
        steps += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    cores = ref.threads()
    del st
    ws = w.with_(nx=single_nxy, ny=single_nxy)
    n1, u1 = initial_fields(ws)
    cfg1 = ref.Config(ws.nx, ws.ny, ws.nz, ws.walls_z, ws.sigma, ws.tau, ws.g)
    st1 = ref.State.from_fields(cfg1, n1, u1)
    ref.set_threads(1)
    t1 = time.perf_counter()
    st1.step(1)
    dt1 = time.perf_counter() - t1
    ref.set_threads(cores)
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        pass
    return {"value": w.N * steps / dt / 1e6, "unit": "MLUPS", "cores": cores, "kind": "oracle",
            "sample": f"{steps} step(s) of the {w.nx}x{w.ny}x{w.nz} sub-lattice (sigma={w.sigma:g}: the same work "
                      f"per node as the full slab) from the same initial state, {dt:.1f} s, OpenMP over z-planes",
            "single_thread_value": ws.N / dt1 / 1e6,
            "single_thread_sample": f"1 step of a {ws.nx}x{ws.ny}x{ws.nz} column, {dt1:.1f} s",
            "cpu_model": model, "host_cpus": os.cpu_count()}


def _percentile(v, q):
    import numpy as np
    return float(np.percentile(np.asarray(v, dtype=np.float64), q)) if len(v) else None


def _lat_stats(lat, span, n_ok):
    """Throughput over the converged requests and their latency percentiles."""
    return {"solves_per_s": round(n_ok / span, 3) if span > 0 else None, "makespan_s": round(span, 3),
            "p50_latency_s": None if not lat else round(_percentile(lat, 50), 4),
            "p99_latency_s": None if not lat else round(_percentile(lat, 99), 4)}


def serving_bench(n_req, planes, max_steps, plain=True):
    """Replay the first n_req requests of the seeded serving trace (Poisson
    arrivals at 200/s, H in 8..96, eta in [0.05, 0.45], g_x log-uniform in
    [1e-7, 1e-5], 16x16 in x,y, sigma = 4, tau = 1; steady when the pore flux
    changes by < 1e-8 over 100 steps) in real time through the batched server
    and through the plain loop (one single-slit context at a time, FIFO, the
    same kernels and the same steady-state test).  Solves/s and the latency
    percentiles count the requests that reached steady state; requests that
    went unstable or hit the step cap are counted, with their latencies,
    separately."""
    from paper_1304_7880_amd import wdlb
    from paper_1304_7880_amd.workloads import serving_requests

    reqs = serving_requests(n=n_req)
    tol, every, sigma = 1e-8, 100, 4.0

    srv = wdlb.Server(16, 16, planes, sigma=sigma, tol=tol, check_every=every, max_steps=max_steps)
    t0 = time.perf_counter()
    ids = []
    for r in reqs:
        dt = r.arrival_s - (time.perf_counter() - t0)
        if dt > 0:
            time.sleep(dt)
        ids.append(srv.submit(r.H, r.eta, r.gx, r.tau))
    srv.drain()
    res_b = [srv.poll(i, H=r.H) for i, r in zip(ids, reqs)]
    st = srv.stats()
    srv.destroy()
    print(f"serving: batched server done ({n_req} requests)", file=sys.stderr, flush=True)

    def split(statuses, lats):
        groups = {"converged": wdlb.OK, "unstable": wdlb.E_UNSTABLE, "not_converged": wdlb.E_NOT_CONVERGED}
        out = {}
        for name, code in groups.items():
            lat = [l for sc, l in zip(statuses, lats) if sc == code]
            out[name] = len(lat)
            if name != "converged":
                out[f"{name}_p50_latency_s"] = None if not lat else round(_percentile(lat, 50), 4)
        return out

    stat_b = [res.status for res, _ in res_b]
    lat_b = [res.t_done - res.t_submit for res, _ in res_b]
    ok_lat_b = [l for sc, l in zip(stat_b, lat_b) if sc == wdlb.OK]
    span_b = max(res.t_done for res, _ in res_b) - min(res.t_submit for res, _ in res_b)
    batched = _lat_stats(ok_lat_b, span_b, len(ok_lat_b))
    batched.update(split(stat_b, lat_b))
    batched.update(max_resident=st["max_resident"],
                   mlups=round(st["node_updates"] / max(st["busy_s"], 1e-9) / 1e6, 1))
    out = {"requests": n_req, "server_planes": planes, "precision": "fp32 storage, fp64 local arithmetic",
           "counted": "solves/s and latency percentiles over the requests that reached steady state",
           "batched": batched}
    if not plain:
        return out

    t0 = time.perf_counter()
    lat_p, stat_p, same, t_last = [], [], True, 0.0
    for r, (rb, uxb) in zip(reqs, res_b):
        now = time.perf_counter() - t0
        if now < r.arrival_s:
            time.sleep(r.arrival_s - now)
        ctx = wdlb.Context(16, 16, r.H, True, "fp32_local64", sigma, r.eta, r.tau, (r.gx, 0.0, 0.0))
        ctx.init_uniform((0.0, 0.0, 0.0))
        steps, Jprev, status, J = 0, None, wdlb.OK, 0.0
        while True:
            ctx.step(every)
            steps += every
            try:
                J, _, _ = ctx.read_flux()
            except wdlb.WdlbError as e:
                status = e.status
                break
            if Jprev is not None and abs(J - Jprev) <= tol * abs(J):
                break
            if steps >= max_steps:
                status = wdlb.E_NOT_CONVERGED
                break
            Jprev = J
        ctx.destroy()
        t_last = time.perf_counter() - t0
        lat_p.append(t_last - r.arrival_s)
        stat_p.append(status)
        if len(lat_p) % 32 == 0:
            print(f"serving: plain loop {len(lat_p)}/{n_req}", file=sys.stderr, flush=True)
        same = same and status == rb.status and steps == rb.steps and (status != wdlb.OK or J == rb.j_pore)
    span_p = t_last - reqs[0].arrival_s
    ok_lat_p = [l for sc, l in zip(stat_p, lat_p) if sc == wdlb.OK]
    out["plain"] = _lat_stats(ok_lat_p, span_p, len(ok_lat_p))
    out["plain"].update(split(stat_p, lat_p))
    if out["plain"]["solves_per_s"] and out["batched"]["solves_per_s"]:
        out["speedup_solves_per_s"] = round(out["batched"]["solves_per_s"] / out["plain"]["solves_per_s"], 2)
    out["results_identical_batched_vs_plain"] = bool(same)
    return out


def transport_bench(parts=("bulk", "sound", "slit")):
    """Transport experiments on the hot path, each part optional: the bulk
    shear-wave viscosity of the 128^3 periodic box at sigma = 8 for each
    packing fraction, with and without the SMDB cross-over term (5000 steps,
    amplitude read every 10); the sound speed and longitudinal viscosity of a
    standing density wave in the same box (2000 steps, read every 2); and the
    effective viscosity of 16x16xH slits at sigma = 8 for eta = 0.11 and 0.32
    (run to steady state); and the collisional thermal conductivity and the
    heat-flux correction coefficient of the sigma = 8 fluid from its thermal
    fields at two long temperature waves; and the heat mode of the coupled
    thermal flow (a temperature wave at constant pressure, L = 128) against
    lambda q^2 / (n c_p)."""
    from paper_1304_7880_amd import transport, wdlb
    from paper_1304_7880_amd.workloads import BULK_128, BULK_ETAS
    HEAT_ETAS = BULK_ETAS
    w = BULK_128
    bulk = []
    for eta in (BULK_ETAS if "bulk" in parts else ()):
        row = {"eta": eta}
        for smdb in (True, False):
            key = "smdb" if smdb else "dsb"
            try:
                r = transport.shear_wave_viscosity(eta, sigma=w.sigma, n=w.nz, steps=w.steps, every=10, tau=w.tau,
                                                   amp=w.shear_amp, smdb=smdb)
            except wdlb.WdlbError as e:  # the uniform state itself is unstable at this packing
                row[f"nu_{key}"] = None
                row[f"status_{key}"] = str(e).split(":")[0]
                continue
            row[f"nu_{key}"] = round(r.nu, 6)
            row[f"seconds_{key}"] = round(r.seconds, 2)
            row[f"mlups_{key}"] = round(w.N * w.steps / r.seconds / 1e6, 1)
        bulk.append(row)
        print(json.dumps({"bulk_row": row}), file=sys.stderr, flush=True)
    # longitudinal waves in the same box: c^2 against Carnahan-Starling, and the
    # bulk viscosity nu_L - (4/3) nu_shear (both with the SMDB term)
    sound = []
    for eta in (BULK_ETAS if "sound" in parts else ()):
        row_b = next((b for b in bulk if b["eta"] == eta), {})
        row = {"eta": eta, "c2_cs": round(transport.carnahan_starling_c2(eta), 6)}
        try:
            r = transport.longitudinal_wave(eta, sigma=w.sigma, n=w.nz, steps=2000, every=2, tau=w.tau, eps=1e-3)
        except wdlb.WdlbError as e:
            row["status"] = str(e).split(":")[0]
            sound.append(row)
            continue
        row.update(c2=round(r.c2, 6), nu_long=round(r.nu_long, 6), seconds=round(r.seconds, 2))
        if row_b.get("nu_smdb") is not None:
            row["nu_bulk"] = round(r.nu_long - 4.0 / 3.0 * row_b["nu_smdb"], 6)
        sound.append(row)
        print(json.dumps({"sound_row": row}), file=sys.stderr, flush=True)
    thermal = []
    for eta in (BULK_ETAS if "thermal" in parts else ()):
        r = transport.thermal_conductivity(eta, sigma=w.sigma)
        dcy = transport.thermal_conduction_decay(eta, sigma=w.sigma, tau=w.tau)
        row = {"eta": eta, "lam_decay": round(dcy.lam, 8), "lam_decay_over_sec4": round(dcy.lam / dcy.lam_sec4, 6),
               "decay_200_steps": [round(v, 6) for v in dcy.decay],
               "lam_coll": round(r.lam_coll, 8), "lam_coll_over_sec4": round(r.lam_coll / r.lam_coll_sec4, 6),
               "b_coef": round(r.b_coef, 8), "b_coef_over_sec4": round(r.b_coef / r.b_coef_sec4, 6),
               "shell_r1": round(r.shell_r1, 6), "shell_r2": round(r.shell_r2, 6),
               "lam_total_tau1_qexplicit": round(r.lam_total(1.0, 2.0), 8),
               "lam_total_tau1_c1exp22": round(r.lam_total(1.0, 4.0), 8)}
        thermal.append(row)
        print(json.dumps({"thermal_row": row}), file=sys.stderr, flush=True)
    heat = []
    for eta in (HEAT_ETAS if "heatmode" in parts else ()):
        try:
            h = transport.heat_mode(eta, sigma=8.0)
            row = {"eta": eta, "rate": h.rate, "rate_rest_over_gamma": h.rate_rest / h.gamma, "ratio": h.ratio,
                   "gamma": h.gamma, "lam_eff": h.lam_eff}
        except wdlb.WdlbError as e:
            row = {"eta": eta, "error": str(e)}
        heat.append(row)
        print(json.dumps({"heat_row": row}), file=sys.stderr, flush=True)
    slits = []
    for eta in ((0.11, 0.32) if "slit" in parts else ()):
        for H in (16, 32, 64, 128, 200):
            r = transport.slit_effective_viscosity(H, eta, sigma=8.0, g=1e-6, nxy=16, tau=1.0, tol=1e-8,
                                                   max_steps=400000)
            row = {"eta": eta, "H": H, "nu_eff": round(r.nu_eff, 6), "steps": r.steps, "converged": r.converged}
            slits.append(row)
            print(json.dumps({"slit_row": row}), file=sys.stderr, flush=True)
    return {"metric": "kinematic viscosity (shear-wave decay; slit nu_eff = g H^2 / (12 u_pore)), squared "
                      "sound speed (density-wave oscillation) and collisional thermal conductivity (thermal fields "
                      "of a temperature wave, fp64)",
            "unit": "lattice units", "dtype": "fp32", "data": "synthetic",
            "config": {"workload": f"{w.name}, shear 5000 steps, sound 2000 steps; slits 16x16xH, sigma=8, tau=1, "
                                   "g_x=1e-6"},
            "bulk": bulk, "sound": sound, "slit": slits, "thermal": thermal, "heatmode": heat}


SHELL_OPS_PER_OFFSET = 26.0   # VALU operations per shell offset counted for the method's shell sums

# Thermal fields (Q, B_i, F^T of Sec. 3) per shell offset: dT, G = gamma rho,
# D = G dT, k_i D (3 FMA), sum D, du (3), V = G du (3), k.V (3 FMA):
# 16 operations, 22 flops (an FMA counted as 2).
THERMAL_OPS_PER_OFFSET = 16.0
THERMAL_FLOPS_PER_OFFSET = 22.0
# the thermal fields at u = 0 (the coupled thermal flow's pass): G = gamma rho, dT, D = G dT,
# k_i D (3 FMA) and sum D -- the velocity terms (du, G du, k.V: 9) dropped
THERMAL_NOU_OPS_PER_OFFSET = 7.0


def thermal_bench(w, prec, reps=5):
    """The thermal fields at seeded random n, u, T on workload w: k_thermal's
    mean duration by HIP events over reps calls and its rate against the FP32
    vector peak; the whole device-resident call (wdlb_thermal_fields_device:
    pads, contact values, thermal kernel); and the host-inclusive time of one
    call from host arrays (the fields cross PCIe both ways)."""
    from paper_1304_7880_amd import wdlb
    from paper_1304_7880_amd.workloads import random_fields, random_temperature
    n, u = random_fields(w.nx, w.ny, w.nz, w.n0, 0.05, 0.01, seed=1)
    T = random_temperature(w.nx, w.ny, w.nz, 1.0 / 3.0, 0.1, seed=2)
    ctx = wdlb.Context(w.nx, w.ny, w.nz, w.walls_z, prec, w.sigma, w.eta, w.tau, w.g)
    ctx.thermal_fields(n, u, T)
    ctx.profile(True, kernels=["k_thermal"])
    t0 = time.perf_counter()
    for _ in range(reps):
        ctx.thermal_fields(n, u, T)
    call_s = (time.perf_counter() - t0) / reps
    ms, cnt = ctx.profile_read()["k_thermal"]
    ctx.profile(False)
    # the device-resident call (fields already in HBM): pads, contact values
    # and the thermal kernel, timed by HIP events on the context's stream
    import torch
    dt = torch.float64 if prec == "fp64" else torch.float32
    dn, du, dT = (torch.tensor(a, dtype=dt, device="cuda") for a in (n, u, T))
    outs = [torch.empty(k * w.N, dtype=dt, device="cuda") for k in (1, 3, 3)]
    ctx.thermal_fields_device(dn, du, dT, *outs)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(ctx.stream)
    for _ in range(reps):
        ctx.thermal_fields_device(dn, du, dT, *outs)
    e1.record(ctx.stream)
    ctx.sync()
    dev_ms = e0.elapsed_time(e1) / reps
    tile, spec = ctx.get_tile()
    ctx.destroy()
    del dn, du, dT, outs
    k_s = ms / cnt * 1e-3
    nS = shell_size(w.sigma)
    ops = THERMAL_OPS_PER_OFFSET * nS * w.N
    flops = THERMAL_FLOPS_PER_OFFSET * nS * w.N
    peak = PEAK_FP64_VECTOR_TFLOPS if prec == "fp64" else PEAK_FP32_VECTOR_TFLOPS
    return {"workload": w.name, "precision": PRECISION_LABEL[prec],
            "kernel": thermal_kernel_name(spec, prec, w.sigma, False),
            "avg_kernel_ms": round(ms / cnt, 5), "launches": cnt,
            "call_ms_device": round(dev_ms, 3),
            "call_ms_host_inclusive": round(call_s * 1e3, 2),
            "roofline": {"bound": "alu", "achieved": round(ops / k_s / 1e12, 3), "peak": peak,
                         "unit": "TFLOP/s", "frac": round(ops / k_s / 1e12 / peak, 4),
                         "count": f"{THERMAL_OPS_PER_OFFSET:g} operations per shell offset x {nS} offsets x "
                                  f"{w.N} nodes",
                         "achieved_22flop": round(flops / k_s / 1e12, 3),
                         "frac_22flop": round(flops / k_s / 1e12 / peak, 4)}}


def thermal_kernel_name(spec, prec, sigma, at_rest):
    """The thermal-sums kernel the library runs: compiled for the shell
    (FP32 at a compiled sigma, FP64 at sigma = 10), at u = 0 its variant with
    all three rings in LDS, else the table-driven ring kernel."""
    if not (spec and (prec != "fp64" or sigma == 10.0)):
        return "k_thermal_r"
    return "k_thermal_s0" if at_rest else "k_thermal_s"


def thermal_flow_bench(w, prec, steps=3, warmup=1, nsub=4):
    """The coupled thermal flow on workload w's lattice in storage mode prec
    (fp64, fp32 or fp32_local64) from its seeded fields and a temperature
    wave across the slit, T = kT (1 + 0.05 cos(2 pi z / nz)): ms per step by
    HIP events on the context's stream over `steps` steps after `warmup`,
    then the library's per-kernel event timing over the same number of steps
    (the step's kernels and the thermal-field kernel; the thermal-flow
    kernels of their own are the rest), and the roofline of the two shell
    kernels against the vector peak of the storage arithmetic (the thermal
    kernel runs its u = 0 variant here: 7 operations per shell offset)."""
    import numpy as np
    import torch
    from paper_1304_7880_amd import wdlb
    from paper_1304_7880_amd.workloads import initial_fields
    n, u = initial_fields(w)
    z = np.repeat(np.arange(w.nz, dtype=np.float64), w.nx * w.ny)
    T = (1.0 / 3.0) * (1.0 + 0.05 * np.cos(2.0 * np.pi * z / w.nz))
    del z
    ctx = wdlb.Context(w.nx, w.ny, w.nz, w.walls_z, prec, w.sigma, w.eta, w.tau, w.g)
    ctx.init_thermal(n, u, T)
    del n, u
    ctx.step_thermal(warmup, nsub)
    ctx.sync()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(ctx.stream)
    ctx.step_thermal(steps, nsub)
    e1.record(ctx.stream)
    ctx.sync()
    ms = e0.elapsed_time(e1) / steps
    ctx.profile(True)
    ctx.step_thermal(steps, nsub)
    prof = {k: v for k, v in ctx.profile_read().items() if v[1]}
    kst = {k: v[0] / steps for k, v in prof.items()}          # ms per step
    kavg = {k: v[0] / v[1] for k, v in prof.items()}          # ms per launch
    ctx.profile(False)
    tile, spec = ctx.get_tile()
    Tn = ctx.read_temperature()
    ctx.destroy()
    nS = shell_size(w.sigma)
    peak = PEAK_FP64_VECTOR_TFLOPS if prec == "fp64" else PEAK_FP32_VECTOR_TFLOPS
    names = {"k_shell": "k_shell_s" if spec else "k_shell",
             "k_thermal": thermal_kernel_name(spec, prec, w.sigma, True)}
    out = {"workload": w.name, "precision": PRECISION_LABEL[prec], "nsub": nsub, "steps": steps,
           "ms_per_step": round(ms, 3), "mlups": round(w.N / (ms * 1e-3) / 1e6, 2),
           "kernels_ms_per_step": {k: round(v, 4) for k, v in kst.items()},
           "other_kernels_ms_per_step": round(ms - sum(kst.values()), 3),
           "T_range": [float(Tn.min()), float(Tn.max())]}
    for k, ops in (("k_shell", SHELL_OPS_PER_OFFSET), ("k_thermal", THERMAL_NOU_OPS_PER_OFFSET)):
        if k in kavg:
            a = ops * nS * w.N / (kavg[k] * 1e-3) / 1e12
            out[f"roofline_{k}"] = {"kernel": names[k], "bound": "alu", "achieved": round(a, 3), "peak": peak,
                                    "unit": "TFLOP/s", "frac": round(a / peak, 4),
                                    "count": f"{ops:g} operations per shell offset x {nS} offsets x {w.N} nodes"}
    return out


def timed_run(w, precision, steps, warmup, stream, init_fields=None):
    """Warm up, then time exactly `steps` steps of workload w between
    synchronisations, with HIP events on the library's stream around every
    launch of the viscous/SMDB shell kernel; then a short per-kernel breakdown
    after the timed region."""
    import torch
    from paper_1304_7880_amd import wdlb
    from paper_1304_7880_amd.workloads import initial_fields
    ctx = wdlb.Context(w.nx, w.ny, w.nz, w.walls_z, precision, w.sigma, w.eta, w.tau, w.g, stream=stream)
    if w.noise or w.shear_amp:
        n, u = initial_fields(w)
        ctx.init_fields(n, u)
    else:  # a uniform fluid at rest: no host fields to build and copy
        ctx.init_uniform((0.0, 0.0, 0.0))
    ctx.step(warmup)
    ctx.sync()
    shell_name = "k_shell_s" if ctx.get_tile()[1] else "k_shell"
    ctx.profile(True, kernels=["k_shell"])
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    ctx.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.sync()
    dev_ms = e0.elapsed_time(e1)
    k_ms, k_n = ctx.profile_read()["k_shell"]
    ctx.profile(False)
    nb = min(steps, 20)
    ctx.profile(True)
    ctx.step(nb)
    kstats = ctx.profile_read()
    ctx.profile(False)
    J, upore, mass = ctx.read_flux()
    ctx.destroy()
    del ctx
    torch.cuda.empty_cache()
    return {"dev_ms": dev_ms, "wall_s": wall, "ms_per_step": dev_ms / steps,
            "mlups": w.N * steps / (dev_ms * 1e-3) / 1e6, "shell_name": shell_name,
            "shell_avg_ms": k_ms / k_n, "kernels_ms_per_step": {k: v[0] / v[1] for k, v in kstats.items() if v[1]},
            "pore_flux": J}


PRECISION_LABEL = {
    "fp32_local64": "fp32 storage; fp32 stencil sums (weighted density, contact values, shell sums); fp64 arithmetic "
                    "in the local kernels (pull, moments, collision); fp64 reductions",
    "fp32": "fp32 storage and arithmetic; fp64 reductions",
    "bf16": "bf16 f - feq storage (fp32 closure populations); fp32 arithmetic; fp64 reductions",
    "bf16_local64": "bf16 f - feq storage (fp32 closure populations); fp32 stencil sums; fp64 arithmetic in the "
                    "local kernels; fp64 reductions",
    "fp64": "fp64 storage and arithmetic",
}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--serving", type=int, default=512, metavar="N",
                    help="requests of the serving trace replayed through the batched server and the plain loop "
                         "(0: skip)")
    ap.add_argument("--serving-planes", type=int, default=4096, help="z-planes of the serving lattice")
    ap.add_argument("--serving-max-steps", type=int, default=60000)
    ap.add_argument("--serving-no-plain", action="store_true", help="batched server only")
    ap.add_argument("--no-extra", action="store_true",
                    help="time only the headline (no other storage modes, no 64^3 slit)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first run one device copy of MIB MiB (a plain copy kernel of known traffic, for "
                         "calibrating HBM byte counters under a profiler)")
    ap.add_argument("--workload", choices=("slab512", "slab64"), default="slab512",
                    help="slab512: the 512x512x256 slab at sigma = 10 (default); slab64: the 64x64x64 slit")
    ap.add_argument("--precision", choices=tuple(PRECISION_LABEL), default="fp32_local64",
                    help="storage and local arithmetic of the timed lattice")
    ap.add_argument("--thermal", action="store_true",
                    help="time only the thermal-field kernel (Q, B_i, F^T) on the workload; one JSON line")
    ap.add_argument("--thermal-flow", action="store_true",
                    help="time only the coupled thermal flow on the workload's lattice (storage as --precision: "
                         "fp64, fp32 or fp32_local64); one JSON line")
    ap.add_argument("--transport", nargs="?", const="bulk,sound,slit", default=None, metavar="PARTS",
                    help="run the transport experiments instead (comma list of bulk, sound, slit, thermal, "
                         "heatmode; "
                         "default bulk, sound, slit); "
                         "one JSON line")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library runs the WDLB step on a single MI355X "
              "(multi-GPU halo exchange is design only); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1304_7880_amd import wdlb
    from paper_1304_7880_amd.workloads import SLAB_64, SLAB_LARGE, SLAB_LARGE_SUB

    w = SLAB_LARGE if args.workload == "slab512" else SLAB_64
    if not os.path.exists(wdlb.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    torch.cuda.set_device(0)
    if args.transport:
        parts = tuple(x for x in args.transport.split(",") if x)
        if not parts or set(parts) - {"bulk", "sound", "slit", "thermal", "heatmode"}:
            sys.exit("--transport takes a comma list of bulk, sound, slit, thermal, heatmode")
        print(json.dumps(transport_bench(parts)), flush=True)
        return
    stream = torch.cuda.current_stream()
    if args.copy_calibration:
        nb = args.copy_calibration << 20
        src = torch.ones(nb // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.thermal:
        print(json.dumps(thermal_bench(w, args.precision)), flush=True)
        return
    if args.thermal_flow:
        print(json.dumps(thermal_flow_bench(w, args.precision, args.steps, args.warmup)), flush=True)
        return

    print(f"bench: {w.name}, {args.precision}, {args.warmup} + {args.steps} steps", file=sys.stderr, flush=True)
    r = timed_run(w, args.precision, args.steps, args.warmup, stream)
    k_avg_s = r["shell_avg_ms"] * 1e-3
    nS = shell_size(w.sigma)
    flops36 = shell_flops_per_node(w.sigma) * w.N
    ops26 = SHELL_OPS_PER_OFFSET * nS * w.N
    traffic, rp_ms = profile_figures(PROFILES[args.workload])
    if args.precision != "fp32_local64":   # counters are taken in the default mode
        traffic, rp_ms = {}, {}
    shell = r["shell_name"]
    step_bytes = sum(traffic.values()) if traffic else None
    # the shell sums run in the storage type's arithmetic (FP32 but for fp64)
    peak = PEAK_FP64_VECTOR_TFLOPS if args.precision == "fp64" else PEAK_FP32_VECTOR_TFLOPS
    out = {
        "metric": "MLUPS (incl. nonlocal force)",
        "value": round(r["mlups"], 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp64" if args.precision == "fp64" else "fp32",
        "data": ("synthetic (seeded +-1% density noise, uniform start)" if w.noise
                 else "synthetic (uniform fluid at rest)"),
        "config": {"workload": w.name, "nodes": w.N, "sigma": w.sigma, "eta": w.eta, "tau": w.tau,
                   "precision": PRECISION_LABEL[args.precision]},
        "roofline": {"bound": "alu", "kernel": shell,
                     "achieved": round(ops26 / k_avg_s / 1e12, 3), "peak": peak,
                     "unit": "TFLOP/s", "frac": round(ops26 / k_avg_s / 1e12 / peak, 4),
                     "traffic": traffic.get(shell),
                     "count": f"{SHELL_OPS_PER_OFFSET:g} operations per shell offset x {nS} offsets x {w.N} nodes",
                     "ops_per_launch": ops26,
                     "achieved_36flop": round(flops36 / k_avg_s / 1e12, 3),
                     "frac_36flop": round(flops36 / k_avg_s / 1e12 / peak, 4),
                     "avg_kernel_ms": round(r["shell_avg_ms"], 5),
                     "avg_kernel_ms_rocprofv3": rp_ms.get(shell)},
        "step_hbm": None if step_bytes is None else {
            "bytes_per_step": step_bytes,
            "achieved_GBs": round(step_bytes / (r["ms_per_step"] * 1e-3) / 1e9, 1), "peak_GBs": PEAK_HBM_GBS,
            "frac": round(step_bytes / (r["ms_per_step"] * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)},
        "kernels_ms_per_step": {k: round(v, 5) for k, v in r["kernels_ms_per_step"].items()},
        "wall_s": round(r["wall_s"], 4),
        "pore_flux": r["pore_flux"],
    }
    if not args.no_extra:
        modes = {}
        for prec in ("fp32", "bf16", "fp64") if args.workload == "slab512" else ():
            print(f"bench: {w.name}, {prec}", file=sys.stderr, flush=True)
            m = timed_run(w, prec, args.steps, args.warmup, stream)
            modes[prec] = {"mlups": round(m["mlups"], 2), "ms_per_step": round(m["ms_per_step"], 5),
                           "precision": PRECISION_LABEL[prec]}
        if modes:
            out["other_precisions"] = modes
        if args.workload == "slab512":
            print(f"bench: {SLAB_64.name}", file=sys.stderr, flush=True)
            m = timed_run(SLAB_64, args.precision, 200, 20, stream)
            out["slab64"] = {"workload": SLAB_64.name, "mlups": round(m["mlups"], 2),
                             "ms_per_step": round(m["ms_per_step"], 5), "steps": 200,
                             "kernels_ms_per_step": {k: round(v, 5) for k, v in m["kernels_ms_per_step"].items()}}
        print(f"bench: thermal fields on {w.name}", file=sys.stderr, flush=True)
        out["thermal_fields"] = thermal_bench(w, args.precision)
        tf_prec = args.precision if args.precision in ("fp64", "fp32", "fp32_local64") else "fp32_local64"
        print(f"bench: coupled thermal flow on {w.name}, {tf_prec}", file=sys.stderr, flush=True)
        out["thermal_flow"] = thermal_flow_bench(w, tf_prec, 5, 2)
    if args.serving:
        out["serving"] = serving_bench(args.serving, args.serving_planes, args.serving_max_steps,
                                       plain=not args.serving_no_plain)
    if not args.no_cpu:
        print("bench: cpu oracle sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(SLAB_LARGE_SUB if args.workload == "slab512" else w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
