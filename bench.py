#!/usr/bin/env python3
"""Throughput of the full-order implicit cell step on one MI355X.

Default mode (one JSON line).  The headline workload is the 128 x 128 x 320
full cell (anode 128 / separator 64 / cathode 128 layers, overlapping-sphere
electrodes with radius 3-6 voxels and porosity drawn in [0.30, 0.40]) under
a 3C fast charge at 268 K with 2 s steps, plating on, run to the 4.2 V
cutoff.  A step is one implicit Euler step (eq. 2.13): FP64 residual,
Newton, multigrid-preconditioned GMRES, step limiter, outputs.  The metric is
DOF x steps / s with DOF = 2 x voxels.  Inputs are resident in HBM before the
timed region; timing brackets exactly --steps steps (after --warmup steps)
with a device synchronisation on both sides and no profiling events inside.
Both precision modes run (mixed: FP32 Krylov and preconditioner with FP64
residual and refinement; fp64): the configured mixed mode is the headline,
the other is reported beside it, with the difference of their states after
the same steps.  After the timed steps each cell runs a short event-timed
region for the roofline; the headline precision then continues to the cutoff
(`to_cutoff`; --cutoff all: both precisions).

Further objects: `batched` (32 sampled queries of 32x32x80 .. 96x96x240,
stepped together in mixed precision), `serve` (parameter queries of
48x48x120 .. 128x128x320, 12 steps of 5 s, Poisson arrivals at a
continuous-batching server: capacity, utilisation at the offered 20 req/s,
p50/p99 latency and completed requests/s, mixed and fp64), `roofline` (the
dominant kernel's algorithmic bytes per launch over its event-timed average
launch duration, on the headline cell), `cpu_baseline` (the CPU oracle on a
16x16x40 copy of the headline workload, one core), `pod` (the POD of Sec.
2.5 by the method of snapshots on captured states and Newton stages),
`half_cell` (the paper's own case study, Sec. 3.2: the 100x100x149 graphite /
Li-foil half cell with germ-grain plated Li, delithiated for 60 s under
adaptive implicit Euler; the paper's one-core full-order time is context).

--mode serve runs the serving leg alone.
"""
import argparse
import json
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PROFILED_KERNEL = "smooth0"     # the largest single kernel by GPU time


def committed_traffic(summary, sources, precision):
    """HBM bytes per launch of a profiled kernel from a committed counter
    summary under profiles/ (rocprofv3 FETCH_SIZE + WRITE_SIZE,
    copy-calibrated), or None when the summary is for another precision or
    the kernel's source files have changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", summary)
    try:
        kv = {}
        for ln in open(path):
            if ":" in ln:
                k, v = ln.split(":", 1)
                kv[k.strip()] = v.split()[0] if v.split() else ""
    except OSError:
        return None
    h = hashlib.sha256()
    for f in sources:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if kv.get("precision") != precision or kv.get("source_sha256") != h.hexdigest():
        return None
    return float(kv["traffic_bytes_per_launch"])


def measured_traffic(precision):
    """Traffic of the level-0 smoother (the roofline kernel of the step)."""
    return committed_traffic("mg0_smooth_traffic.txt",
                             ("paper_1704_04139_amd/csrc/mg.hip", "paper_1704_04139_amd/csrc/mbx_dev.h"), precision)


def run_gpu(w, precision, steps, warmup, stream, prof_steps=4, V_cut=None, to_cutoff=True):
    """Steps one cell: warmup steps, `steps` timed steps (no events), then
    prof_steps with the roofline kernel event-timed, then on to the voltage
    cutoff.  Returns the timings and the state after warmup + steps."""
    import torch
    from paper_1704_04139_amd import mbx
    cell = mbx.Cell(w.labels, w.params, precision=precision, stream=stream,
                    **({"V_cut": V_cut} if V_cut else {}))
    t_start = time.perf_counter()
    infos = []
    for k in range(warmup):
        infos.append(cell.step(w.dt))
        print(f"[bench] {precision}: warm-up step {k + 1}/{warmup} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        infos.append(cell.step(w.dt))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    timed = infos[warmup:]
    state = cell.get_state()
    mean_solid = cell.mean_solid()
    V_timed = timed[-1]["V"]
    print(f"[bench] {precision}: {steps} timed steps done", file=sys.stderr, flush=True)
    mbx.profile(PROFILED_KERNEL)
    for k in range(prof_steps):
        infos.append(cell.step(w.dt))
        print(f"[bench] {precision}: event-timed step {k + 1}/{prof_steps} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    launches, ms, nbytes = mbx.profile_read()
    mbx.profile(None)
    cut = None
    if to_cutoff and V_cut:
        while infos[-1]["V"] < V_cut and len(infos) < w.steps:
            infos.append(cell.step(w.dt))
        torch.cuda.synchronize()
        cut = {"steps": len(infos), "wall_s": time.perf_counter() - t_start, "V_end": infos[-1]["V"],
               "reached": bool(infos[-1]["V"] >= V_cut),
               "retried_steps": sum(1 for i in infos if i["substeps"] > 1)}
    counts = cell.counts
    shape = cell.launch_shape()
    cell.close()
    wall = t1 - t0
    dof = 2 * counts.n_vox
    if cut:
        cut["value"] = dof * cut["steps"] / cut["wall_s"]
    return {
        "value": dof * steps / wall,
        "ms_per_step": 1e3 * wall / steps,
        "newton_per_step": sum(i["newton_iters"] for i in timed) / steps,
        "krylov_per_step": sum(i["krylov_iters"] for i in timed) / steps,
        "retried_steps": sum(1 for i in timed if i["substeps"] > 1),
        "V_end": V_timed,
        "kernel": {"launches": launches, "ms": ms, "bytes": nbytes},
        "counts": counts,
        "launch_shape": {"smooth0_threads": shape[0], "matvec_threads": shape[1]},
        "state": state,
        "s_ac": mean_solid,
        "to_cutoff": cut,
    }


PAPER_FULL_ORDER_S = 56315.0    # Sec. 3.2: 15 h 38 min 35 s, one Xeon E5-2698 v3 core, the paper's own constants


def run_half_cell(precision, current_density, stream, t_end=60.0, tol=1e-3):
    """The paper's case study (Sec. 3.2) at its size: the 100 x 100 x 149
    half cell (graphite | separator | Li foil) with germ-grain plated Li,
    delithiated at a constant current density for 60 s under adaptive
    implicit Euler (dt0 0.25 s, dt in [1e-3, 10] s, tol 1e-3)."""
    import torch
    from paper_1704_04139_amd import inputs as I
    from paper_1704_04139_amd import mbx
    w = I.paper_half_cell(seed=3, current_density=current_density)
    mask, n_plated, germs = I.germ_grain_plating(w.labels, w.meta["z_sep_face"], w.params.h, 3)
    cell = mbx.Cell(w.labels, w.params, precision=precision, stream=stream)
    c, p, n = cell.get_state()
    n = n.copy()
    n[mask] = n_plated
    cell.set_state(c, p, n)
    inv0 = cell.inventory()
    counts = cell.counts
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    try:
        t, V, rejected, _ = cell.run_adaptive(t_end, 0.25, 1e-3, 10.0, tol)
        status = "ok"
    except mbx.MbxError as e:
        t, V, rejected, status = np.zeros(0), np.zeros(0), -1, str(e)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    inv = cell.inventory()
    cell.close()
    dof = 2 * counts.n_vox
    steps = int(t.size)
    dts = np.diff(np.concatenate([[0.0], t])) if steps else np.zeros(0)
    return {"workload": f"half cell 100x100x149 (graphite 100 / separator 40 / Li foil 9), germ-grain plated Li, "
                        f"{current_density:g} A/m^2 for {t_end:g} s, adaptive implicit Euler",
            "precision": precision, "status": status, "voxels": counts.n_vox, "dof": dof,
            "germs": int(len(germs)), "plated_faces": int(mask.sum()), "current_density_A_m2": current_density,
            "t_reached_s": float(t[-1]) if steps else 0.0, "steps": steps, "rejected": rejected, "wall_s": wall,
            "dof_steps_per_s": dof * steps / wall if steps else None,
            "dt_min_s": float(dts.min()) if steps else None, "dt_max_s": float(dts.max()) if steps else None,
            "V_first": float(V[0]) if steps else None, "V_end": float(V[-1]) if steps else None,
            "plated_mol": [inv0["plated"], inv["plated"]],
            "paper_full_order_wall_s": PAPER_FULL_ORDER_S,
            "note": "the paper's figure is its own 60 s full-order run on one CPU core with its own constants: context"}


def state_difference(w, a, b):
    """Relative L2 differences per field (c_e, c_s, phi, n) and |dV| between
    two runs of the same cell (Sec. 3.3's relative error in space)."""
    lab = w.labels.ravel()
    pore = lab == 0
    (ca, pa, na), (cb, pb, nb) = a["state"], b["state"]
    rel = lambda x, y, floor=0.0: float(np.linalg.norm(x - y) / max(np.linalg.norm(y), floor))  # noqa: E731
    out = {"c_e": rel(ca[pore], cb[pore]), "c_s": rel(ca[~pore], cb[~pore]), "phi": rel(pa, pb),
           "n": rel(na, nb, w.params.n_c * np.sqrt(max(nb.size, 1))), "V_abs": abs(a["V_end"] - b["V_end"]),
           "s_ac_rel": [abs(x - y) / abs(y) for x, y in zip(a["s_ac"], b["s_ac"])]}
    return out


CPU_SNIPPET = r"""
import json, os, sys, time
cpus = sorted(os.sched_getaffinity(0))
os.sched_setaffinity(0, {{cpus[0]}})                 # one core
sys.path.insert(0, {root!r})
import oracle
from paper_1704_04139_amd import inputs as I
w = I.config2(seed=2, scale=8)
model = oracle.Model(oracle.Geometry(w.labels), w.params.as_dict())
u = model.initial_state()
t0 = time.perf_counter()
n = 0
while n < 2:
    u, _ = oracle.newton_step(model, u, w.dt)
    n += 1
t = time.perf_counter() - t0
print(json.dumps({{"voxels": model.N, "steps": n, "seconds": t, "shape": list(w.labels.shape),
                  "core": cpus[0], "affinity": sorted(os.sched_getaffinity(0))}}))
"""


def cpu_baseline():
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-c", CPU_SNIPPET.format(root=ROOT)], capture_output=True, text=True,
                       env=env, timeout=600)
    if r.returncode != 0:
        return {"value": None, "error": r.stderr[-400:]}
    d = json.loads(r.stdout.strip().splitlines()[-1])
    nz, ny, nx = d["shape"]
    cpu = "unknown"
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                cpu = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": 2 * d["voxels"] * d["steps"] / d["seconds"], "unit": "DOF*steps/s", "cores": 1,
            "kind": "oracle",
            "sample": f"extrapolated: the first {d['steps']} steps of a {nx}x{ny}x{nz} copy of the headline "
                      f"workload (same generator, 3C at 268 K, dt 2 s), {d['seconds']:.1f} s, SuperLU Newton, "
                      f"1 thread pinned to core {d['core']}; the 128x128x320 cell itself is out of the oracle's "
                      f"reach (sparse LU fill)",
            "host_cpu": cpu, "host_nproc": os.cpu_count()}


FP64_MFMA_PEAK_TFLOPS = 78.6   # MI355X dense FP64 matrix peak


def run_pod(w, n_snap, reps, stream, with_oracle):
    """POD by the method of snapshots (Sec. 2.5) of the concentration and the
    potential snapshot sets of the benchmark cell: its states and Newton
    stages, captured on the device while it steps (untimed), then reps timed
    POD calls per field at rtol 1e-7 (the tolerance of Sec. 3.2)."""
    import torch
    from paper_1704_04139_amd import mbx
    cell = mbx.Cell(w.labels, w.params, precision="fp64", stream=stream)
    N = cell.counts.n_vox
    dc = torch.empty((n_snap, N), dtype=torch.float64, device="cuda")
    dp = torch.empty((n_snap, N), dtype=torch.float64, device="cuda")
    cell.capture(dc.data_ptr(), dp.data_ptr(), N, n_snap)
    steps = 0
    while cell.captured()[0] < n_snap and steps < 200:
        cell.step(w.dt)
        steps += 1
    m = cell.captured()[0]
    cell.close()
    torch.cuda.synchronize()
    print(f"[bench] pod: {m} snapshots per field captured over {steps} steps", file=sys.stderr, flush=True)
    du = torch.empty((m, N), dtype=torch.float64, device="cuda")
    ks = {}
    for name, buf in (("c", dc), ("phi", dp)):          # warm-up
        _, ks[name] = mbx.pod(buf.data_ptr(), N, m, N, du.data_ptr(), N, m, 1e-7, stream=stream)
    torch.cuda.synchronize()
    mbx.profile("gram")
    t0 = time.perf_counter()
    for _ in range(reps):
        for buf in (dc, dp):
            mbx.pod(buf.data_ptr(), N, m, N, du.data_ptr(), N, m, 1e-7, stream=stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    launches, ms, nbytes = mbx.profile_read()
    mbx.profile(None)
    flops = float(N) * m * (m + 1)                  # the m(m+1)/2 distinct entries, 2 flops per row each
    avg_s = ms * 1e-3 / max(launches, 1)
    out = {"snapshots": m, "rows": N, "fields": ["c", "phi"], "steps_captured": steps, "rtol": 1e-7,
           "k": ks, "ms_per_pod": 1e3 * (t1 - t0) / (2 * reps),
           "gram": {"bound": "mfma", "kernel": "gram", "achieved": flops / avg_s / 1e12 if launches else None,
                    "peak": FP64_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": flops / avg_s / 1e12 / FP64_MFMA_PEAK_TFLOPS if launches else None,
                    "traffic": committed_traffic("gram_traffic.txt", ("paper_1704_04139_amd/csrc/pod.hip",), "fp64"),
                    "launches": launches, "avg_us": 1e6 * avg_s, "flops_per_launch": flops,
                    "bytes_per_launch": nbytes / max(launches, 1),
                    "hbm_gbs": nbytes / max(launches, 1) / avg_s / 1e9 if launches else None}}
    if with_oracle:
        import oracle
        from threadpoolctl import threadpool_limits
        S = dc[:m].cpu().numpy().T.copy()
        with threadpool_limits(1):
            t0 = time.perf_counter()
            oracle.pod(S, rtol=1e-7)
            t1 = time.perf_counter()
        out["cpu_oracle"] = {"ms_per_pod": 1e3 * (t1 - t0), "cores": 1, "kind": "oracle",
                             "sample": f"the same {N} x {m} concentration snapshots, NumPy/LAPACK, 1 thread"}
    del dc, dp, du
    torch.cuda.empty_cache()
    return out


def run_batched(n_cells, steps, precision, stream):
    """32-cell batch (sampled queries), all cells advanced by shared launches."""
    import torch
    from paper_1704_04139_amd import inputs as I
    from paper_1704_04139_amd import mbx
    ws = I.config3(n_cells=n_cells)
    cells = [mbx.Cell(w.labels, w.params, precision=precision, stream=stream) for w in ws]
    dof = sum(2 * c.counts.n_vox for c in cells)
    print(f"[bench] batched: {n_cells} cells created, {dof} DOF", file=sys.stderr, flush=True)
    st, _ = mbx.batch_step(cells, ws[0].dt)          # warm-up step (also builds the batch tables)
    torch.cuda.synchronize()
    print("[bench] batched: warm-up step done", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    kry = newt = 0
    for k in range(steps):
        st, infos = mbx.batch_step(cells, ws[0].dt)
        kry += sum(i["krylov_iters"] for i in infos)
        newt += sum(i["newton_iters"] for i in infos)
        print(f"[bench] batched: step {k + 1}/{steps} done at {time.perf_counter() - t0:.1f} s", file=sys.stderr,
              flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    for c in cells:
        c.close()
    return {"value": dof * steps / wall, "unit": "DOF*steps/s", "cells": n_cells, "dof": dof, "steps": steps,
            "ms_per_step": 1e3 * wall / steps, "failed": {str(k): int(x) for k, x in enumerate(st) if x != 0},
            "newton_per_cell_step": newt / (steps * n_cells), "krylov_per_cell_step": kry / (steps * n_cells),
            "precision": precision}


def _drain(srv, what, limit_s=3600.0):
    """Wait for the server to go idle, printing progress every 30 s."""
    from paper_1704_04139_amd import mbx
    t0 = time.perf_counter()
    while True:
        try:
            srv.drain(30.0)
            return
        except mbx.MbxError as e:
            if e.code != mbx.MBX_ESTATE or time.perf_counter() - t0 > limit_s:
                raise
        st = srv.stats()
        print(f"[serve] {what}: {st['running']} running, {st['queued']} queued, {st['steps_run']} cell-steps done",
              file=sys.stderr, flush=True)


def serving_requests(n):
    """The served parameter queries (generated once, shared by both precisions)."""
    from paper_1704_04139_amd import inputs as I
    t0 = time.perf_counter()
    reqs = I.config4_requests(n)
    print(f"[serve] {n} requests generated in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    return reqs


def run_serving(precision, rate_offered, reqs, n_cap, stream, budget_gb, steps=12):
    """Poisson arrivals at a continuous-batching server: capacity from a closed
    burst of the first n_cap requests, then the remaining requests arriving at
    the offered rate, or at 70% of capacity if the offered rate exceeds it."""
    from paper_1704_04139_amd import inputs as I
    from paper_1704_04139_amd import mbx
    n_req = len(reqs) - n_cap
    dofsteps = [2 * w.labels.size * steps for w in reqs]
    srv = mbx.Server(int(budget_gb * 2**30), precision, dt=5.0, stream=stream)
    t0 = srv.clock()
    ids = [srv.submit(w.labels, w.params, steps) for w in reqs[:n_cap]]
    _drain(srv, f"{precision} capacity burst")
    cinfos = [srv.poll(i) for i in ids]
    cap_errors = {k: srv.error(i) for k, (i, inf) in enumerate(zip(ids, cinfos)) if inf["status"] < 0}
    t1 = max(inf["t_done"] for inf in cinfos)
    srv.close()
    # DOF x steps actually completed (a failed request stops early)
    cap = sum(2 * w.labels.size * inf["steps_done"] for w, inf in zip(reqs[:n_cap], cinfos)) / (t1 - t0)
    mean_req = float(np.mean(dofsteps[n_cap:]))
    rho_offered = rate_offered * mean_req / cap
    rate = rate_offered if rho_offered < 1.0 else 0.7 * cap / mean_req
    arrivals = I.poisson_arrivals(rate, n_req)
    print(f"[serve] {precision}: capacity {cap:.3e} DOF*steps/s, offered rho {rho_offered:.1f}, "
          f"running at {rate:.3f} req/s", file=sys.stderr, flush=True)
    srv = mbx.Server(int(budget_gb * 2**30), precision, dt=5.0, stream=stream)
    base = srv.clock()
    ids = []
    for a, w in zip(arrivals, reqs[n_cap:]):
        while srv.clock() - base < a:
            time.sleep(min(0.005, max(0.0, a - (srv.clock() - base))))
        ids.append(srv.submit(w.labels, w.params, steps))
        if len(ids) % 10 == 0:
            print(f"[serve] {precision} request {len(ids)}/{n_req} at {srv.clock() - base:.2f} s", file=sys.stderr,
                  flush=True)
    _drain(srv, f"{precision} Poisson run")
    infos = [srv.poll(i) for i in ids]
    errors = {k: srv.error(i) for k, (i, inf) in enumerate(zip(ids, infos)) if inf["status"] < 0}
    st = srv.stats()
    srv.close()
    status = [int(i["status"]) for i in infos]
    span = max(i["t_done"] for i in infos) - base
    ok = [i for i in infos if i["status"] == mbx.MBX_REQ_DONE]
    # latency percentiles over the requests that completed all their steps (a
    # failed request retires early and would pull them down)
    lat = np.sort(np.array([i["t_done"] - i["t_submit"] for i in ok])) if ok else np.array([np.nan])
    rank99 = int(np.ceil(0.99 * lat.size)) - 1          # nearest-rank p99
    return {"precision": precision, "capacity_dofsteps_per_s": cap, "capacity_requests": n_cap,
            "offered_rate_hz": rate_offered, "rho_offered": rho_offered, "rate_hz": rate,
            "rho": rate * mean_req / cap, "requests": n_req, "completed": len(ok),
            "completed_per_s": len(ok) / span, "dofsteps_per_s": sum(dofsteps[n_cap:][k] for k, i in
                                                                    enumerate(infos) if i["status"] == 0) / span,
            "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "p99_nearest_rank_s": float(lat[rank99]), "mean_s": float(lat.mean()), "max_s": float(lat.max()),
            "busy_frac": st["busy_s"] / span, "batches": st["batches"],
            "retried_steps": int(sum(i["retried"] for i in infos)), "failed": [k for k, x in enumerate(status) if x < 0],
            "errors": errors, "capacity_errors": cap_errors}


HEADLINE_PRECISION = "mixed"   # the precision the 128x128x320 workload is specified in


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precision", choices=["mixed", "fp64", "both"], default="both")
    ap.add_argument("--mode", choices=["step", "serve"], default="step")
    ap.add_argument("--cutoff", choices=["headline", "all", "none"], default="headline",
                    help="which precisions continue to the 4.2 V cutoff after the timed steps")
    ap.add_argument("--no-cutoff", action="store_true", help="same as --cutoff none")
    ap.add_argument("--batch-cells", type=int, default=32)
    ap.add_argument("--batch-steps", type=int, default=2, help="timed batched steps (0: skip the batched run)")
    ap.add_argument("--serve-requests", type=int, default=24, help="Poisson-run requests per precision (0: skip)")
    ap.add_argument("--serve-capacity-requests", type=int, default=8,
                    help="requests of the closed burst that measures the server's capacity")
    ap.add_argument("--serve-rate", type=float, default=20.0, help="offered arrival rate, requests/s")
    ap.add_argument("--budget-gb", type=float, default=200.0)
    ap.add_argument("--half-cell-densities", default="-250",
                    help="comma-separated current densities (A/m^2, negative: delithiation) of the paper's half-cell "
                         "case run for 60 s ('' to skip)")
    ap.add_argument("--pod-snapshots", type=int, default=96,
                    help="snapshots per field for the POD measurement (0: skip it)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run one device-to-device copy of this size first (calibrates profiler byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); independent cells shard across GPUs "
              "without communication, which this benchmark does not launch.", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1704_04139_amd import inputs as I
    from paper_1704_04139_amd import mbx
    mbx.load()
    torch.cuda.init()
    stream = torch.cuda.current_stream().cuda_stream
    if args.copy_probe_mib > 0:
        n = args.copy_probe_mib * 2**20 // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        print(f"[bench] copy probe: {args.copy_probe_mib} MiB device-to-device", file=sys.stderr, flush=True)
        del a, b
    precs = ["mixed", "fp64"] if args.precision == "both" else [args.precision]
    serve_workload = ("parameter queries 48x48x120 .. 128x128x320, C-rate U[0.5,4], T U[268,308] K, plating rate "
                      "log-U[1e-2,1e2] x default, 12 x 5 s, Poisson arrivals, continuous batching")
    if args.mode == "serve":
        reqs = serving_requests(args.serve_requests + args.serve_capacity_requests)
        out = {"metric": "served requests/s", "unit": "requests/s", "n_gpus": 1, "higher_is_better": True,
               "data": "synthetic", "config": {"workload": serve_workload}}
        for prec in precs:
            out[prec] = run_serving(prec, args.serve_rate, reqs, args.serve_capacity_requests, stream,
                                    args.budget_gb)
            print(f"[bench] serve {prec}: {json.dumps(out[prec])}", file=sys.stderr, flush=True)
        main_prec = HEADLINE_PRECISION if HEADLINE_PRECISION in out else precs[0]
        out["value"] = out[main_prec]["completed_per_s"]
        out["p50_s"], out["p99_s"] = out[main_prec]["p50_s"], out[main_prec]["p99_s"]
        print(json.dumps(out), flush=True)
        return
    w = I.config2()
    V_cut = w.meta["cutoff_V"]
    print(f"[bench] workload {w.name}, {args.warmup} warmup + {args.steps} timed steps", file=sys.stderr, flush=True)
    res = {}
    for prec in precs:
        cutoff = "none" if args.no_cutoff else args.cutoff
        to_cut = cutoff == "all" or (cutoff == "headline" and prec == HEADLINE_PRECISION)
        res[prec] = run_gpu(w, prec, args.steps, args.warmup, stream, V_cut=V_cut, to_cutoff=to_cut)
        cut = res[prec]["to_cutoff"]
        print(f"[bench] {prec}: {res[prec]['ms_per_step']:.1f} ms/step" +
              (f", {cut['steps']} steps to the cutoff in {cut['wall_s']:.1f} s" if cut else ""),
              file=sys.stderr, flush=True)
    main_prec = HEADLINE_PRECISION if HEADLINE_PRECISION in res else precs[0]
    r = res[main_prec]
    k = r["kernel"]
    achieved = (k["bytes"] / k["launches"]) / (k["ms"] / k["launches"] * 1e-3) / 1e9 if k["launches"] else None
    counts = r["counts"]
    line = {
        "metric": "DOF*timesteps/s",
        "value": r["value"],
        "unit": "DOF*steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32" if main_prec == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": "full cell 128x128x320 (anode 128 / separator 64 / cathode 128), 3C charge at "
                               "268 K, dt 2 s, plating on, to the 4.2 V cutoff",
                   "voxels": counts.n_vox, "dof": 2 * counts.n_vox, "anode_faces": counts.n_an_faces,
                   "cathode_faces": counts.n_ca_faces, "precision": main_prec, "parallelism": "1 GPU"},
        "newton_per_step": r["newton_per_step"],
        "krylov_per_step": r["krylov_per_step"],
        "retried_steps": r["retried_steps"],
        "launch_shape": r["launch_shape"],
        "to_cutoff": r["to_cutoff"],
        "roofline": {"bound": "hbm", "kernel": PROFILED_KERNEL, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS if achieved else None,
                     "traffic": measured_traffic(main_prec),
                     "launches": k["launches"], "avg_us": 1e3 * k["ms"] / max(k["launches"], 1),
                     "bytes_per_launch": k["bytes"] / max(k["launches"], 1),
                     "timing": "HIP events on the kernel's stream over steps run after the timed region"},
    }
    for other in res:
        if other != main_prec:
            f = res[other]
            line[other] = {"value": f["value"], "ms_per_step": f["ms_per_step"],
                           "newton_per_step": f["newton_per_step"], "krylov_per_step": f["krylov_per_step"],
                           "retried_steps": f["retried_steps"], "to_cutoff": f["to_cutoff"]}
    if "mixed" in res and "fp64" in res:
        # at this size the CPU oracle is out of reach: the FP64 GPU path is the reference of the mixed one
        line["mixed_vs_fp64"] = dict(state_difference(w, res["mixed"], res["fp64"]),
                                     after_steps=args.warmup + args.steps)
    del res
    if args.batch_steps > 0:
        print(f"[bench] batched: {args.batch_cells} cells, {args.batch_steps} timed steps", file=sys.stderr, flush=True)
        line["batched"] = run_batched(args.batch_cells, args.batch_steps, HEADLINE_PRECISION, stream)
    if args.serve_requests > 0:
        reqs = serving_requests(args.serve_requests + args.serve_capacity_requests)
        line["serve"] = {"workload": serve_workload}
        for prec in precs:
            line["serve"][prec] = run_serving(prec, args.serve_rate, reqs, args.serve_capacity_requests, stream,
                                              args.budget_gb)
            sv = line["serve"][prec]
            print(f"[bench] serve {prec}: p50 {sv['p50_s']:.2f} s, p99 {sv['p99_s']:.2f} s, "
                  f"{sv['completed_per_s']:.3f} req/s", file=sys.stderr, flush=True)
        del reqs
    dens = [float(x) for x in args.half_cell_densities.split(",") if x.strip()]
    if dens:
        line["half_cell"] = []
        for mu in dens:
            r = run_half_cell(HEADLINE_PRECISION, mu, stream)
            line["half_cell"].append(r)
            print(f"[bench] half cell {mu:g} A/m^2: {r['steps']} steps ({r['rejected']} rejected) to "
                  f"{r['t_reached_s']:.1f} s in {r['wall_s']:.1f} s, {r['status']}", file=sys.stderr, flush=True)
    if args.pod_snapshots > 0:
        line["pod"] = run_pod(I.config1(), args.pod_snapshots, 3, stream, not args.no_cpu_baseline)
        print(f"[bench] pod: {line['pod']['ms_per_pod']:.2f} ms per field, Gram "
              f"{line['pod']['gram']['avg_us']:.1f} us", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle, 1 core)", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
