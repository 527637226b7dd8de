#!/usr/bin/env python3
"""Throughput of the full-order implicit cell step on one MI355X.

Default mode (one JSON line): a step is one implicit Euler step (eq. 2.13)
of the 64 x 64 x 160 full cell (anode 64 / separator 32 / cathode 64
layers, overlapping-sphere electrodes with radius 3-6 voxels and porosity
drawn in [0.30, 0.40], 2C charge, dt = 5 s, plating on): FP64 residual,
Newton, multigrid-preconditioned GMRES, step limiter, outputs.  The metric is
DOF x steps / s with DOF = 2 x voxels.  Inputs are resident in HBM before
the timed region; timing brackets exactly --steps steps with a device
synchronisation on both sides.  Extra objects: `fp64` (the plain FP64 path
on the same workload), `batched` (32 cells of 32x32x80 .. 96x96x240 with
sampled C-rate, temperature and plating rate, stepped together),
`roofline` (the dominant kernel's algorithmic bytes per launch over its
event-timed average launch duration), `cpu_baseline` (the CPU oracle on a
bounded down-scaled sample of the same workload), `pod` (the POD of Sec.
2.5 by the method of snapshots, on 96 captured states and Newton stages per
field of the same cell, with the Gram kernel's FP64 matrix-core roofline
and the oracle POD timed on one core).

--mode serve (one JSON line): parameter queries of 48x48x120 .. 128x128x320
cells, 12 steps of 5 s each, arriving as a Poisson stream at a continuous-
batching server; reports completed requests/s and p50/p99 latency from
arrival to result, mixed and FP64.
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
PROFILED_KERNEL = "smooth0"     # the kernel class with the largest share of GPU time


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


def run_gpu(w, precision, steps, warmup, stream):
    import torch
    from paper_1704_04139_amd import mbx
    cell = mbx.Cell(w.labels, w.params, precision=precision, stream=stream)
    for _ in range(warmup):
        cell.step(w.dt)
    torch.cuda.synchronize()
    mbx.profile(PROFILED_KERNEL)
    infos = []
    t0 = time.perf_counter()
    for _ in range(steps):
        infos.append(cell.step(w.dt))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    launches, ms, nbytes = mbx.profile_read()
    mbx.profile(None)
    counts = cell.counts
    cell.close()
    wall = t1 - t0
    dof = 2 * counts.n_vox
    return {
        "value": dof * steps / wall,
        "ms_per_step": 1e3 * wall / steps,
        "newton_per_step": sum(i["newton_iters"] for i in infos) / steps,
        "krylov_per_step": sum(i["krylov_iters"] for i in infos) / steps,
        "V_end": infos[-1]["V"],
        "kernel": {"launches": launches, "ms": ms, "bytes": nbytes},
        "counts": counts,
    }


CPU_SNIPPET = r"""
import json, sys, time
sys.path.insert(0, {root!r})
import oracle
from paper_1704_04139_amd import inputs as I
w = I.config1(seed=1, scale=4)
model = oracle.Model(oracle.Geometry(w.labels), w.params.as_dict())
u = model.initial_state()
u, _ = oracle.newton_step(model, u, w.dt)            # first step from equilibrium, untimed
t0 = time.perf_counter()
n = 0
while n < 2:
    u, _ = oracle.newton_step(model, u, w.dt)
    n += 1
t = time.perf_counter() - t0
print(json.dumps({{"voxels": model.N, "steps": n, "seconds": t, "shape": list(w.labels.shape)}}))
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
            "sample": f"{nx}x{ny}x{nz} copy of the 64x64x160 recipe (same generator, 2C, dt 5 s), "
                      f"steps 2-3 after the first step, {d['seconds']:.1f} s, SuperLU Newton, 1 thread",
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


def run_serving(precision, rate_offered, n_req, n_cap, stream, budget_gb):
    """Poisson arrivals at a continuous-batching server; capacity first, then
    a run at 70% utilisation if the offered rate exceeds the capacity."""
    from paper_1704_04139_amd import inputs as I
    from paper_1704_04139_amd import mbx
    steps = 12
    reqs = I.config4_requests(n_req + n_cap)
    dofsteps = [2 * w.labels.size * steps for w in reqs]
    # capacity: a closed burst of n_cap requests
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
    srv = mbx.Server(int(budget_gb * 2**30), precision, dt=5.0, stream=stream)
    base = srv.clock()
    ids = []
    for a, w in zip(arrivals, reqs[n_cap:]):
        while srv.clock() - base < a:
            time.sleep(min(0.005, max(0.0, a - (srv.clock() - base))))
        ids.append(srv.submit(w.labels, w.params, steps))
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
    lat = np.array([i["t_done"] - i["t_submit"] for i in ok]) if ok else np.array([np.nan])
    return {"precision": precision, "capacity_dofsteps_per_s": cap, "offered_rate_hz": rate_offered,
            "rho_offered": rho_offered, "rate_hz": rate, "rho": rate * mean_req / cap, "requests": n_req,
            "completed": len(ok), "completed_per_s": len(ok) / span, "p50_s": float(np.percentile(lat, 50)),
            "p99_s": float(np.percentile(lat, 99)), "mean_s": float(lat.mean()), "max_s": float(lat.max()),
            "busy_frac": st["busy_s"] / span, "batches": st["batches"], "status": status, "errors": errors,
            "capacity_errors": cap_errors}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precision", choices=["mixed", "fp64", "both"], default="both")
    ap.add_argument("--mode", choices=["step", "serve"], default="step")
    ap.add_argument("--batch-cells", type=int, default=32)
    ap.add_argument("--batch-steps", type=int, default=2, help="timed batched steps (0: skip the batched run)")
    ap.add_argument("--serve-requests", type=int, default=10)
    ap.add_argument("--serve-capacity-requests", type=int, default=6,
                    help="requests of the closed burst that measures the server's capacity")
    ap.add_argument("--serve-rate", type=float, default=20.0, help="offered arrival rate, requests/s")
    ap.add_argument("--budget-gb", type=float, default=200.0)
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
    if args.mode == "serve":
        out = {"metric": "served requests/s", "unit": "requests/s", "n_gpus": 1, "higher_is_better": True,
               "data": "synthetic", "config": {"workload": "parameter queries 48x48x120 .. 128x128x320, 12 x 5 s, "
                                                           "Poisson arrivals, continuous batching"}}
        for prec in (["fp64", "mixed"] if args.precision == "both" else [args.precision]):
            out[prec] = run_serving(prec, args.serve_rate, args.serve_requests, args.serve_capacity_requests, stream,
                                    args.budget_gb)
            print(f"[bench] serve {prec}: {json.dumps(out[prec])}", file=sys.stderr, flush=True)
        main_prec = "fp64" if "fp64" in out else "mixed"
        out["value"] = out[main_prec]["completed_per_s"]
        out["p50_s"], out["p99_s"] = out[main_prec]["p50_s"], out[main_prec]["p99_s"]
        print(json.dumps(out), flush=True)
        return
    w = I.config1()
    print(f"[bench] workload {w.name}, {args.warmup} warmup + {args.steps} timed steps", file=sys.stderr, flush=True)
    res = {}
    for prec in (["mixed", "fp64"] if args.precision == "both" else [args.precision]):
        res[prec] = run_gpu(w, prec, args.steps, args.warmup, stream)
        print(f"[bench] {prec}: {res[prec]['ms_per_step']:.1f} ms/step", file=sys.stderr, flush=True)
    # the headline is the plain FP64 path when it ran (the more robust mode and, at
    # this size, as fast as the mixed mode); the other mode is reported beside it
    main_prec = "fp64" if "fp64" in res else "mixed"
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
        "config": {"workload": "full cell 64x64x160 (anode 64 / separator 32 / cathode 64), 2C charge, dt 5 s, "
                               "plating on",
                   "voxels": counts.n_vox, "dof": 2 * counts.n_vox, "anode_faces": counts.n_an_faces,
                   "cathode_faces": counts.n_ca_faces, "precision": main_prec, "parallelism": "1 GPU"},
        "newton_per_step": r["newton_per_step"],
        "krylov_per_step": r["krylov_per_step"],
        "roofline": {"bound": "hbm", "kernel": PROFILED_KERNEL, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS if achieved else None,
                     "traffic": measured_traffic(main_prec),
                     "launches": k["launches"], "avg_us": 1e3 * k["ms"] / max(k["launches"], 1),
                     "bytes_per_launch": k["bytes"] / max(k["launches"], 1)},
    }
    for other in res:
        if other != main_prec:
            f = res[other]
            line[other] = {"value": f["value"], "ms_per_step": f["ms_per_step"],
                           "newton_per_step": f["newton_per_step"], "krylov_per_step": f["krylov_per_step"]}
    if args.pod_snapshots > 0:
        line["pod"] = run_pod(w, args.pod_snapshots, 3, stream, not args.no_cpu_baseline)
        print(f"[bench] pod: {line['pod']['ms_per_pod']:.2f} ms per field, Gram "
              f"{line['pod']['gram']['avg_us']:.1f} us", file=sys.stderr, flush=True)
    if args.batch_steps > 0:
        print(f"[bench] batched: {args.batch_cells} cells, {args.batch_steps} timed steps", file=sys.stderr, flush=True)
        line["batched"] = run_batched(args.batch_cells, args.batch_steps, main_prec, stream)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle, 1 thread)", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
