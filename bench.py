#!/usr/bin/env python3
"""Benchmark: simulation steps per second of the subsystem-based ADMM step on one GPU.

Workload (default): 1024 independent legged articulated scenes (4-6 limbs of 2-4 links,
6-48 DOF subsystems, ~12k subsystems, 2-16 ground contacts per scene, mu U[0.3, 1.0]),
FP32, dt = 1e-3, penalty of Eq. (23), stopping test r_theta <= 1e-6 per scene (at most
1000 iterations), previous-step warm start.  One step = construction, factorisation,
the ADMM iteration and the state update for all 1024 scenes (Algorithm 1 once).

Prints one JSON line.  The loop kernel's achieved bandwidth is the algorithmic bytes of
the streamed per-iteration model (factor, J, b, slot state and interface rows of every
iterating scene) times its iterations, over the kernel time measured with HIP events on
the library's stream.  ``cpu_baseline`` times the FP64 CPU oracle on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_legged1024.md")
KERNEL_SRC = os.path.join(ROOT, "paper_2302_14344_amd", "csrc", "kernels_admm.hip")


def measured_traffic():
    """HBM bytes per loop-kernel launch from the committed rocprofv3 counter summary
    (FETCH_SIZE and WRITE_SIZE scaled by a plain-copy calibration), or None when the
    kernel source changed after the counters were taken."""
    import hashlib
    try:
        txt = open(TRAFFIC_FILE).read()
        h = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]
    except OSError:
        return None
    for line in txt.splitlines():
        line = line.strip()
        if line.startswith("{") and '"hbm_bytes_per_launch"' in line:
            d = json.loads(line)
            if d.get("source_sha256_16") == h:
                return d["hbm_bytes_per_launch"]
    return None


def streamed_bytes_per_iteration(sc, real_bytes=4):
    """Per-scene algorithmic bytes of one ADMM iteration (x-update + residual + z/u):
    the Cholesky factor n_i(n_i+1)/2 and b_i of each subsystem, the J values of each
    slot row (12 for a row spanning two bodies of one subsystem, else 6), 16 bytes of
    slot state per slot row (w read, y written, y read, w written), and per interface
    e_j and lambda_j (d_j each) plus one beta per member."""
    R = real_bytes
    ns = sc.n_scenes
    out = np.zeros(ns)
    n = sc.sub_ndof.astype(np.int64)
    np.add.at(out, sc.sub_scene, R * (n * (n + 1) // 2 + n))
    for j in range(sc.n_if):
        s = sc.sub_scene[sc.if_sub[j, 0]]
        d = int(sc.if_dim[j])
        m = int(sc.if_nsub[j])
        intra_two_bodies = (sc.if_kind[j] == 0 and m == 1)
        nnz = 12 if intra_two_bodies else 6
        out[s] += m * d * (R * nnz + 16) + R * (2 * d + m)
    return out


def cpu_baseline(sc, seconds=12.0, threads=None):
    """The FP64 oracle (as it stands) on the same workload, previous-step warm start,
    timed on the host cores over a bounded number of steps."""
    import oracle as O
    if threads is None:
        try:
            threads = len(os.sched_getaffinity(0))
        except AttributeError:
            threads = os.cpu_count() or 1
        threads = max(1, min(threads, 16))
    state = (sc.pos, sc.rot, sc.vel, sc.omega)
    z = u = None
    # two untimed steps, then time whole steps until the budget is used
    for _ in range(2):
        state, r = O.rigid_step(sc, max_iters=1000, tol=1e-6, z0=z, u0=u, n_threads=threads, state=state)
        z, u = r.z, r.u
    n = 0
    t0 = time.perf_counter()
    while True:
        state, r = O.rigid_step(sc, max_iters=1000, tol=1e-6, z0=z, u0=u, n_threads=threads, state=state)
        z, u = r.z, r.u
        n += 1
        if time.perf_counter() - t0 >= seconds:
            break
    dt = time.perf_counter() - t0
    return {"value": n / dt, "unit": "steps/s", "cores": threads, "kind": "oracle",
            "sample": f"{n} consecutive steps (after 2 untimed) of the full {sc.n_scenes}-scene workload, "
                      f"FP64 oracle with OpenMP over scenes, previous-step warm start, tol 1e-6"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--scenes", type=int, default=1024)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--max-iters", type=int, default=1000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="only run a plain device copy of this many MiB (HBM counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU only; --gpus {args.gpus} is not supported "
              "(scenes are independent, so more GPUs would each take a share of the batch).", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py: no GPU available", file=sys.stderr)
        sys.exit(2)

    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_mib": args.copy_calibration}))
        return

    from paper_2302_14344_amd import scenes as S
    from paper_2302_14344_amd.solver import Problem, rigid_state_tensors

    sc = S.legged_scenes(args.scenes)
    pr = Problem.from_rigid(sc, dtype=torch.float32)
    st = rigid_state_tensors(sc, dtype=torch.float32)
    for _ in range(args.warmup):
        pr.rigid_step(*st, max_iters=args.max_iters, tol=args.tol, warm="prev")
    torch.cuda.synchronize()
    pr.reset_totals()
    pr.timing_begin(16 * args.steps + 16)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(pr.stream)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        pr.rigid_step(*st, max_iters=args.max_iters, tol=args.tol, warm="prev")
    ev1.record(pr.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kt = pr.timing_end()
    ms = ev0.elapsed_time(ev1)
    stats = pr.stats()
    pr.check()

    steps_per_s = args.steps / (ms / 1e3)
    iters_total = stats["iters_total"].astype(np.float64)
    unconv = int(stats["unconverged_total"].sum())
    per_it = streamed_bytes_per_iteration(sc)
    alg_bytes = float(np.sum(per_it * iters_total))
    loop_ms, loop_n = kt["loop"]
    achieved = alg_bytes / (loop_ms / 1e3) / 1e9 / 1.0
    per_launch_bytes = alg_bytes / max(loop_n, 1)
    line = {
        "metric": "sim steps/sec at residual<=1e-6 (plain ADMM, previous-step warm start)",
        "value": round(steps_per_s, 3),
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded legged articulated scenes)",
        "config": {
            "workload": f"legged-{args.scenes}: batched articulated scenes, {sc.n_sub} subsystems of 6-48 DOF, "
                        f"{sc.n_if} interfaces, {len(sc.contact_body)} ground contacts",
            "scenes": args.scenes, "dt": sc.dt, "tol": args.tol, "max_iters": args.max_iters,
            "warm_start": "previous step", "beta": "Eq. (23)",
            "scene_steps_per_s": round(steps_per_s * args.scenes, 1),
            "mean_iters_per_scene_step": round(float(iters_total.sum()) / (args.scenes * args.steps), 2),
            "unconverged_scene_steps": unconv,
            "kernel_ms_per_step": {k: round(v[0] / args.steps, 5) for k, v in kt.items()},
            "kernel_launches_per_step": {k: v[1] / args.steps for k, v in kt.items()},
            "wall_s": round(wall, 3),
        },
        "roofline": {
            "kernel": "loop_kernel (the ADMM iteration)",
            "bound": "hbm",
            "achieved": round(achieved, 2),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(),
            "traffic_unit": "bytes per launch",
            "algorithmic_bytes_per_launch": round(per_launch_bytes),
            "avg_launch_ms": round(loop_ms / max(loop_n, 1), 5),
        },
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(sc, seconds=args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
