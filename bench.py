#!/usr/bin/env python3
"""Benchmark: batched compact finite-difference step on one MI355X.

One step applies the first and second derivative along x, y and z (the
pentadiagonal 8th-order tuned scheme with its matched closures) to 22 fields
on 64 mesh blocks whose extents are drawn from {16,24,32,48}^3, all in one
graph launch.  Inputs are resident in HBM before timing starts.

Prints one JSON line: derivative evaluations per second (interior points x
fields x (direction, order) pairs), the roofline of the line kernels against
HBM bandwidth, and the oracle's CPU throughput on a bounded sample.
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
OPS_PENTA = [("(1)QP_O8[1]", 0), ("(1)QP_O8[1]", 1), ("(1)QP_O8[1]", 2),
             ("(2)QP_O8[1]", 0), ("(2)QP_O8[1]", 1), ("(2)QP_O8[1]", 2)]


def algorithmic_bytes(wl, ops, esize):
    """Every input value a derivative needs read once (interior plus the ghost
    faces of the differentiated directions; no edges or corners), every output
    written once."""
    dirs = sorted({op[1] for op in ops})
    rd = wr = 0
    for b in wl.blocks:
        nx, ny, nz = b.n
        n3 = nx * ny * nz
        faces = {0: ny * nz, 1: nx * nz, 2: nx * ny}
        ghost = sum(2 * b.ng * faces[d] for d in dirs if b.boundary[d] == 0)
        rd += wl.nfields * (n3 + ghost)
        wr += len(ops) * wl.nfields * n3
    return (rd + wr) * esize, rd * esize, wr * esize


def run_gpu(wl, ops, dtype, steps, warmup, autotune=True):
    import torch
    import paper_2302_14858_amd as P
    from tests import helpers as H
    tdt = torch.float64 if dtype == P.CFD_F64 else torch.float32
    plan = H.make_plan(wl, ops, dtype=dtype)
    nin, nout = plan.sizes()
    x = torch.from_numpy(wl.data).to(device="cuda", dtype=tdt)
    y = torch.empty(nout, dtype=tdt, device="cuda")
    if autotune:
        plan.autotune(x, y, cache_path=os.path.join(ROOT, "_work", "autotune_cache.txt")
                      if os.path.isdir(os.path.join(ROOT, "_work")) else None)
    plan.capture_graph(x, y)
    for _ in range(warmup):
        plan.launch_graph()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        plan.launch_graph()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = e0.elapsed_time(e1) / steps
    launches, items = plan.stats()
    return plan, x, y, ev_ms, wall, launches, items


def check_sample(plan, y, wl, ops, blocks):
    """Sampled parity against the oracle on a few blocks (all fields, all ops)."""
    from tests import helpers as H
    _, ooffs = plan.offsets()
    flat = y.double().cpu().numpy()
    g = H.unpack(wl, ops, flat, ooffs)
    o = H.oracle_run(wl, ops, blocks=blocks)
    return H.max_rel_err(g, o)


def cpu_baseline(wl, ops, budget_s=12.0):
    """Oracle (plain C, OpenMP over lines) on a bounded sample of the same workload."""
    from oracle import lines as OL
    from oracle import schemes as OS
    schemes = {op[0]: OS.named(op[0]) for op in ops}
    threads = OL.max_threads()
    evals = 0
    t0 = time.perf_counter()
    nb = 0
    passes = 0
    while time.perf_counter() - t0 < budget_s:
        for b, blk in enumerate(wl.blocks):
            for f in range(wl.nfields):
                fv = wl.field_view(b, f)
                for name, d in ops:
                    OL.apply_block(schemes[name], fv, blk.ng, blk.h[d], d)
                evals += len(ops) * int(np.prod(blk.n))
            nb += 1
            if time.perf_counter() - t0 > budget_s:
                break
        passes += 1
    dt = time.perf_counter() - t0
    return {"value": evals / dt, "unit": "evals/s", "cores": threads, "kind": "oracle",
            "sample": f"{nb} block passes over the {len(wl.blocks)} blocks ({passes} sweeps) x {wl.nfields} "
                      f"fields x {len(ops)} ops: {evals} evals in {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import torch
    import synth
    import paper_2302_14858_amd as P
    torch.cuda.init()
    print("bench: generating batch64 workload", file=sys.stderr, flush=True)
    wl = synth.batch64()
    ops = OPS_PENTA
    evals = wl.interior_points * wl.nfields * len(ops)

    print("bench: FP64 batched step", file=sys.stderr, flush=True)
    plan, x, y, ev_ms, wall, launches, items = run_gpu(wl, ops, P.CFD_F64, args.steps, args.warmup,
                                                       autotune=not args.no_autotune)
    alg, rd, wr = algorithmic_bytes(wl, ops, 8)
    achieved = alg / (ev_ms * 1e-3) / 1e9
    err64 = check_sample(plan, y, wl, ops, blocks=[0, 1, 2])
    result = {
        "metric": "derivative evals/s (points x fields x (dir, order) pairs), FP64, batched penta O(8) D1+D2",
        "value": evals / (ev_ms * 1e-3),
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ev_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "batch64: 64 blocks, extents from {16,24,32,48}^3 (seed 3), ng=5, 22 fields, "
                               "D1+D2 along x,y,z, (d)QP_O8[1] + matched closures, one graph launch",
                   "interior_points": wl.interior_points, "fields": wl.nfields, "ops": len(ops),
                   "evals_per_step": evals, "kernel_launches_per_step": launches, "work_items": items},
        "err_vs_oracle": err64,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "algorithmic_bytes": alg, "read_bytes": rd, "write_bytes": wr},
    }
    del x, y, plan
    torch.cuda.empty_cache()
    if not args.no_extra:
        print("bench: FP32 batched step", file=sys.stderr, flush=True)
        plan, x, y, ms32, _, _, _ = run_gpu(wl, ops, P.CFD_F32, args.steps, args.warmup,
                                            autotune=not args.no_autotune)
        alg32, _, _ = algorithmic_bytes(wl, ops, 4)
        err32 = check_sample(plan, y, wl, ops, blocks=[0, 1, 2])
        result["extra"] = {"f32": {"value": evals / (ms32 * 1e-3), "ms_per_step": ms32, "err_vs_oracle": err32,
                                   "achieved_GBs": alg32 / (ms32 * 1e-3) / 1e9}}
        del x, y, plan
        torch.cuda.empty_cache()
    if not args.no_cpu:
        print("bench: CPU oracle sample", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(wl, ops)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
