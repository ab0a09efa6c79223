#!/usr/bin/env python3
"""Benchmark: batched compact finite-difference step on one MI355X.

One step applies the first and second derivative along x, y and z (the
pentadiagonal 8th-order tuned scheme with its matched closures) to 22 fields
on 64 mesh blocks whose extents are drawn from {16,24,32,48}^3, all in one
graph launch.  Inputs are resident in HBM before timing starts.

Prints one JSON line: derivative evaluations per second (interior points x
fields x (direction, order) pairs), the roofline of the line kernels against
HBM bandwidth, and the oracle's CPU throughput on a bounded sample.  Under
"extra": the same step in FP32, one 128^3 block with closures (tridiagonal
D1+D2), the shift-advection term with the biased X_2 upwind pair and the
Kreiss-Oliger / mixed-derivative part of the Z4c derivative set on the same
blocks, the periodic 256^3 precision study (banded FP64 / banded FP32 / dense
mixed BF16 with FP64 residual refinement, each with its error against the
oracle) and the RK4 wave evolution on a periodic 192^3 grid.
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
# HBM bytes per batch64 FP64 step (the one launch of the tuned schedule, flags 4), from rocprofv3
# FETCH_SIZE and WRITE_SIZE passes scaled by what the same counters read for a 1 GiB device copy
# (x2.0 and x1.0): 0.701 GB read + 1.937 GB written.  Valid for the line kernels as they are now; set
# to None when they change until the counters are taken again.
MEASURED_TRAFFIC_BYTES = 2.638e9
MEASURED_TRAFFIC_FLAGS = 4      # the launch shape the counters were taken on (reported only for that shape
MEASURED_TRAFFIC_PARTS = "16:0:1,16:1:2,24:0:2,24:1:2,32:0:2,32:1:4,48:0:4,48:1:4"   # these partitions
MEASURED_TRAFFIC_LAUNCHES = 1   # and this many kernel launches per step)
OPS_PENTA = [("(1)QP_O8[1]", 0), ("(1)QP_O8[1]", 1), ("(1)QP_O8[1]", 2),
             ("(2)QP_O8[1]", 0), ("(2)QP_O8[1]", 1), ("(2)QP_O8[1]", 2)]
OPS_TRI = [("(1)Q1_3[1]", 0), ("(1)Q1_3[1]", 1), ("(1)Q1_3[1]", 2),
           ("(2)Q1_3[1]", 0), ("(2)Q1_3[1]", 1), ("(2)Q1_3[1]", 2)]
OPS_D1_TRI = [("(1)Q1_3[1]", 0), ("(1)Q1_3[1]", 1), ("(1)Q1_3[1]", 2)]
# shift advection beta^i d_i f of every field: the X_2 upwind pair along x, y, z with the velocity
# read from fields 0, 1, 2 (the three shift components)
OPS_UPWIND = [("(1)X2", 0, -1, 0), ("(1)X2", 1, -1, 1), ("(1)X2", 2, -1, 2)]
OPS_UPWIND_W = [("(1)W2", 0, -1, 0), ("(1)W2", 1, -1, 1), ("(1)W2", 2, -1, 2)]


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


def result_parts(sched):
    """Partitions per line class of a schedule, as N:xlines:P,..."""
    return ",".join(f"{n}:{xl}:{pp}" for n, xl, pp in sched["classes"])


def run_gpu(wl, ops, dtype, steps, warmup, autotune=True, schedule=None):
    """schedule: None (autotune or defaults) or (flags, [(N, xlines, partitions), ...]) set by hand."""
    import torch
    import paper_2302_14858_amd as P
    from paper_2302_14858_amd import _lib
    from tests import helpers as H
    tdt = torch.float64 if dtype == P.CFD_F64 else torch.float32
    plan = H.make_plan(wl, ops, dtype=dtype)
    nin, nout = plan.sizes()
    x = torch.from_numpy(wl.data).to(device="cuda", dtype=tdt)
    y = torch.empty(nout, dtype=tdt, device="cuda")
    if schedule is not None:
        flags, parts = schedule
        kw = dict(persistent=bool(flags & _lib.CFD_SCHED_PERSISTENT), split_x=bool(flags & _lib.CFD_SCHED_SPLIT_X),
                  xcd=bool(flags & _lib.CFD_SCHED_XCD), concurrent=bool(flags & _lib.CFD_SCHED_CONCURRENT))
        plan.set_schedule(0, **kw)
        for N, xl, Pp in parts:
            plan.set_schedule(N, xl, Pp, **kw)
    elif autotune:
        plan.autotune(x, y)   # no cache: every run tunes on the device it runs on
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


def oracle_reference(plan, wl, ops):
    """The oracle's result for every block, field and operator, in the plan's output layout."""
    from tests import helpers as H
    _, ooffs = plan.offsets()
    _, nout = plan.sizes()
    return H.oracle_flat(wl, ops, ooffs, nout)


def err_vs_oracle(plan, y, wl, ops, ref):
    """Worst relative max-norm error over every output node (each block, field and operator)."""
    from tests import helpers as H
    _, ooffs = plan.offsets()
    return H.compare_flat(y.double().cpu().numpy(), ref, wl, ops, ooffs)


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl, ops, budget_s=12.0, one_core_s=3.0):
    """Oracle (plain C, OpenMP over lines) on a bounded sample of the same workload: all host
    threads for budget_s, and one thread for one_core_s (run first; the all-thread run then sets
    the thread count back)."""
    from oracle import lines as OL
    from oracle import schemes as OS
    schemes = {op[0]: OS.named(op[0]) for op in ops}
    threads = OL.max_threads()

    def sample(nthreads, budget):
        evals = nb = passes = 0
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < budget:
            for b, blk in enumerate(wl.blocks):
                for f in range(wl.nfields):
                    fv = wl.field_view(b, f)
                    for name, d in ops:
                        OL.apply_block(schemes[name], fv, blk.ng, blk.h[d], d, nthreads=nthreads)
                    evals += len(ops) * int(np.prod(blk.n))
                nb += 1
                if time.perf_counter() - t0 > budget:
                    break
            passes += 1
        return evals, nb, passes, time.perf_counter() - t0

    e1, nb1, _, dt1 = sample(1, one_core_s)
    evals, nb, passes, dt = sample(threads, budget_s)
    return {"value": evals / dt, "unit": "evals/s", "cores": threads, "kind": "oracle",
            "sample": f"{nb} block passes over the {len(wl.blocks)} blocks ({passes} sweeps) x {wl.nfields} "
                      f"fields x {len(ops)} ops: {evals} evals in {dt:.1f} s",
            "one_core": {"value": e1 / dt1, "unit": "evals/s",
                         "sample": f"{nb1} block passes x {wl.nfields} fields x {len(ops)} ops in {dt1:.1f} s"},
            "cpu_model": _cpu_model(), "nproc": os.cpu_count()}


def extra_block128(steps, warmup, autotune, ng=4):
    """One 128^3 block, tridiagonal tuned D1 + D2 along x, y, z, FP64: at ng = 4 with the matched
    closures, at ng = 3 with the order-only closures (:E)."""
    import torch
    import synth
    import paper_2302_14858_amd as P
    ops = OPS_TRI if ng >= 4 else [(n + ":E", d) for n, d in OPS_TRI]
    wl = synth.block128(ng=ng)
    plan, x, y, ms, _, _, _ = run_gpu(wl, ops, P.CFD_F64, steps, warmup, autotune=autotune)
    evals = wl.interior_points * wl.nfields * len(ops)
    alg, _, _ = algorithmic_bytes(wl, ops, 8)
    closure = "matched closures" if ng >= 4 else "order-only closures (:E)"
    out = {"workload": f"block128: one 128^3 block on [-1,1]^3, ng={ng}, Gaussian + N(0,1e-3) noise modes, "
                       f"(d)Q1_3[1] D1+D2 along x,y,z with {closure}, FP64",
           "ms_per_step": ms, "value": evals / (ms * 1e-3), "unit": "evals/s",
           "achieved_GBs": alg / (ms * 1e-3) / 1e9,
           "err_vs_oracle": err_vs_oracle(plan, y, wl, ops, oracle_reference(plan, wl, ops))}
    del plan, x, y
    torch.cuda.empty_cache()
    return out


def extra_upwind64(steps, warmup, autotune):
    """batch64 blocks (ng = 5), 22 fields: beta^i d_i f for every field with the X_2 upwind pair
    (left-biased where beta^i > 0, right-biased where beta^i < 0, Eq. biasderapproxadv), FP64 and FP32;
    then the W_2 pair (embedded compact second derivative, Tab. ccuw_deg_one_col) in both precisions."""
    import torch
    import synth
    import paper_2302_14858_amd as P
    wl = synth.batch64()
    evals = wl.interior_points * wl.nfields * len(OPS_UPWIND)
    out = {"workload": "upwind64: batch64 blocks (extents from {16,24,32,48}^3, ng=5), 22 fields, beta^i d_i f "
                       "with the (1)X2 upwind pair along x,y,z, beta^i = fields 0,1,2; w2_*: the same with the "
                       "(1)W2 pair (its embedded (2)P1_2 pass and scratch traffic are not algorithmic bytes)"}
    refs = {}
    for label, ops, dt, es in (("f64", OPS_UPWIND, P.CFD_F64, 8), ("f32", OPS_UPWIND, P.CFD_F32, 4),
                               ("w2_f64", OPS_UPWIND_W, P.CFD_F64, 8), ("w2_f32", OPS_UPWIND_W, P.CFD_F32, 4)):
        plan, x, y, ms, _, launches, items = run_gpu(wl, ops, dt, steps, warmup, autotune=autotune)
        alg, _, _ = algorithmic_bytes(wl, ops, es)
        key = ops[0][0]
        if key not in refs:
            refs[key] = oracle_reference(plan, wl, ops)
        ref = refs[key]
        out[label] = {"ms_per_step": ms, "value": evals / (ms * 1e-3), "unit": "evals/s",
                      "achieved_GBs": alg / (ms * 1e-3) / 1e9, "frac_of_hbm_peak": alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                      "err_vs_oracle": err_vs_oracle(plan, y, wl, ops, ref),
                      "err_scope": "every output node"}
        del plan, x, y
        torch.cuda.empty_cache()
    return out


OPS_KO = [("KO8[0.04]", 0), ("KO8[0.04]", 1), ("KO8[0.04]", 2)]
OPS_MIXED = [("(1)QP_O8[1]", 0, -1, -1, 1), ("(1)QP_O8[1]", 0, -1, -1, 2), ("(1)QP_O8[1]", 1, -1, -1, 2)]


def mixed_algorithmic_bytes(wl, esize):
    """The three mixed pairs: every field read once with its face ghosts in all three directions
    and the edge ghosts of each pair (4 ng^2 per unit length of the third direction), one output
    per pair written."""
    rd = wr = 0
    for b in wl.blocks:
        nx, ny, nz = b.n
        n3 = nx * ny * nz
        g = b.ng
        faces = 2 * g * (ny * nz + nx * nz + nx * ny)
        edges = 4 * g * g * (nz + ny + nx)
        rd += wl.nfields * (n3 + faces + edges)
        wr += 3 * wl.nfields * n3
    return (rd + wr) * esize


def extra_z4c64(steps, warmup, autotune):
    """batch64 blocks (ng = 5), 22 fields: Kreiss-Oliger Q^(8) (sigma = 0.04) along x, y, z, and
    the symmetrised mixed derivatives d_x d_y, d_x d_z, d_y d_z with (1)QP_O8[1], FP64."""
    import torch
    import synth
    import paper_2302_14858_amd as P
    wl = synth.batch64()
    out = {"workload": "z4c64: batch64 blocks (extents from {16,24,32,48}^3, ng=5), 22 fields; 'ko8': "
                       "Kreiss-Oliger Q^(8), sigma=0.04, along x,y,z; 'mixed': 1/2 (D_i D_j + D_j D_i), "
                       "(1)QP_O8[1], pairs xy, xz, yz; FP64"}
    for label, ops in (("ko8", OPS_KO), ("mixed", OPS_MIXED)):
        plan, x, y, ms, _, launches, items = run_gpu(wl, ops, P.CFD_F64, steps, warmup, autotune=autotune)
        evals = wl.interior_points * wl.nfields * len(ops)
        alg = algorithmic_bytes(wl, ops, 8)[0] if label == "ko8" else mixed_algorithmic_bytes(wl, 8)
        ref = oracle_reference(plan, wl, ops)
        out[label] = {"ms_per_step": ms, "value": evals / (ms * 1e-3), "unit": "evals/s",
                      "achieved_GBs": alg / (ms * 1e-3) / 1e9, "frac_of_hbm_peak": alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                      "kernel_launches_per_step": launches,
                      "err_vs_oracle": err_vs_oracle(plan, y, wl, ops, ref), "err_scope": "every output node"}
        del plan, x, y, ref
        torch.cuda.empty_cache()
    return out


def extra_periodic256(steps, warmup, autotune):
    """Periodic 256^3 x 8 fields, tridiagonal D1 along x, y, z: banded FP64, banded FP32, dense mixed."""
    import torch
    import synth
    import paper_2302_14858_amd as P
    wl = synth.periodic256()
    evals = wl.interior_points * wl.nfields * len(OPS_D1_TRI)
    out = {"workload": "periodic256: 256^3, 8 fields of 32 modes with k up to 120, (1)Q1_3[1] D1 along x,y,z"}
    ref = None
    for label, dt, es in (("f64_banded", P.CFD_F64, 8), ("f32_banded", P.CFD_F32, 4),
                          ("mixed_dense_bf16", P.CFD_MIXED_BF16, 4)):
        plan, x, y, ms, _, _, _ = run_gpu(wl, OPS_D1_TRI, dt, steps, warmup, autotune=autotune)
        alg, _, _ = algorithmic_bytes(wl, OPS_D1_TRI, es)
        if ref is None:
            ref = oracle_reference(plan, wl, OPS_D1_TRI)
        out[label] = {"ms_per_step": ms, "value": evals / (ms * 1e-3), "unit": "evals/s",
                      "achieved_GBs": alg / (ms * 1e-3) / 1e9,
                      "err_vs_oracle": err_vs_oracle(plan, y, wl, OPS_D1_TRI, ref),
                      "err_sample": "all 8 fields, all three directions, every node"}
        del plan, x, y
        torch.cuda.empty_cache()
    out["speedup_mixed_vs_f64"] = out["f64_banded"]["ms_per_step"] / out["mixed_dense_bf16"]["ms_per_step"]
    out["speedup_f32_vs_f64"] = out["f64_banded"]["ms_per_step"] / out["f32_banded"]["ms_per_step"]
    return out


def extra_wave192(nsteps=200):
    """RK4 of the first-order wave system on a periodic 192^3 grid, k = (3,5,7), dt = h/4.

    Two discretisations of the same domain: one periodic 192^3 block (cyclic lines), and a 4 x 4 x 4
    lattice of 48^3 blocks with N_g = 4, matched closures and a device ghost exchange every stage."""
    import torch
    import synth
    import paper_2302_14858_amd as P
    from paper_2302_14858_amd.wave import WaveRK4
    n = 192
    k = np.array(synth.WAVE_K, dtype=np.float64)
    w = float(np.sqrt(np.sum(k * k)))
    out = {"workload": f"wave192: periodic 192^3, plane wave k=(3,5,7), dt=h/4, {nsteps} RK4 steps, (1)Q1_3[1]; "
                       "'f64'/'f32': one periodic block; 'blocks_*': 64 blocks of 48^3, ng=4, closures + halo exchange; "
                       "each stage a derivative apply + the stage kernel ('*_fused': the stage folded into the "
                       "line kernels' epilogues); schedules autotuned"}
    for variant, bpd in (("", 1), ("blocks_", 4)):
        wl = synth.wave192(n=n, blocks_per_dim=bpd, ng=4)
        h = wl.blocks[0].h[0]
        dt = 0.25 * h
        T = nsteps * dt
        xs = np.arange(n) * h
        ex = [np.exp(-1j * k[a] * xs) for a in range(3)]
        exact = synth.wave_state(xs, xs, xs, T)[0]
        for label, dt_code, fused in (("f64", P.CFD_F64, False), ("f32", P.CFD_F32, False),
                                      ("f64_fused", P.CFD_F64, True), ("f32_fused", P.CFD_F32, True)):
            blocks = [dict(n=b.n, ng=b.ng, h=b.h, boundary=b.boundary) for b in wl.blocks]
            rk = WaveRK4(blocks, P.Scheme.named("(1)Q1_3[1]"), dt, dtype=dt_code,
                         lattice=(bpd,) * 3 if bpd > 1 else None, fused=fused)
            rk.load(wl.data)
            rk.plan.autotune(rk.u, rk.d)     # the plain apply's schedule (the fused stage follows it)
            rk.load(wl.data)
            rk.capture()
            rk.load(wl.data)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            rk.run(nsteps)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / nsteps
            if bpd == 1:
                phi = rk.u[: n ** 3].double().cpu().numpy().reshape(n, n, n)
            else:
                nb, ng = n // bpd, 4
                m = nb + 2 * ng
                u = rk.u.double().cpu().numpy().reshape(bpd, bpd, bpd, 5, m, m, m)[:, :, :, 0, ng:ng + nb, ng:ng + nb,
                                                                                  ng:ng + nb]
                phi = u.transpose(0, 3, 1, 4, 2, 5).reshape(n, n, n)   # (kz, z, ky, y, kx, x)
            F = np.einsum("zyx,x,y,z->", phi, ex[0], ex[1], ex[2]) / n ** 3
            F_exact = np.exp(-1j * w * T) / 2j
            dphase = float(np.angle(F / F_exact))
            l2 = float(np.sqrt(np.mean((phi - exact) ** 2)) / np.sqrt(np.mean(exact ** 2)))
            out[variant + label] = {"ms_per_step": ms, "evals_per_s": 6 * 4 * n ** 3 / (ms * 1e-3),
                                    "l2_rel_err_vs_exact": l2, "phase_err_rad": abs(dphase), "T": T}
            del rk
            torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    # the clocks settle over the first ~100 replays (0.594 ms per step after 5, 0.560 after 100)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--flags", type=int, default=None,
                    help="set the batch64 launch shape by hand (a set of CFD_SCHED_* bits) instead of autotuning")
    ap.add_argument("--parts", default="",
                    help="with --flags: partitions per class as N:xlines:P,... (as printed in config.schedule)")
    ap.add_argument("--only", choices=["block128", "periodic256", "wave192", "upwind64", "z4c64"], default=None,
                    help="run just one of the other workloads and print its JSON object (for profiling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    if args.only:
        import torch
        torch.cuda.init()
        if args.only == "block128":
            r = extra_block128(args.steps, args.warmup, not args.no_autotune)
        elif args.only == "periodic256":
            r = extra_periodic256(min(args.steps, 20), args.warmup, not args.no_autotune)
        elif args.only == "upwind64":
            r = extra_upwind64(args.steps, args.warmup, not args.no_autotune)
        elif args.only == "z4c64":
            r = extra_z4c64(args.steps, args.warmup, not args.no_autotune)
        else:
            r = extra_wave192(min(args.steps, 200))
        print(json.dumps({args.only: r}), flush=True)
        return

    import torch
    import synth
    import paper_2302_14858_amd as P
    torch.cuda.init()
    print("bench: generating batch64 workload", file=sys.stderr, flush=True)
    wl = synth.batch64()
    ops = OPS_PENTA
    evals = wl.interior_points * wl.nfields * len(ops)

    print("bench: FP64 batched step", file=sys.stderr, flush=True)
    schedule = None
    if args.flags is not None:
        parts = [tuple(int(v) for v in t.split(":")) for t in args.parts.split(",") if t]
        schedule = (args.flags, parts)
    plan, x, y, ev_ms, wall, launches, items = run_gpu(wl, ops, P.CFD_F64, args.steps, args.warmup,
                                                       autotune=not args.no_autotune, schedule=schedule)
    sched = plan.get_schedule()
    alg, rd, wr = algorithmic_bytes(wl, ops, 8)
    achieved = alg / (ev_ms * 1e-3) / 1e9
    print("bench: oracle over every block, field and operator", file=sys.stderr, flush=True)
    ref = oracle_reference(plan, wl, ops)
    err64 = err_vs_oracle(plan, y, wl, ops, ref)
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
                   "evals_per_step": evals, "kernel_launches_per_step": launches, "work_items": items,
                   "schedule": {"flags": sched["flags"],
                                "parts": result_parts(sched)}},
        "err_vs_oracle": err64,
        "err_scope": "every output node of every block, field and operator",
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": (MEASURED_TRAFFIC_BYTES if sched["flags"] == MEASURED_TRAFFIC_FLAGS and
                                 result_parts(sched) == MEASURED_TRAFFIC_PARTS and
                                 launches == MEASURED_TRAFFIC_LAUNCHES else None),
                     "algorithmic_bytes": alg, "read_bytes": rd, "write_bytes": wr},
    }
    del x, y, plan
    torch.cuda.empty_cache()
    if not args.no_extra:
        print("bench: FP32 batched step", file=sys.stderr, flush=True)
        plan, x, y, ms32, _, _, _ = run_gpu(wl, ops, P.CFD_F32, args.steps, args.warmup,
                                            autotune=not args.no_autotune)
        alg32, _, _ = algorithmic_bytes(wl, ops, 4)
        err32 = err_vs_oracle(plan, y, wl, ops, ref)
        result["extra"] = {"f32": {"value": evals / (ms32 * 1e-3), "ms_per_step": ms32, "err_vs_oracle": err32,
                                   "achieved_GBs": alg32 / (ms32 * 1e-3) / 1e9}}
        del x, y, plan
        torch.cuda.empty_cache()
        del ref
        print("bench: block128", file=sys.stderr, flush=True)
        result["extra"]["block128"] = extra_block128(args.steps, args.warmup, not args.no_autotune)
        print("bench: block128 at ng=3", file=sys.stderr, flush=True)
        result["extra"]["block128_ng3"] = extra_block128(args.steps, args.warmup, not args.no_autotune, ng=3)
        print("bench: upwind64 shift advection", file=sys.stderr, flush=True)
        result["extra"]["upwind64"] = extra_upwind64(args.steps, args.warmup, not args.no_autotune)
        print("bench: z4c64 dissipation and mixed derivatives", file=sys.stderr, flush=True)
        result["extra"]["z4c64"] = extra_z4c64(args.steps, args.warmup, not args.no_autotune)
        print("bench: periodic256 precision study", file=sys.stderr, flush=True)
        result["extra"]["periodic256"] = extra_periodic256(min(args.steps, 20), args.warmup, not args.no_autotune)
        print("bench: wave192 RK4", file=sys.stderr, flush=True)
        result["extra"]["wave192"] = extra_wave192()
    if not args.no_cpu:
        print("bench: CPU oracle sample", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(wl, ops)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
