"""Benchmark: projection/backprojection throughput on one MI355X.

One step = the operator pair the paper times (Section 3.1: the ray-voxel intersection projector and
the FDK-weighted backprojector) on the 512^3 workload: p = A x (Siddon, 360 angles, 512^2 detector)
then v = B p (voxel-driven FDK backprojection), inputs resident in HBM.  value = 2 * Nx Ny Nz N_angles
/ step time, in Gvoxel.proj/s.  Prints one JSON line.

The roofline entry is for the dominant kernel of the step, with algorithmic bytes under the
gather model (bytes each unit of work must read if nothing were reused):
  Siddon forward      segments * 4 B, 1.132 segments per voxel.proj at this workload
  FDK backprojection  4 bilinear taps * 4 B = 16 B per voxel.proj
divided by the kernel's average duration measured with HIP events on its stream.
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
# Siddon pieces per voxel.proj for the 512^3 / 360 / 512^2 workload (oracle count over a seeded
# sample of 20000 rays, scaled)
SIDDON_SEG_PER_VP = 1.132
BYTES_PER_VP = {"siddon": 4.0 * SIDDON_SEG_PER_VP, "fdk": 16.0}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(w, vol, proj_sample_s=8.0, bp_sample_s=8.0):
    """The FP64 oracle, as it stands, on a bounded seeded sample of the same workload."""
    import oracle
    og = oracle.Geometry.from_dict(w.geometry_dict())
    threads = oracle.get_threads()
    from paper_1905_03748_amd import inputs
    nrays_total = len(w.angles) * w.ndet[0] * w.ndet[1]
    nvox_total = int(np.prod(w.nvox))
    v64 = vol.astype(np.float64)
    # Siddon on sampled rays: grow the sample until it takes >= proj_sample_s
    n = 2000
    while True:
        idx = inputs.sample_indices(nrays_total, n, 71)
        t = time.perf_counter()
        oracle.siddon_rays(og, w.angles, idx, v64)
        dt_f = time.perf_counter() - t
        if dt_f >= proj_sample_s or n >= nrays_total:
            break
        n = int(n * min(8.0, max(1.5, 1.2 * proj_sample_s / max(dt_f, 1e-3))))
    t_fwd_full = dt_f * nrays_total / n
    nr = n
    y = np.ones((len(w.angles), w.ndet[1], w.ndet[0]))
    m = 200
    while True:
        idx = inputs.sample_indices(nvox_total, m, 72)
        t = time.perf_counter()
        oracle.bp_voxels(og, w.angles, y, idx, oracle.W_FDK)
        dt_b = time.perf_counter() - t
        if dt_b >= bp_sample_s or m >= nvox_total:
            break
        m = int(m * min(8.0, max(1.5, 1.2 * bp_sample_s / max(dt_b, 1e-3))))
    t_bp_full = dt_b * nvox_total / m
    value = 2.0 * w.voxel_proj / (t_fwd_full + t_bp_full) / 1e9
    return {"value": value, "unit": "Gvoxel·proj/s", "cores": threads, "kind": "oracle",
            "sample": f"Siddon on {nr} seeded rays ({dt_f:.1f} s) and FDK backprojection on {m} seeded voxels "
                      f"({dt_b:.1f} s) of the 512^3/360/512^2 workload, extrapolated to one full Ax + A^T y"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the build targets single-GPU boxes (no collectives); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1905_03748_amd import inputs
    from paper_1905_03748_amd.operators import Plan

    dev = torch.device("cuda:0")
    w = inputs.workload("medium")
    log(f"[bench] building phantom {w.nvox} with {w.n_ellipsoids} ellipsoids")
    vol = inputs.voxelize(w)
    plan = Plan(w.geometry_dict(), w.angles)
    x = torch.from_numpy(vol).to(dev)
    p = torch.empty(plan.proj_shape, dtype=torch.float32, device=dev)
    v = torch.empty(plan.vol_shape, dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream()

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        plan.forward(x, "siddon", out=p)
        if ev is not None:
            ev[1].record(stream)
        plan.backproject(p, "fdk", out=v)
        if ev is not None:
            ev[2].record(stream)

    log(f"[bench] warmup {args.warmup}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    log(f"[bench] timing {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(evs[k])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    fwd_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in evs]))
    bp_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in evs]))
    vp = w.voxel_proj
    value = 2.0 * vp / (ms_step * 1e-3) / 1e9
    dom = "siddon" if fwd_ms >= bp_ms else "fdk"
    dom_ms = fwd_ms if dom == "siddon" else bp_ms
    achieved = BYTES_PER_VP[dom] * vp / (dom_ms * 1e-3) / 1e9
    out = {
        "metric": "Gvoxel·proj/s for Ax and A^T y (% HBM roofline); CGLS p50/p99 served",
        "value": round(value, 3), "unit": "Gvoxel·proj/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic (seeded 40-ellipsoid phantom)",
        "config": {"workload": "512^3 volume of 0.5 mm, 360 angles over 360 deg, 512x512 detector of 0.8 mm, "
                               "DSO 1000 mm, DSD 1500 mm; step = Siddon Ax + FDK-weighted A^T y",
                   "parallelism": "single GPU"},
        "ops": {"siddon_fwd_ms": round(fwd_ms, 3), "fdk_bp_ms": round(bp_ms, 3),
                "siddon_fwd_gvps": round(vp / (fwd_ms * 1e-3) / 1e9, 2),
                "fdk_bp_gvps": round(vp / (bp_ms * 1e-3) / 1e9, 2)},
        "roofline": {"bound": "hbm", "kernel": "k_siddon" if dom == "siddon" else "k_bp_voxel<FDK>",
                     "byte_model": "gather model: %s B per voxel.proj" % BYTES_PER_VP[dom],
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None},
    }

    if not args.no_extras:
        def timed(fn, reps=3):
            fn()
            torch.cuda.synchronize()
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            for _ in range(reps):
                fn()
            b.record(stream)
            torch.cuda.synchronize()
            return a.elapsed_time(b) / reps

        log("[bench] extras")
        ex = {}
        ex["interp_fwd_ms"] = timed(lambda: plan.forward(x, "interp", out=p), 2)
        ex["pm_bp_ms"] = timed(lambda: plan.backproject(p, "pm", out=v), 2)
        ex["adjoint_bp_ms"] = timed(lambda: plan.backproject(p, "adjoint", out=v), 2)
        for k in list(ex):
            ex[k.replace("_ms", "_gvps")] = round(vp / (ex[k] * 1e-3) / 1e9, 2)
            ex[k] = round(ex[k], 3)
        xs = torch.zeros_like(x)
        r = torch.empty(4, dtype=torch.float64, device=dev)
        ws = torch.empty(plan.cgls_workspace_bytes(), dtype=torch.uint8, device=dev)
        ex["cgls_iter_ms"] = round(timed(lambda: plan.cgls(p, 3, x=xs.zero_(), resid=r, workspace=ws), 1) / 3, 3)
        out["ops"].update(ex)

    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(w, vol)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
