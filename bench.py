"""Benchmark: projection/backprojection throughput on one MI355X.

One step = the operator pair the paper times (Section 3.1: the ray-voxel intersection projector and
the FDK-weighted backprojector) on the 512^3 workload: p = A x (Siddon, 360 angles, 512^2 detector)
then v = B p (voxel-driven FDK backprojection), inputs resident in HBM.  value = 2 * Nx Ny Nz N_angles
/ step time, in Gvoxel.proj/s.  Prints one JSON line.

The roofline entry is for the dominant kernel of the step, with algorithmic bytes under the
gather model (bytes each unit of work must read if nothing were reused):
  Siddon forward      segments * 4 B, 1.133 segments per voxel.proj at this workload
  FDK backprojection  4 bilinear taps * 4 B = 16 B per voxel.proj
divided by the kernel's average duration measured with HIP events on its stream.  The model counts no
reuse, so the caches can carry a kernel past 100 % of it; the bytes that actually leave L2, and the
unit that the counters show busiest, are printed beside it from the committed counter record.
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
# Siddon pieces per voxel.proj for the 512^3 / 360 / 512^2 workload: the oracle's count over a seeded
# sample of rays, stored by tests/golden/make_siddon_segments.py (and re-checked by the CPU tests)
SIDDON_SEG_PER_VP = json.load(open(os.path.join(ROOT, "tests", "golden", "siddon_segments.json")))["pieces_per_voxel_proj"]
BYTES_PER_VP = {"siddon": 4.0 * SIDDON_SEG_PER_VP, "fdk": 16.0}


def kernel_source_hash(name):
    import hashlib
    path = os.path.join(ROOT, "paper_1905_03748_amd", "csrc", name)
    return hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]


def recorded_traffic(kernel_key):
    """Counter figures of a kernel per launch from the committed counter runs (profiles/traffic.json):
    bytes between L2 and the memory fabric summed over the size-resolved request counters
    (32/64/128-byte reads, 32/64-byte writes), with no calibration factor, plus L2 hit rate and the
    busy fractions of the vector ALU and the texture-address unit.  None when the kernel's source has
    changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path)).get(kernel_key)
    if not rec or rec.get("source_sha256") != kernel_source_hash(rec["source"]):
        return None
    return rec


def A_sart_ws(plan, block=1):
    return plan.sart_workspace_bytes(block)


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
    cpu = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": value, "unit": "Gvoxel·proj/s", "cores": threads, "kind": "oracle",
            "host": {"cpu_model": cpu, "nproc": len(os.sched_getaffinity(0)), "os_cpu_count": os.cpu_count()},
            "sample": f"Siddon on {nr} seeded rays ({dt_f:.1f} s) and FDK backprojection on {m} seeded voxels "
                      f"({dt_b:.1f} s) of the 512^3/360/512^2 workload, extrapolated to one full Ax + A^T y"}


def serving_bench(dev, n_requests=12, seed=7, slots=8):
    """Reconstruction requests (10 CGLS iterations + 5 TV steps each) with volumes uniform in
    {128,192,256,384,512}^3 and angle counts uniform in {90,180,360,720}: one-at-a-time capacity,
    continuous batching of the same set, and Poisson arrivals at 0.9x the one-at-a-time capacity."""
    import torch
    from paper_1905_03748_amd import inputs
    from paper_1905_03748_amd.operators import Plan
    from paper_1905_03748_amd.serve import Request, Server

    rng = np.random.default_rng(seed)
    sizes = rng.choice([128, 192, 256, 384, 512], n_requests)
    angs = rng.choice([90, 180, 360, 720], n_requests)
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    reqs = []
    for r, (n, na) in enumerate(zip(sizes, angs)):
        w = inputs.workload(f"serve_{int(n)}", n_angles=int(na), seed=1000 + r)
        x = inputs.voxelize_torch(w, device=dev)
        plan = Plan(w.geometry_dict(), w.angles)
        p = plan.forward(x, "siddon")
        # photon noise, 1e5 photons per ray (densities read as 1/cm, lengths in mm)
        counts = torch.poisson(1e5 * torch.exp(-p / 10.0), generator=gen).clamp_min(1.0)
        b = (-10.0 * torch.log(counts / 1e5)).float().cpu().pin_memory()
        plan.close()
        reqs.append(Request(w.geometry_dict(), w.angles, b, niter=10, tv_steps=5, tv_lambda=0.01, rid=r))
    torch.cuda.synchronize()

    def clone(q):
        return Request(q.geometry, q.angles, q.b, niter=q.niter, tv_steps=q.tv_steps, tv_lambda=q.tv_lambda, rid=q.rid)

    budget = 200 << 30
    out = {"requests": n_requests, "mix": [f"{int(n)}^3 x {int(a)}" for n, a in zip(sizes, angs)],
           "per_request": "10 CGLS iterations + 5 TV steps (lambda 0.01)", "hbm_budget_gib": budget >> 30}
    # warm the allocator and kernels once
    srv = Server(budget, max_slots=1, device=dev)
    srv.submit(clone(reqs[0])).done.wait()
    srv.close()
    # "_fit": a request joins running ones only while their summed work stays within one
    # 256^3 x 360 reconstruction (larger ones fill the GPU alone)
    fit = 256.0 ** 3 * 360
    modes = (("one_at_a_time", 1, None), ("batched_2", 2, None), ("batched_4", 4, None), ("batched_8", 8, None),
             ("batched_4_fit", 4, fit), ("batched_8_fit", 8, fit))
    for name, nslots, lim in modes:
        srv = Server(budget, max_slots=nslots, device=dev, max_overlap_work=lim)
        t0 = time.perf_counter()
        for q in reqs:
            srv.submit(clone(q))
        srv.drain()
        dt = time.perf_counter() - t0
        st = srv.stats()
        srv.close()
        log(f"[bench] serving {name}: {dt:.2f} s")
        out[name] = {"slots": nslots, "max_overlap_work": lim, "wall_s": round(dt, 3),
                     "throughput_req_s": round(n_requests / dt, 3),
                     "p50_s": round(st["p50_s"], 3), "p99_s": round(st["p99_s"], 3),
                     "throughput_gvps": round(st["throughput_gvps"], 1), "max_active": st["max_active"]}
    cap = out["one_at_a_time"]["throughput_req_s"]
    best = max((m[0] for m in modes[1:]), key=lambda k: out[k]["throughput_req_s"])
    slots, lim = out[best]["slots"], out[best]["max_overlap_work"]
    # Poisson arrivals (seeded exponential gaps) at 0.5x, 0.9x and 1.2x the one-at-a-time capacity
    loads = {}
    for load in (0.5, 0.9, 1.2):
        qps = load * cap
        gaps = np.random.default_rng(seed + 1).exponential(1.0 / qps, n_requests)
        srv = Server(budget, max_slots=slots, device=dev, max_overlap_work=lim)
        t0 = time.perf_counter()
        for q, g in zip(reqs, np.cumsum(gaps)):
            while time.perf_counter() - t0 < g:
                time.sleep(0.0005)
            srv.submit(clone(q))
        srv.drain()
        st = srv.stats()
        srv.close()
        log(f"[bench] serving poisson at {load}x capacity: p50 {st['p50_s']:.2f} s, p99 {st['p99_s']:.2f} s")
        loads[str(load)] = {"qps": round(qps, 3), "load": load, "mode": best, "slots": slots,
                            "p50_s": round(st["p50_s"], 3), "p99_s": round(st["p99_s"], 3),
                            "max_active": st["max_active"], "peak_hbm_gib": round(st["peak_hbm_bytes"] / 2 ** 30, 2)}
    out["poisson"] = loads["0.9"]
    out["poisson_loads"] = loads
    out["batched_vs_one_at_a_time"] = round(out[best]["throughput_req_s"] / cap, 3)
    out["best_batched_mode"] = best
    # a second, separate mix of small requests, which do not fill the GPU on their own
    small = []
    for r in range(24):
        n, na = (128, 90) if r % 2 == 0 else (128, 180)
        w = inputs.workload(f"serve_{n}", n_angles=na, seed=2000 + r)
        x = inputs.voxelize_torch(w, device=dev)
        plan = Plan(w.geometry_dict(), w.angles)
        b = plan.forward(x, "siddon").cpu().pin_memory()
        plan.close()
        small.append(Request(w.geometry_dict(), w.angles, b, niter=10, tv_steps=5, tv_lambda=0.01, rid=100 + r))
    torch.cuda.synchronize()
    sm = {"requests": len(small), "mix": "128^3 x 90 and 128^3 x 180, alternating; same per-request work"}
    for name, nslots in (("one_at_a_time", 1), ("batched_4", 4), ("batched_8", 8)):
        srv = Server(budget, max_slots=nslots, device=dev)
        t0 = time.perf_counter()
        for q in small:
            srv.submit(clone(q))
        srv.drain()
        dt = time.perf_counter() - t0
        st = srv.stats()
        srv.close()
        log(f"[bench] serving small requests {name}: {dt:.2f} s")
        sm[name] = {"slots": nslots, "wall_s": round(dt, 3), "throughput_req_s": round(len(small) / dt, 3),
                    "p50_s": round(st["p50_s"], 3), "p99_s": round(st["p99_s"], 3), "max_active": st["max_active"]}
    sm["batched_vs_one_at_a_time"] = round(max(sm["batched_4"]["throughput_req_s"], sm["batched_8"]["throughput_req_s"])
                                           / sm["one_at_a_time"]["throughput_req_s"], 3)
    out["small_requests"] = sm
    return out


def precision_bench(dev, cgls_iters=20):
    """1024^3 volume, 720 angles, 1024^2 detector: FP32 vs FP16 vs BF16 storage (FP32 arithmetic).
    Speed of Ax (Siddon), A^T y (FDK, exact adjoint), relative L2 error against the FP64 oracle on
    seeded samples of rays / voxels (both against the oracle on the original FP32 inputs, which
    includes the storage rounding, and on the rounded inputs, which is the kernel error alone),
    and the CGLS reconstruction after `cgls_iters` iterations relative to the FP32 one."""
    import torch
    import oracle
    from paper_1905_03748_amd import inputs
    from paper_1905_03748_amd.operators import Plan

    w = inputs.workload("precision")
    og = oracle.Geometry.from_dict(w.geometry_dict())
    plan = Plan(w.geometry_dict(), w.angles)
    x32 = inputs.voxelize_torch(w, device=dev)
    rng = np.random.default_rng(44)
    y32 = torch.from_numpy(rng.uniform(0.0, 50.0, plan.proj_shape).astype(np.float32)).to(dev)
    ray_idx = inputs.sample_indices(int(np.prod(plan.proj_shape)), 1500, 45)
    vox_idx = inputs.sample_indices(int(np.prod(plan.vol_shape)), 300, 46)
    x_host = x32.cpu().numpy().astype(np.float64)
    y_host = y32.cpu().numpy()
    ref_ax = oracle.siddon_rays(og, w.angles, ray_idx, x_host)
    ref_bp = oracle.bp_voxels(og, w.angles, y_host.astype(np.float64), vox_idx, oracle.W_FDK)
    b = plan.forward(x32, "siddon")
    b = (b + 0.0).contiguous()

    def ms(fn, reps=2):
        fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) * 1e3 / reps

    def rel(a, r):
        return float(np.linalg.norm(a - r) / np.linalg.norm(r))

    out = {"workload": "1024^3 of 0.25 mm, 720 angles, 1024^2 detector of 0.4 mm", "dtypes": {}}
    x_ref = None
    for name, dt in (("f32", torch.float32), ("f16", torch.float16), ("bf16", torch.bfloat16)):
        log(f"[precision] {name}")
        xd = x32.to(dt)
        yd = y32.to(dt)
        p = torch.empty(plan.proj_shape, dtype=dt, device=dev)
        v = torch.empty(plan.vol_shape, dtype=dt, device=dev)
        r = {"ax_ms": round(ms(lambda: plan.forward(xd, "siddon", out=p)), 2),
             "fdk_ms": round(ms(lambda: plan.backproject(yd, "fdk", out=v)), 2),
             "adjoint_ms": round(ms(lambda: plan.backproject(yd, "adjoint", out=v), 1), 2)}
        ax = plan.forward(xd, "siddon", out=p).float().cpu().numpy().ravel()[ray_idx]
        r["ax_rel_l2_vs_fp64"] = rel(ax, ref_ax)
        r["ax_rel_l2_kernel_only"] = rel(ax, oracle.siddon_rays(og, w.angles, ray_idx,
                                                                 xd.float().cpu().numpy().astype(np.float64)))
        bp = plan.backproject(yd, "fdk", out=v).float().cpu().numpy().ravel()[vox_idx]
        r["fdk_rel_l2_vs_fp64"] = rel(bp, ref_bp)
        r["fdk_rel_l2_kernel_only"] = rel(bp, oracle.bp_voxels(og, w.angles, yd.float().cpu().numpy().astype(np.float64),
                                                               vox_idx, oracle.W_FDK))
        bd = b.to(dt)
        t = time.perf_counter()
        xr, res = plan.cgls(bd, cgls_iters, vol_dtype=dt)
        torch.cuda.synchronize()
        r["cgls_s"] = round(time.perf_counter() - t, 2)
        xr = xr.float()
        if x_ref is None:
            x_ref = xr
        r["cgls_rel_l2_vs_f32_recon"] = float(torch.linalg.vector_norm((xr - x_ref).double()) /
                                              torch.linalg.vector_norm(x_ref.double()))
        r["cgls_rel_l2_vs_phantom"] = float(torch.linalg.vector_norm((xr - x32).double()) /
                                            torch.linalg.vector_norm(x32.double()))
        out["dtypes"][name] = r
        del xd, yd, p, v, bd, xr
        torch.cuda.empty_cache()
    f32 = out["dtypes"]["f32"]
    for name in ("f16", "bf16"):
        d = out["dtypes"][name]
        d["ax_speedup_vs_f32"] = round(f32["ax_ms"] / d["ax_ms"], 3)
        d["fdk_speedup_vs_f32"] = round(f32["fdk_ms"] / d["fdk_ms"], 3)
    return out


def ooc_bench(dev, cap_gib=32):
    """3072^3 FP32 volume (108 GiB) and 3072 projections of 3072^2 (108 GiB) in pageable host memory
    (the streamer stages it through its pinned ring; a single 108 GiB pinned allocation is refused
    on the GPU machines), device memory capped at cap_gib GiB: one out-of-core Siddon Ax, one FDK and one
    exact-adjoint A^T y, then the FDK reconstruction of the same projections."""
    import torch
    from paper_1905_03748_amd import inputs
    from paper_1905_03748_amd.operators import Plan

    w = inputs.workload("ooc")
    plan = Plan(w.geometry_dict(), w.angles)
    cap = cap_gib << 30
    t = time.perf_counter()
    vol = torch.from_numpy(np.empty(plan.vol_shape, dtype=np.float32))
    proj = torch.from_numpy(np.empty(plan.proj_shape, dtype=np.float32))
    t_alloc = time.perf_counter() - t
    log("[ooc] building the phantom slab by slab")
    ells = inputs.ellipsoids(w)
    nz = w.nvox[2]
    step = 256
    for z0 in range(0, nz, step):
        h = min(step, nz - z0)
        ws = inputs.Workload("slab", (w.nvox[0], w.nvox[1], h), w.dvox, w.ndet, w.ddet, 1, 0, 0,
                             off_origin=(0.0, 0.0, (z0 + h / 2.0 - nz / 2.0) * w.dvox[2]))
        vol[z0:z0 + h].copy_(inputs.voxelize_torch(ws, ells, device=dev))
        torch.cuda.synchronize()
    out = {"workload": "3072^3 FP32 (108 GiB) volume, 3072 angles of 3072^2 (108 GiB), pageable host memory",
           "cap_gib": cap_gib, "alloc_s": round(t_alloc, 1)}
    log("[ooc] forward")
    st = plan.forward_host(vol, proj, "siddon", cap_bytes=cap)
    out["forward"] = {k: (round(v, 3) if isinstance(v, float) else v) for k, v in st.items()}
    out["forward"]["gvps"] = round(w.voxel_proj / st["t_total_s"] / 1e9, 1)
    out["forward"]["h2d_gbs"] = round(st["bytes_h2d"] / st["t_total_s"] / 1e9, 1)
    log(f"[ooc] forward done: {out['forward']}")
    log("[ooc] backprojection")
    st = plan.backproject_host(proj, vol, "fdk", cap_bytes=cap)
    out["backprojection"] = {k: (round(v, 3) if isinstance(v, float) else v) for k, v in st.items()}
    out["backprojection"]["gvps"] = round(w.voxel_proj / st["t_total_s"] / 1e9, 1)
    out["backprojection"]["h2d_gbs"] = round(st["bytes_h2d"] / st["t_total_s"] / 1e9, 1)
    log(f"[ooc] backprojection done: {out['backprojection']}")
    log("[ooc] exact adjoint")
    st = plan.backproject_host(proj, vol, "adjoint", cap_bytes=cap)
    out["adjoint"] = {k: (round(v, 3) if isinstance(v, float) else v) for k, v in st.items()}
    out["adjoint"]["gvps"] = round(w.voxel_proj / st["t_total_s"] / 1e9, 1)
    log(f"[ooc] exact adjoint done: {out['adjoint']}")
    log("[ooc] FDK reconstruction")
    st = plan.fdk_host(proj, vol, cap_bytes=cap)
    out["fdk_reconstruction"] = {k: (round(v, 3) if isinstance(v, float) else v) for k, v in st.items()}
    out["fdk_reconstruction"]["gvps"] = round(w.voxel_proj / st["t_total_s"] / 1e9, 1)
    # how close the reconstruction of the phantom's own projections comes to the phantom, in the 8
    # middle slices (where the cone angle vanishes); a property of FDK, not a parity figure
    z0 = nz // 2 - 4
    ws = inputs.Workload("mid", (w.nvox[0], w.nvox[1], 8), w.dvox, w.ndet, w.ddet, 1, 0, 0,
                         off_origin=(0.0, 0.0, (z0 + 4 - nz / 2.0) * w.dvox[2]))
    ph = inputs.voxelize_torch(ws, ells, device=dev).double()
    rec = vol[z0:z0 + 8].to(dev).double()
    out["fdk_reconstruction"]["mid_slices_rel_l2_vs_phantom"] = round(float((rec - ph).norm() / ph.norm()), 4)
    log(f"[ooc] FDK reconstruction done: {out['fdk_reconstruction']}")
    del vol, proj
    return out


def ooc_tv_bench(dev, cap_gib=32, nsteps=2):
    """TV steepest descent on the 3072^3 FP32 phantom (108 GiB, pageable host memory) under a
    cap_gib GiB device cap: the exact form (slabs with one halo slice, two passes over the image per
    step), then the halo splitting with depths 8 and 60 (one pass per round of that many steps)."""
    import torch
    from paper_1905_03748_amd import inputs
    from paper_1905_03748_amd.operators import tv_steps_host

    w = inputs.workload("ooc")
    nx, ny, nz = w.nvox
    vol = torch.from_numpy(np.empty((nz, ny, nx), dtype=np.float32))
    log("[ooc tv] building the phantom slab by slab")
    ells = inputs.ellipsoids(w)
    for z0 in range(0, nz, 256):
        h = min(256, nz - z0)
        ws = inputs.Workload("slab", (nx, ny, h), w.dvox, w.ndet, w.ddet, 1, 0, 0,
                             off_origin=(0.0, 0.0, (z0 + h / 2.0 - nz / 2.0) * w.dvox[2]))
        vol[z0:z0 + h].copy_(inputs.voxelize_torch(ws, ells, device=dev))
        torch.cuda.synchronize()
    out = {"workload": "3072^3 FP32 (108 GiB) phantom, pageable host memory", "cap_gib": cap_gib}
    # exact steps (two passes per step), then the halo splitting at depth 8 and at the paper's 60
    for depth, steps in ((0, nsteps), (8, 8), (60, 60)):
        log(f"[ooc tv] halo depth {depth}: {steps} steps")
        st = tv_steps_host(w.geometry_dict(), vol, steps, 0.01, cap_bytes=cap_gib << 30, halo_depth=depth)
        r = {"steps": steps}
        r.update({k: (round(v, 3) if isinstance(v, float) else v) for k, v in st.items()
                  if k in ("n_slabs", "slab_slices", "bytes_h2d", "bytes_d2h", "t_total_s")})
        r["s_per_step"] = round(st["t_total_s"] / steps, 2)
        r["host_link_gbs"] = round((st["bytes_h2d"] + st["bytes_d2h"]) / st["t_total_s"] / 1e9, 2)
        out["exact" if depth == 0 else f"halo_{depth}"] = r
        log(f"[ooc tv] {r}")
    del vol
    return out


def ooc_rof_bench(dev, cap_gib=32, n=2048):
    """The ROF minimiser (Chambolle's projection) on an n^3 FP32 phantom in pageable host memory under
    a cap_gib GiB device cap, its dual field in a host workspace of three volumes: halo depths 8 and
    60 (iterations per round).  n = 2048 because at 3072^3 the image and its dual field need 432 GB
    of host memory."""
    import torch
    from paper_1905_03748_amd import inputs
    from paper_1905_03748_amd.operators import rof_host

    base = inputs.workload("ooc")
    w = inputs.scaled_workload(base, (n, n, n), (n, n), 1, name=f"rof_{n}")
    ells = inputs.ellipsoids(base)
    nx, ny, nz = w.nvox
    vol = torch.from_numpy(np.empty((nz, ny, nx), dtype=np.float32))
    log(f"[ooc rof] building the {n}^3 phantom slab by slab")
    for z0 in range(0, nz, 256):
        h = min(256, nz - z0)
        ws = inputs.Workload("slab", (nx, ny, h), w.dvox, w.ndet, w.ddet, 1, 0, 0,
                             off_origin=(0.0, 0.0, (z0 + h / 2.0 - nz / 2.0) * w.dvox[2]))
        vol[z0:z0 + h].copy_(inputs.voxelize_torch(ws, ells, device=dev))
        torch.cuda.synchronize()
    work = torch.empty(3 * vol.numel() * 4, dtype=torch.uint8)
    out = {"workload": f"{n}^3 FP32 phantom ({vol.numel() * 4 / 2**30:.0f} GiB), pageable host memory; dual field "
                       f"in a {work.numel() / 2**30:.0f} GiB host workspace", "cap_gib": cap_gib}
    for depth, iters in ((8, 16), (60, 60)):
        log(f"[ooc rof] halo depth {depth}: {iters} iterations")
        st = rof_host(w.geometry_dict(), vol, iters, 0.05, halo_depth=depth, cap_bytes=cap_gib << 30, workspace=work)
        r = {"iterations": iters}
        r.update({k: (round(v, 3) if isinstance(v, float) else v) for k, v in st.items()
                  if k in ("n_slabs", "slab_slices", "bytes_h2d", "bytes_d2h", "t_total_s")})
        r["s_per_iteration"] = round(st["t_total_s"] / iters, 3)
        r["host_link_gbs"] = round((st["bytes_h2d"] + st["bytes_d2h"]) / st["t_total_s"] / 1e9, 2)
        out[f"halo_{depth}"] = r
        log(f"[ooc rof] {r}")
    del vol, work
    return out


def views_bench(dev, reps=3):
    """Operator times on the 512^3 workload's grid and detector with per-view geometry: a helical scan
    (360 views over one turn, 40 mm pitch) and a C-arm scan (360 views, detectors turned by up to
    10 degrees, sources and detectors displaced by up to 5 mm, orbit tilted by 5 degrees), against
    the circular orbit of the same angles."""
    import torch
    from paper_1905_03748_amd import inputs
    from paper_1905_03748_amd.operators import Plan

    w = inputs.workload("medium")
    vol = inputs.voxelize(w)
    x = torch.from_numpy(vol).to(dev)
    stream = torch.cuda.current_stream()
    sets = {"circular": w.angles,
            "helical": inputs.helical_views(w.DSO, w.DSD, w.angles, pitch=40.0, z0=-20.0),
            "carm": inputs.carm_views(w.DSO, w.DSD, w.angles, 7, tilt_deg=10.0, jitter_mm=5.0, orbit_tilt_deg=5.0)}
    out = {"workload": "512^3 volume of 0.5 mm, 360 views, 512x512 detector of 0.8 mm, DSO 1000 mm, DSD 1500 mm"}
    for name, ang in sets.items():
        plan = Plan(w.geometry_dict(), ang)
        p = torch.empty(plan.proj_shape, dtype=torch.float32, device=dev)
        v = torch.empty(plan.vol_shape, dtype=torch.float32, device=dev)
        r = {}
        for op, fn in (("siddon_fwd", lambda: plan.forward(x, "siddon", out=p)),
                       ("interp_fwd", lambda: plan.forward(x, "interp", out=p)),
                       ("fdk_bp", lambda: plan.backproject(p, "fdk", out=v)),
                       ("pm_bp", lambda: plan.backproject(p, "pm", out=v)),
                       ("adjoint_bp", lambda: plan.backproject(p, "adjoint", out=v))):
            log(f"[views] {name} {op}")
            fn()
            torch.cuda.synchronize()
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            for _ in range(reps):
                fn()
            b.record(stream)
            torch.cuda.synchronize()
            ms = a.elapsed_time(b) / reps
            r[op + "_ms"] = round(ms, 3)
            r[op + "_gvps"] = round(w.voxel_proj / (ms * 1e-3) / 1e9, 1)
        out[name] = r
        log(f"[views] {name}: {r}")
        del plan, p, v
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--precision", action="store_true", help="print the 16-bit storage report instead")
    ap.add_argument("--ooc", action="store_true", help="print the 3072^3 out-of-core report instead")
    ap.add_argument("--ooc-tv", action="store_true", help="print the 3072^3 out-of-core TV report instead")
    ap.add_argument("--ooc-rof", action="store_true", help="print the 2048^3 out-of-core ROF report instead")
    ap.add_argument("--views", action="store_true", help="print operator times with helical and C-arm views instead")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 1 GiB copy (ct_convert F32->F32) for HBM counter calibration")
    ap.add_argument("--profile-kernels", action="store_true",
                    help="only launch each resident operator of the 512^3 workload (Siddon and interpolated "
                         "forward, FDK, pseudo-matched and exact-adjoint backprojection, and the per-view Siddon, "
                         "FDK and adjoint kernels on a C-arm scan) --steps times after one warm-up, and a 1 GiB "
                         "plain copy, for rocprofv3 counter runs; prints nothing else")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the build targets single-GPU boxes (no collectives); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1905_03748_amd import inputs
    from paper_1905_03748_amd.operators import Plan

    dev = torch.device("cuda:0")
    if args.precision:
        print(json.dumps({"precision": precision_bench(dev)}), flush=True)
        return
    if args.ooc:
        print(json.dumps({"out_of_core": ooc_bench(dev)}), flush=True)
        return
    if args.ooc_tv:
        print(json.dumps({"out_of_core_tv": ooc_tv_bench(dev)}), flush=True)
        return
    if args.ooc_rof:
        print(json.dumps({"out_of_core_rof": ooc_rof_bench(dev)}), flush=True)
        return
    if args.views:
        print(json.dumps({"views": views_bench(dev)}), flush=True)
        return
    w = inputs.workload("medium")
    log(f"[bench] building phantom {w.nvox} with {w.n_ellipsoids} ellipsoids")
    vol = inputs.voxelize(w)
    plan = Plan(w.geometry_dict(), w.angles)
    x = torch.from_numpy(vol).to(dev)
    p = torch.empty(plan.proj_shape, dtype=torch.float32, device=dev)
    v = torch.empty(plan.vol_shape, dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream()

    if args.profile_kernels:
        from paper_1905_03748_amd.operators import convert
        ops = [("siddon", lambda: plan.forward(x, "siddon", out=p)), ("interp", lambda: plan.forward(x, "interp", out=p)),
               ("fdk", lambda: plan.backproject(p, "fdk", out=v)), ("pm", lambda: plan.backproject(p, "pm", out=v)),
               ("adjoint", lambda: plan.backproject(p, "adjoint", out=v))]
        # the per-view kernels on a C-arm scan of the same grid, detector and angles
        pv = Plan(w.geometry_dict(), inputs.carm_views(w.DSO, w.DSD, w.angles, 7, tilt_deg=10.0, jitter_mm=5.0,
                                                          orbit_tilt_deg=5.0))
        ops += [("views_siddon", lambda: pv.forward(x, "siddon", out=p)),
                ("views_fdk", lambda: pv.backproject(p, "fdk", out=v)),
                ("views_adjoint", lambda: pv.backproject(p, "adjoint", out=v))]
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        ops.append(("copy_1gib", lambda: convert(src, torch.float32)))
        for name, fn in ops:
            log(f"[bench] profile {name}")
            for _ in range(1 + args.steps):
                fn()
            torch.cuda.synchronize()
        print(json.dumps({"profile_kernels": [n for n, _ in ops], "launches_each": 1 + args.steps}), flush=True)
        return

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
        "roofline": {"bound": "hbm",
                     "kernel": "k_siddon_col<float, float, 2>" if dom == "siddon" else "k_bp_lds<0, 37, float, float>",
                     "byte_model": "gather model: %s B per voxel.proj x %.4g voxel.proj per launch"
                                   % (round(BYTES_PER_VP[dom], 3), vp),
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None},
    }
    rec = recorded_traffic("siddon_fwd" if dom == "siddon" else "fdk_bp")
    if rec is not None:
        gb = (rec["read_bytes"] + rec["write_bytes"]) / 1e9
        rl = out["roofline"]
        rl["traffic"] = round(gb, 2)
        rl["traffic_unit"] = ("GB per launch between L2 and the memory fabric (size-resolved TCC_EA0 read and "
                              "write requests, no calibration factor; an upper bound on HBM bytes, since the "
                              "last-level cache may serve some; %s)" % rec["profile"])
        # what the counters say bounds the kernel: the busiest of the L2-miss stream (against HBM peak),
        # the vector ALU and the texture-address unit that issues every gather
        miss = gb / (dom_ms * 1e-3) / 1e3 / (HBM_PEAK_GBS / 1e3)
        busy = {"texture_address_unit": rec["ta_busy"], "vector_alu": rec["valu"], "l2_miss_bytes_vs_hbm_peak": round(miss, 3)}
        rl["limiter"] = {"unit": max(busy, key=busy.get), "busy": busy, "l2_hit": rec["l2_hit"],
                         "counters_avg_ms": rec["avg_ms"]}

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
        r = torch.empty(8, dtype=torch.float64, device=dev)
        ws = torch.empty(plan.cgls_workspace_bytes(), dtype=torch.uint8, device=dev)
        t1 = timed(lambda: plan.cgls(p, 1, x=xs.zero_(), resid=r, workspace=ws), 1)
        t4 = timed(lambda: plan.cgls(p, 4, x=xs.zero_(), resid=r, workspace=ws), 1)
        ex["cgls_iter_ms"] = round((t4 - t1) / 3, 3)
        sws = torch.empty(A_sart_ws(plan), dtype=torch.uint8, device=dev)
        ex["sart_sweep_ms"] = round(timed(lambda: plan.sart(p, 1, x=xs.zero_(), workspace=sws), 1), 3)
        ows = torch.empty(A_sart_ws(plan, 10), dtype=torch.uint8, device=dev)
        ex["os_sart10_sweep_ms"] = round(timed(lambda: plan.sart(p, 1, x=xs.zero_(), block=10, workspace=ows), 1), 3)
        del ows
        from paper_1905_03748_amd.operators import tv_steps, tv_workspace_bytes
        tws = torch.empty(tv_workspace_bytes(plan.geometry), dtype=torch.uint8, device=dev)
        xt = x.clone()
        ex["tv_5steps_ms"] = round(timed(lambda: tv_steps(plan.geometry, xt, 5, 0.01, workspace=tws), 1), 3)
        from paper_1905_03748_amd.operators import rof, rof_workspace_bytes
        rws = torch.empty(rof_workspace_bytes(plan.geometry), dtype=torch.uint8, device=dev)
        ex["rof_10iter_ms"] = round(timed(lambda: rof(plan.geometry, xt, 10, 0.05, workspace=rws), 1), 3)
        del rws
        fq = torch.empty(plan.proj_shape, dtype=torch.float32, device=dev)
        ex["fdk_filter_ms"] = round(timed(lambda: plan.fdk_filter(p, out=fq), 2), 3)
        ex["fdk_recon_ms"] = round(timed(lambda: plan.fdk(p, out=v, workspace=fq.view(torch.uint8)), 2), 3)
        del fq
        out["ops"].update(ex)

    if not args.no_serving:
        log("[bench] serving")
        out["serving"] = serving_bench(dev)
        out["serving_p50_s"] = out["serving"]["poisson"]["p50_s"]
        out["serving_p99_s"] = out["serving"]["poisson"]["p99_s"]

    if args.copy_calibration:
        from paper_1905_03748_amd.operators import convert
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        convert(src, torch.float32)
        torch.cuda.synchronize()

    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(w, vol)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
