"""Continuous-batching reconstruction server on one GPU.

Requests (a geometry, its angles and measured projections b) each run CGLS iterations followed by
TV steepest-descent steps, entirely on the device.  The scheduler admits queued requests in
arrival order whenever a slot is free and the request's device footprint fits the HBM budget; an
admitted request gets its own stream, its projections are copied in once, and its whole
reconstruction is enqueued at once (the library's CGLS and TV keep their scalars on the device, so
nothing waits on the host).  Work of co-resident requests therefore overlaps on the GPU, and new
requests join as soon as earlier ones finish and release their memory.  An optional bound on the
summed work of co-resident requests keeps reconstructions that fill the GPU by themselves from
sharing it (their kernels are bound by cache and memory traffic, which overlap only splits), while
small requests still run side by side.

Kernels are deterministic and their launch shapes depend only on the request, so a request's
result is bitwise the same whether it runs alone or among others.
"""
from __future__ import annotations

import collections
import threading
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from .operators import Plan, tv_steps, tv_workspace_bytes


@dataclass
class Request:
    geometry: dict
    angles: np.ndarray
    b: torch.Tensor                 # host projections [n_angles, Nv, Nu], FP32 (pinned for async copy-in)
    niter: int = 10
    tv_steps: int = 5
    tv_lambda: float = 0.01
    tv_eps: float = 1e-8
    rid: int = 0
    # filled by the server
    t_submit: float = 0.0
    t_admit: float = 0.0
    t_done: float = 0.0
    x: torch.Tensor | None = None   # host result [Nz, Ny, Nx]
    resid: np.ndarray | None = None
    done: threading.Event = field(default_factory=threading.Event)

    @property
    def latency(self) -> float:
        return self.t_done - self.t_submit

    def work(self) -> float:
        return float(np.prod(self.geometry["nVoxel"])) * len(self.angles)

    def device_bytes(self) -> int:
        nx, ny, nz = self.geometry["nVoxel"]
        vol = int(nx) * int(ny) * int(nz) * 4
        proj = int(np.prod(self.b.shape)) * 4
        nv = int(self.b.shape[1])
        yq = proj // nv * (nv + 2)                         # adjoint's transposed copy (4 B per pixel)
        col = int(nx) * int(ny) * (int(nz) + 2) * 4        # projector's column-major copy
        # b, x, CGLS workspace (r, q: projections; s, p: volumes; the two copies), TV gradient,
        # small scalars
        return proj + vol + (2 * proj + 2 * vol + col + yq) + vol + (1 << 20)


class _Slot:
    def __init__(self, device):
        self.stream = torch.cuda.Stream(device=device)   # default priority
        self.req: Request | None = None
        self.event = None
        self.keep = None
        self.bytes = 0


class Server:
    """max_overlap_work: a request joins others already on the device only while their summed
    work (voxels x angles) stays within this bound, so reconstructions large enough to fill the GPU
    on their own run alone (overlapping them only makes their cache working sets compete) while
    small ones share it; None admits whenever a slot and memory are free."""

    def __init__(self, hbm_budget_bytes: int, max_slots: int = 8, device="cuda:0", max_overlap_work=None):
        self.device = torch.device(device)
        self.budget = int(hbm_budget_bytes)
        self.max_overlap_work = max_overlap_work
        self.slots = [_Slot(self.device) for _ in range(max_slots)]
        # request buffers come from one allocation stream, so blocks freed by one request are reused
        # by the next whatever its slot (each buffer is marked as used on its slot's stream, and the
        # caching allocator hands it out again only after that stream's work on it has finished)
        self.alloc_stream = torch.cuda.Stream(device=self.device)   # default priority
        self.queue: collections.deque[Request] = collections.deque()
        self.finished: list[Request] = []
        self.in_use = 0
        self.peak_in_use = 0
        self.max_queue = 0
        self.max_active = 0
        self._lock = threading.Lock()
        self._wake = threading.Event()
        self._stop = False
        self._thread = threading.Thread(target=self._loop, daemon=True)
        self._thread.start()

    # -- client side ------------------------------------------------------------------------------
    def submit(self, req: Request) -> Request:
        if req.device_bytes() > self.budget:
            raise ValueError(f"request {req.rid} needs {req.device_bytes()} B, above the HBM budget {self.budget} B")
        req.t_submit = time.perf_counter()
        with self._lock:
            self.queue.append(req)
            self.max_queue = max(self.max_queue, len(self.queue))
        self._wake.set()
        return req

    def close(self):
        self._stop = True
        self._wake.set()
        self._thread.join()

    def drain(self, timeout=None):
        t0 = time.perf_counter()
        while True:
            with self._lock:
                busy = bool(self.queue) or any(s.req is not None for s in self.slots)
            if not busy:
                return True
            if timeout is not None and time.perf_counter() - t0 > timeout:
                return False
            time.sleep(0.001)

    # -- scheduler ----------------------------------------------------------------------------------
    def _admit(self, slot: _Slot, req: Request):
        req.t_admit = time.perf_counter()
        geo = req.geometry
        plan = Plan(geo, req.angles)
        with torch.cuda.stream(self.alloc_stream):
            b = torch.empty(req.b.shape, dtype=torch.float32, device=self.device)
            x = torch.empty(plan.vol_shape, dtype=torch.float32, device=self.device)
            resid = torch.empty(req.niter + 1, dtype=torch.float64, device=self.device)
            ws = torch.empty(plan.cgls_workspace_bytes(), dtype=torch.uint8, device=self.device)
            tws = torch.empty(tv_workspace_bytes(geo), dtype=torch.uint8, device=self.device) if req.tv_steps > 0 else None
        for t in (b, x, resid, ws, tws):
            if t is not None:
                t.record_stream(slot.stream)
        with torch.cuda.stream(slot.stream):
            b.copy_(req.b, non_blocking=True)
            x.zero_()
            plan.cgls(b, req.niter, x=x, resid=resid, workspace=ws, stream=slot.stream)
            if tws is not None:
                tv_steps(geo, x, req.tv_steps, req.tv_lambda, req.tv_eps, workspace=tws, stream=slot.stream)
            xh = torch.empty(plan.vol_shape, dtype=torch.float32, pin_memory=True)
            rh = torch.empty(req.niter + 1, dtype=torch.float64, pin_memory=True)
            xh.copy_(x, non_blocking=True)
            rh.copy_(resid, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(slot.stream)
        slot.req = req
        slot.event = ev
        slot.keep = (plan, b, x, resid, ws, tws, xh, rh)

    def _finish(self, slot: _Slot):
        req = slot.req
        plan, b, x, resid, ws, tws, xh, rh = slot.keep
        req.x = xh
        req.resid = rh.numpy().copy()
        req.t_done = time.perf_counter()
        slot.req = None
        slot.event = None
        slot.keep = None
        plan.close()
        with self._lock:
            self.in_use -= slot.bytes
            self.finished.append(req)
        slot.bytes = 0
        req.done.set()

    def _loop(self):
        while not self._stop:
            progressed = False
            for s in self.slots:
                if s.req is not None and s.event is not None and s.event.query():
                    self._finish(s)
                    progressed = True
            with self._lock:
                free = [s for s in self.slots if s.req is None]
                while free and self.queue and self.in_use + self.queue[0].device_bytes() <= self.budget and \
                        self._may_overlap(self.queue[0]):
                    req = self.queue.popleft()
                    slot = free.pop()
                    # the slot is taken before the lock is released, so drain() never sees the
                    # request neither queued nor in a slot
                    slot.req = req
                    slot.bytes = req.device_bytes()
                    self.in_use += slot.bytes
                    self.peak_in_use = max(self.peak_in_use, self.in_use)
                    admit = (slot, req)
                    self._lock.release()
                    try:
                        self._admit(*admit)
                    finally:
                        self._lock.acquire()
                    progressed = True
                self.max_active = max(self.max_active, sum(1 for s in self.slots if s.req is not None))
            if not progressed:
                self._wake.wait(0.0005)
                self._wake.clear()

    def _may_overlap(self, req: Request) -> bool:
        active = [s.req.work() for s in self.slots if s.req is not None]
        if not active or self.max_overlap_work is None:
            return True
        return sum(active) + req.work() <= self.max_overlap_work

    # -- reporting --------------------------------------------------------------------------------------
    def stats(self) -> dict:
        lat = np.array([r.latency for r in self.finished])
        if len(lat) == 0:
            return {}
        t0 = min(r.t_submit for r in self.finished)
        t1 = max(r.t_done for r in self.finished)
        vp = sum(float(np.prod(r.geometry["nVoxel"])) * len(r.angles) * 2 * (r.niter + 1) for r in self.finished)
        return {"requests": len(lat), "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
                "mean_s": float(lat.mean()), "throughput_req_s": len(lat) / (t1 - t0),
                "throughput_gvps": vp / (t1 - t0) / 1e9, "peak_hbm_bytes": self.peak_in_use,
                "max_queue": self.max_queue, "max_active": self.max_active}
