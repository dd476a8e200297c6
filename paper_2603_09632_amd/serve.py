"""Serving form: continuous batching of render requests over resident scenes.

Scenes (Gaussian sets) stay resident in HBM.  A request names a scene, a pose
and a camera of one of the configured resolutions.  The scheduler thread admits
requests first-come first-served whenever (a) fewer than ``max_inflight`` are
on the GPU and (b) the scratch they need fits the HBM budget; requests that
arrive while others run are admitted as soon as both free up, so their work
overlaps on the device.

Scratch lives in buffer sets (projection, binning, image) keyed by (scene,
resolution) and pooled: a finished request returns its set to the pool, and
the HBM ledger counts every set that exists.  When a new set would exceed the
budget, free sets are evicted (least recently used); if none is free the
request waits.  A buffer set runs its first request eagerly and then carries a
HIP graph of project -> tile sort -> render forward, captured on its second
use; the pose enters through a 16-float device buffer (xgs_project_posed), so
a replay serves any pose.  Replays go round-robin to a pool of streams.

Results are independent of what else is in flight: every kernel of a request
reads only that request's scene and buffers, per-tile order is deterministic
and the forward pass uses no atomics, so a request renders bit-identically
alone and in a mix.
"""
from __future__ import annotations

import collections
import queue
import threading
import time
from concurrent.futures import Future
from dataclasses import dataclass, field
from typing import Optional

import numpy as np
import torch

from . import (Binning, Gaussians, Projected, alloc_binning, camera, grid_dims, xgs_project_posed,
               xgs_render_fwd, xgs_tile_sort)


@dataclass(frozen=True)
class Resolution:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float


@dataclass
class RenderResult:
    image: torch.Tensor       # [4 + C_sem, H, W] on the GPU
    final_T: torch.Tensor     # [H, W]
    latency_s: float
    queued_s: float


@dataclass
class _Request:
    rid: int
    scene: str
    res: Resolution
    viewmat: np.ndarray
    t_arrival: float
    future: Future = field(default_factory=Future)


class _BufferSet:
    """Scratch for one in-flight request of a (scene, resolution) pair."""

    def __init__(self, server: "Server", scene: str, res: Resolution, cap: int):
        g = server.scenes[scene]
        dev = server.device
        self.key = (scene, res)
        self.cam = camera(res.width, res.height, res.fx, res.fy, res.cx, res.cy, near=server.near)
        hs, ws, _, _ = grid_dims(self.cam)
        self.viewmat_host = torch.empty((4, 4), dtype=torch.float32).pin_memory()
        self.viewmat_dev = torch.zeros((4, 4), dtype=torch.float32, device=dev)
        self.proj = Projected.alloc(g.n, dev)
        self.cap = cap
        self.binning: Binning = alloc_binning(g.n, self.cap, self.cam, dev)
        self.out = torch.empty((4 + g.c_sem, hs, ws), device=dev)
        self.final_T = torch.empty((hs, ws), device=dev)
        self.n_last = torch.empty((hs, ws), dtype=torch.int32, device=dev)
        self.status_host = torch.zeros(1, dtype=torch.int32).pin_memory()
        self.graph: Optional[torch.cuda.CUDAGraph] = None
        self.uses = 0
        self.nbytes = sum(t.numel() * t.element_size() for t in (
            self.viewmat_dev, self.proj.splat, self.proj.radius, self.proj.tile_rect, self.proj.tiles_touched,
            self.binning.keys, self.binning.vals, self.binning.ranges, self.binning.workspace,
            self.binning.tile_order, self.out, self.final_T, self.n_last))
        # The fills above ran on this thread's current stream; the set is used
        # on the (non-blocking) launch streams, which wait for this event first.
        self.ready = torch.cuda.Event()
        self.ready.record()

    def enqueue(self, g: Gaussians):
        """project -> sort -> render on the current stream (also the body that
        gets captured)."""
        xgs_project_posed(g, self.cam, self.viewmat_dev, out=self.proj)
        xgs_tile_sort(self.proj, self.cam, g.n, self.binning)
        xgs_render_fwd(g, self.proj, self.binning, self.cam, out=self.out, final_T=self.final_T,
                       n_last=self.n_last)


class Server:
    """Continuous-batching render server.  ``scenes`` maps ids to resident
    Gaussians; ``submit`` returns a Future of RenderResult."""

    def __init__(self, scenes: dict[str, Gaussians], hbm_budget_bytes: int = 4 << 30, max_inflight: int = 8,
                 streams: int = 4, use_graphs: bool = True, near: float = 0.2, device=None):
        self.device = device or torch.device("cuda")
        self.scenes = scenes
        self.budget = int(hbm_budget_bytes)
        self.max_inflight = int(max_inflight)
        self.use_graphs = use_graphs
        self.near = near
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(streams)]
        self._side = torch.cuda.Stream(device=self.device)
        self._rr = 0
        self._pool: dict = collections.defaultdict(list)  # key -> free buffer sets
        self._lru: collections.OrderedDict = collections.OrderedDict()  # free sets, LRU order
        self.ledger_bytes = 0
        self.peak_ledger_bytes = 0
        self._capacity: dict = {}
        self._queue: queue.Queue = queue.Queue()
        self._pending: collections.deque = collections.deque()
        self._inflight: list = []
        self._rid = 0
        self._lock = threading.Lock()
        self._stop = threading.Event()
        self.completed: list[RenderResult] = []
        self.rejected = 0
        self.overflows = 0
        self.sets_created = 0
        self.evictions = 0
        self.graphs_captured = 0
        self._thread = threading.Thread(target=self._loop, name="xgs-serve", daemon=True)
        self._thread.start()

    # ------------------------------------------------------------ capacity
    def capacity(self, scene: str, res: Resolution) -> int:
        """Instance capacity of a new buffer set.  Until a (scene, resolution)
        pair has been measured this is a generous bound (4 instances per
        Gaussian, at least the tile count), used for admission; the first
        buffer set of a pair measures the instance count at its request's pose
        and keeps 1.5x of it.  A later overflow is detected on the device:
        the capacity grows to 1.25x of what the request needed, the undersized
        set is discarded and the request goes back to the head of the queue."""
        key = (scene, res)
        if key in self._capacity:
            return self._capacity[key]
        n = self.scenes[scene].n
        _, _, ty, tx = grid_dims(camera(res.width, res.height, res.fx, res.fy, res.cx, res.cy))
        return max(4 * n, ty * tx) + 1024

    def _measure_capacity(self, scene: str, res: Resolution, viewmat: np.ndarray) -> int:
        key = (scene, res)
        if key not in self._capacity:
            g = self.scenes[scene]
            cam = camera(res.width, res.height, res.fx, res.fy, res.cx, res.cy, near=self.near)
            # on the side stream: the host waits for this projection only,
            # not for the replays queued on the launch streams
            with torch.cuda.stream(self._side):
                vm = torch.from_numpy(viewmat).to(self.device, non_blocking=False)
                p = xgs_project_posed(g, cam, vm)
                m = int(p.tiles_touched.to(torch.int64).sum().item())
            _, _, ty, tx = grid_dims(cam)
            self._capacity[key] = max(int(1.5 * m), ty * tx) + 1024
        return self._capacity[key]

    # ----------------------------------------------------------------- api
    def submit(self, scene: str, viewmat, res: Resolution) -> Future:
        if scene not in self.scenes:
            raise KeyError(scene)
        with self._lock:
            self._rid += 1
            rid = self._rid
        req = _Request(rid, scene, res, np.asarray(viewmat, dtype=np.float32).reshape(4, 4), time.perf_counter())
        self._queue.put(req)
        return req.future

    def render_now(self, scene: str, viewmat, res: Resolution) -> RenderResult:
        return self.submit(scene, viewmat, res).result()

    def close(self):
        self._stop.set()
        self._thread.join()

    def stats(self) -> dict:
        lat = np.array([r.latency_s for r in self.completed]) * 1e3
        if len(lat) == 0:
            return {"completed": 0}
        qd = np.array([r.queued_s for r in self.completed]) * 1e3
        return {"completed": len(lat), "p50_ms": float(np.percentile(lat, 50)),
                "p99_ms": float(np.percentile(lat, 99)), "mean_ms": float(lat.mean()),
                "p50_queued_ms": float(np.percentile(qd, 50)), "p99_queued_ms": float(np.percentile(qd, 99)),
                "peak_hbm_scratch_MB": self.peak_ledger_bytes / 2 ** 20, "budget_MB": self.budget / 2 ** 20,
                "sets_created": self.sets_created, "evictions": self.evictions,
                "graphs_captured": self.graphs_captured, "overflows": self.overflows}

    # ------------------------------------------------------------ internals
    def _acquire(self, scene: str, res: Resolution, viewmat: np.ndarray) -> Optional[_BufferSet]:
        key = (scene, res)
        if self._pool[key]:
            bs = self._pool[key].pop()
            self._lru.pop(id(bs), None)
            return bs
        need = self._estimate(scene, res)
        while self.ledger_bytes + need > self.budget and self._lru:
            _, victim = self._lru.popitem(last=False)
            self._pool[victim.key].remove(victim)
            self.ledger_bytes -= victim.nbytes
            self.evictions += 1
            del victim
        if self.ledger_bytes + need > self.budget:
            return None
        bs = _BufferSet(self, scene, res, self._measure_capacity(scene, res, viewmat))
        self.sets_created += 1
        self.ledger_bytes += bs.nbytes
        self.peak_ledger_bytes = max(self.peak_ledger_bytes, self.ledger_bytes)
        return bs

    def _release(self, bs: _BufferSet):
        self._pool[bs.key].append(bs)
        self._lru[id(bs)] = bs

    def _estimate(self, scene: str, res: Resolution) -> int:
        g = self.scenes[scene]
        cap = self.capacity(scene, res)
        hs, ws, ty, tx = grid_dims(camera(res.width, res.height, res.fx, res.fy, res.cx, res.cy))
        from . import lib
        ws_bytes = int(lib.xgs_tile_sort_workspace(g.n, cap, ty * tx))
        return (64 + g.n * 48 + cap * 12 + ty * tx * 12 + 16 + ws_bytes + (4 + g.c_sem) * hs * ws * 4
                + hs * ws * 8)

    def _launch(self, req: _Request, bs: _BufferSet):
        g = self.scenes[req.scene]
        s = self.streams[self._rr % len(self.streams)]
        self._rr += 1
        bs.viewmat_host.copy_(torch.from_numpy(req.viewmat))
        with torch.cuda.stream(s):
            s.wait_event(bs.ready)
            bs.viewmat_dev.copy_(bs.viewmat_host, non_blocking=True)
            if self.use_graphs and bs.uses > 0:
                if bs.graph is None:
                    # A set is captured on its second use (a set evicted after
                    # one request never pays for a capture).  The capture runs
                    # on the launch stream itself: unlike the torch.cuda.graph
                    # context it does not synchronise the device, so requests
                    # on the other streams keep running.
                    graph = torch.cuda.CUDAGraph()
                    graph.capture_begin(capture_error_mode="thread_local")
                    try:
                        bs.enqueue(g)
                    finally:
                        graph.capture_end()
                    bs.graph = graph
                    self.graphs_captured += 1
                bs.graph.replay()
            else:
                bs.enqueue(g)
            bs.uses += 1
            image = bs.out.clone()
            final_T = bs.final_T.clone()
            bs.status_host.copy_(bs.binning.status, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(s)
        self._inflight.append((req, bs, ev, image, final_T, time.perf_counter()))

    def _finish(self, item):
        req, bs, ev, image, final_T, t_launch = item
        if int(bs.status_host.item()) != 0:
            # Capacity overflow.  The set still holds this request's
            # projection: count the instances it needed (a small reduction on
            # a side stream), grow the pair's capacity, drop the undersized
            # set and put the request back at the head of the queue, so the
            # loop never blocks on a re-render.
            with torch.cuda.stream(self._side):
                self._side.wait_event(ev)
                m = int(bs.proj.tiles_touched.to(torch.int64).sum().item())
            self._capacity[bs.key] = max(self._capacity.get(bs.key, 0), int(m * 1.25) + 1024)
            self.overflows += 1
            self.ledger_bytes -= bs.nbytes
            self._pending.appendleft(req)
            return
        t = time.perf_counter()
        res = RenderResult(image, final_T, t - req.t_arrival, t_launch - req.t_arrival)
        self.completed.append(res)
        self._release(bs)
        req.future.set_result(res)

    def _loop(self):
        while not (self._stop.is_set() and self._queue.empty() and not self._pending and not self._inflight):
            try:
                while True:
                    self._pending.append(self._queue.get_nowait())
            except queue.Empty:
                pass
            # admit in arrival order while slots and memory allow
            while self._pending and len(self._inflight) < self.max_inflight:
                req = self._pending[0]
                bs = self._acquire(req.scene, req.res, req.viewmat)
                if bs is None:
                    if not self._inflight:  # cannot fit even on an idle GPU
                        self._pending.popleft()
                        self.rejected += 1
                        req.future.set_exception(MemoryError("request scratch exceeds the HBM budget"))
                        continue
                    break
                self._pending.popleft()
                try:
                    self._launch(req, bs)
                except Exception as e:  # surface launch errors on the request
                    self._release(bs)
                    req.future.set_exception(e)
            # retire finished work
            still = []
            for item in self._inflight:
                if item[2].query():
                    self._finish(item)
                else:
                    still.append(item)
            self._inflight = still
            if not self._pending and not self._inflight:
                try:
                    self._pending.append(self._queue.get(timeout=0.001))
                except queue.Empty:
                    pass
            else:
                time.sleep(0)


def poisson_load(server: Server, requests: list, qps: float, seed: int = 48) -> list[Future]:
    """Submits (scene, viewmat, resolution) requests with exponential
    inter-arrival times at the given rate; returns their futures."""
    rng = np.random.default_rng(seed)
    futures = []
    t_next = time.perf_counter()
    for scene, vm, res in requests:
        t_next += rng.exponential(1.0 / qps)
        while True:
            now = time.perf_counter()
            if now >= t_next:
                break
            time.sleep(min(t_next - now, 0.0005))
        futures.append(server.submit(scene, vm, res))
    return futures
