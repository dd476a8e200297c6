"""Serving form: continuous batching of render requests over resident scenes.

Scenes (Gaussian sets) stay resident in HBM.  A request names a scene, a pose
and a camera of one of the configured resolutions.  Requests are rendered in
batches: a batch is one projection launch, one tile sort and one compositing
launch for all of its requests (xgs_batch_project, xgs_tile_sort over the
batch, xgs_batch_render_fwd), each request a slot with its own band of tile
rows, so the sort is keyed by (slot, tile, depth).

Batches run in arenas: fixed buffers (batch projection, binning, sort
workspace, slot table) sized once from the HBM budget, with capacities in
Gaussians, tile rows, instances and slots.  Each arena has its own stream and
carries HIP graphs of the three calls, one per capacity bucket (Gaussian rows
and tile rows rounded up to powers of two), all captured when the arena is
created; a batch rewrites the arena's device slot table (scene
pointers, pose, output pointers) and replays its bucket's graph, so any mix
of scenes, poses and resolutions within a bucket replays the same graph, and
a small batch does not pay for the full capacity.  With two arenas one batch
is formed and launched while the other runs (continuous batching): requests
that arrive while a batch is on the GPU go into the next batch as soon as an
arena frees up, first come first served, as many as fit.

Admission by memory: the arenas' bytes plus the outputs of the requests in
flight stay within the budget; a request whose scene does not fit an arena
fails with MemoryError.  A batch whose instances overflow the binning is
detected on the device (status), its requests go back to the head of the
queue with larger per-(scene, resolution) instance estimates, and an arena
grows when a single request needs more than it holds.

Results are independent of the batch: each slot's tiles hold only its own
Gaussians, per-tile order is (depth, index) and the forward pass has no
atomics, so a request renders bit-identically alone, batched, or through the
single-request calls.
"""
from __future__ import annotations

import collections
import ctypes
import gc
import queue
import threading
import time
from concurrent.futures import Future
from dataclasses import dataclass, field
from typing import Optional

import numpy as np
import torch

from . import (BatchLayout, Gaussians, Projected, XgsBatchSlot, alloc_binning, batch_table, camera, grid_dims,
               lib, xgs_batch_check, xgs_batch_project, xgs_batch_render_fwd, xgs_tile_sort)

TILES_X = 75               # virtual grid width: the widest resolution served (1200 px) in tiles
ORDER_TILES = 16384        # the tile sort orders up to this many tiles longest-first
G_BUCKET0 = 1 << 16        # smallest Gaussian-row bucket of a batch
R_BUCKET0 = 16             # smallest tile-row bucket of a batch


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
    image: Optional[torch.Tensor]    # [4 + C_sem, H, W] on the GPU (None when discarded)
    final_T: Optional[torch.Tensor]  # [H, W]
    latency_s: float
    queued_s: float


@dataclass
class _Request:
    rid: int
    scene: str
    res: Resolution
    viewmat: np.ndarray
    t_arrival: float
    discard: bool = False
    future: Future = field(default_factory=Future)


def _bucket(value: int, top: int, first: int) -> int:
    """Smallest of first, 2 first, 4 first, ... that is >= value, at most top."""
    b = first
    while b < value and b < top:
        b *= 2
    return min(b, top)


class _Arena:
    """Buffers, stream and graphs of one batch in flight.  Launch grids cover
    a capacity bucket (Gaussian rows and tile rows rounded up to a power-of-two
    multiple), one graph per bucket, so a small batch does not pay for the
    arena's full capacity."""

    def __init__(self, server: "Server", cap_gaussians: int, tile_rows: int, max_instances: int):
        dev = server.device
        self.server = server
        self.cap_gaussians, self.tile_rows, self.max_instances = cap_gaussians, tile_rows, max_instances
        self.stream = torch.cuda.Stream(device=dev)
        self.proj = Projected.alloc(cap_gaussians, dev)
        full = BatchLayout(TILES_X, tile_rows, cap_gaussians, [], [])
        self.binning = alloc_binning(cap_gaussians, max_instances, full.sort_camera(), dev)
        slot_bytes = ctypes.sizeof(XgsBatchSlot)
        self.h_table = torch.zeros(server.max_slots * slot_bytes, dtype=torch.uint8).pin_memory()
        self.d_table = torch.zeros(server.max_slots * slot_bytes, dtype=torch.uint8, device=dev)
        self.status_host = torch.zeros(1, dtype=torch.int32).pin_memory()
        self.graphs: dict = {}
        self.uses: collections.Counter = collections.Counter()
        self.batches = 0
        self.busy = None            # (requests, layout, outputs, event, t_launch, output bytes) while a batch runs
        self.nbytes = sum(t.numel() * t.element_size() for t in (
            self.proj.splat, self.proj.radius, self.proj.tile_rect, self.proj.tiles_touched, self.binning.keys,
            self.binning.vals, self.binning.ranges, self.binning.workspace, self.binning.tile_order, self.d_table))
        self.ready = torch.cuda.Event()
        self.ready.record()

    @staticmethod
    def bytes_for(cap_gaussians: int, tile_rows: int, max_instances: int, max_slots: int) -> int:
        tiles = TILES_X * tile_rows
        ws = int(lib.xgs_tile_sort_workspace(cap_gaussians, max_instances, tiles))
        return (cap_gaussians * 48 + max_instances * 12 + tiles * 12 + ws + 16
                + max_slots * ctypes.sizeof(XgsBatchSlot))

    def bucket(self, gaussians: int, rows: int) -> tuple:
        return (_bucket(gaussians, self.cap_gaussians, G_BUCKET0), _bucket(rows, self.tile_rows, R_BUCKET0))

    def buckets(self) -> list:
        out, g = [], G_BUCKET0
        while True:
            r = R_BUCKET0
            while True:
                out.append((min(g, self.cap_gaussians), min(r, self.tile_rows)))
                if r >= self.tile_rows:
                    break
                r *= 2
            if g >= self.cap_gaussians:
                break
            g *= 2
        return out

    def empty_table(self, key: tuple):
        """Slot table with every slot unused (no Gaussians, no tile rows)."""
        full = (XgsBatchSlot * self.server.max_slots)()
        for k in range(self.server.max_slots):
            full[k].cam.stride = 1
            full[k].gauss_base = key[0]
            full[k].row_base = key[1]
        return full

    def body(self, key: tuple):
        """The batch's launches on the current stream (also what is captured)."""
        s = self.server
        layout = BatchLayout(TILES_X, key[1], key[0], [], [])
        xgs_batch_project(self.d_table, s.max_slots, layout, self.proj)
        xgs_tile_sort(self.proj, layout.sort_camera(), key[0], self.binning)
        xgs_batch_render_fwd(self.d_table, s.max_slots, s.c_sem, layout, self.proj, self.binning)


class Server:
    """Continuous-batching render server.  ``scenes`` maps ids to resident
    Gaussians (one semantic channel count for all); ``submit`` returns a
    Future of RenderResult.  ``max_inflight`` is the number of slots of a
    batch, ``streams`` the number of arenas (batches in flight)."""

    def __init__(self, scenes: dict[str, Gaussians], hbm_budget_bytes: int = 4 << 30, max_inflight: int = 8,
                 streams: int = 2, use_graphs: bool = True, near: float = 0.2, device=None,
                 cap_gaussians: Optional[int] = None, max_instances: Optional[int] = None):
        self.device = device or torch.device("cuda")
        self.scenes = scenes
        c_sems = {g.c_sem for g in scenes.values()}
        if len(c_sems) != 1:
            raise ValueError("all served scenes need the same semantic channel count")
        self.c_sem = c_sems.pop()
        self.budget = int(hbm_budget_bytes)
        self.max_slots = max(1, min(int(max_inflight), 16))
        self.use_graphs = use_graphs
        self.near = near
        n_arenas = max(1, int(streams))
        largest = max(g.n for g in scenes.values())
        tile_rows = ORDER_TILES // TILES_X
        # Arena capacities: by default room for about four of the largest
        # scenes per batch (at most max_slots), within half of the budget;
        # the other half is for the outputs of the requests in flight.
        cap = int(cap_gaussians or min(4 * largest, self.max_slots * largest))
        inst = int(max_instances or 2 * cap)
        while cap > 1 and n_arenas * _Arena.bytes_for(cap, tile_rows, inst, self.max_slots) > self.budget // 2:
            cap = cap * 3 // 4
            inst = inst * 3 // 4
        self._arena_args = (cap, tile_rows, inst)
        self._n_arenas = n_arenas
        self.arenas: list[_Arena] = []
        self.ledger_bytes = 0
        self.peak_ledger_bytes = 0
        self._out_bytes = 0
        self._est: dict = {}
        self._queue: queue.Queue = queue.Queue()
        self._pending: collections.deque = collections.deque()
        self._rid = 0
        self._lock = threading.Lock()
        self._stop = threading.Event()
        self.completed: list = []           # (latency_s, queued_s) of each finished request
        self.rejected = 0
        self.overflows = 0
        self.batches = 0
        self.batched_requests = 0
        self.graphs_captured = 0
        self.arena_growths = 0
        self._thread = threading.Thread(target=self._loop, name="xgs-serve", daemon=True)
        self._thread.start()

    # ----------------------------------------------------------------- api
    def submit(self, scene: str, viewmat, res: Resolution, discard: bool = False) -> Future:
        """Queues a request.  discard: the image is rendered but not kept (the
        future's RenderResult carries the timings only), as for a client that
        consumes results as they come."""
        if scene not in self.scenes:
            raise KeyError(scene)
        with self._lock:
            self._rid += 1
            rid = self._rid
        req = _Request(rid, scene, res, np.asarray(viewmat, dtype=np.float32).reshape(4, 4), time.perf_counter(),
                       discard)
        self._queue.put(req)
        return req.future

    def render_now(self, scene: str, viewmat, res: Resolution) -> RenderResult:
        return self.submit(scene, viewmat, res).result()

    def close(self):
        self._stop.set()
        self._thread.join()

    def stats(self) -> dict:
        lat = np.array([c[0] for c in self.completed]) * 1e3
        if len(lat) == 0:
            return {"completed": 0}
        qd = np.array([c[1] for c in self.completed]) * 1e3
        return {"completed": len(lat), "p50_ms": float(np.percentile(lat, 50)),
                "p99_ms": float(np.percentile(lat, 99)), "mean_ms": float(lat.mean()),
                "p50_queued_ms": float(np.percentile(qd, 50)), "p99_queued_ms": float(np.percentile(qd, 99)),
                "peak_hbm_MB": self.peak_ledger_bytes / 2 ** 20, "budget_MB": self.budget / 2 ** 20,
                "batches": self.batches, "mean_batch": self.batched_requests / max(self.batches, 1),
                "graphs_captured": self.graphs_captured, "overflows": self.overflows,
                "arena_growths": self.arena_growths}

    # ------------------------------------------------------------ internals
    def _cam(self, res: Resolution, viewmat=None):
        return camera(res.width, res.height, res.fx, res.fy, res.cx, res.cy, viewmat=viewmat, near=self.near)

    def _out_nbytes(self, res: Resolution) -> int:
        hs, ws, _, _ = grid_dims(self._cam(res))
        return (4 + self.c_sem) * hs * ws * 4 + hs * ws * 8

    def _estimate(self, req: _Request) -> int:
        """Instance estimate of a (scene, resolution): 1.5 per Gaussian until
        an overflow measured more."""
        return self._est.get((req.scene, req.res), int(1.5 * self.scenes[req.scene].n) + 1024)

    def _charge(self, nbytes: int):
        self.ledger_bytes += nbytes
        self.peak_ledger_bytes = max(self.peak_ledger_bytes, self.ledger_bytes)

    def _ensure_arenas(self):
        while len(self.arenas) < self._n_arenas:
            a = _Arena(self, *self._arena_args)
            self._charge(a.nbytes)
            self.arenas.append(a)
            if self.use_graphs:
                self._precapture(a)

    @staticmethod
    def _capture(body) -> "torch.cuda.CUDAGraph":
        """Captures body() into a graph on the current stream.  Python's
        garbage collector runs before and not during the capture: a collection
        inside it could free a GPU tensor or event from this thread, a call the
        capture forbids (the process aborts in the destructor)."""
        gc.collect()
        was_enabled = gc.isenabled()
        gc.disable()
        try:
            graph = torch.cuda.CUDAGraph()
            graph.capture_begin(capture_error_mode="thread_local")
            try:
                body()
            finally:
                graph.capture_end()
        finally:
            if was_enabled:
                gc.enable()
        return graph

    def _precapture(self, arena: _Arena):
        """Captures every capacity bucket's graph up front (on an all-empty
        slot table), so that no capture stalls a request later."""
        with torch.cuda.stream(arena.stream):
            arena.stream.wait_event(arena.ready)
            for key in arena.buckets():
                full = arena.empty_table(key)
                ctypes.memmove(arena.h_table.data_ptr(), full, ctypes.sizeof(full))
                arena.d_table.copy_(arena.h_table, non_blocking=True)
                arena.body(key)                      # first run eager
                arena.graphs[key] = self._capture(lambda: arena.body(key))
                arena.uses[key] += 1
                self.graphs_captured += 1
                # the host table is rewritten for the next bucket only after
                # this copy has read it
                arena.stream.synchronize()

    def _form_batch(self, arena: _Arena) -> list:
        """Pending requests that fit the arena together, in arrival order."""
        batch, g_used, rows, inst, out_b = [], 0, 0, 0, 0
        while self._pending and len(batch) < self.max_slots:
            req = self._pending[0]
            n = self.scenes[req.scene].n
            _, _, ty, tx = grid_dims(self._cam(req.res))
            if n > arena.cap_gaussians or ty > arena.tile_rows or tx > TILES_X:
                self._pending.popleft()
                self.rejected += 1
                req.future.set_exception(MemoryError("request does not fit a batch arena within the HBM budget"))
                continue
            est, ob = self._estimate(req), self._out_nbytes(req.res)
            if batch and (g_used + n > arena.cap_gaussians or rows + ty > arena.tile_rows
                          or inst + est > arena.max_instances):
                break
            if self.ledger_bytes + self._out_bytes + out_b + ob > self.budget:
                if not batch and not any(a.busy for a in self.arenas):
                    self._pending.popleft()
                    self.rejected += 1
                    req.future.set_exception(MemoryError("request output exceeds the HBM budget"))
                    continue
                break
            batch.append(self._pending.popleft())
            g_used, rows, inst, out_b = g_used + n, rows + ty, inst + est, out_b + ob
        return batch

    def _launch(self, arena: _Arena, batch: list):
        dev = self.device
        cams = [self._cam(r.res, r.viewmat) for r in batch]
        gs = [self.scenes[r.scene] for r in batch]
        gb, rb, g0, r0 = [], [], 0, 0
        for g, c in zip(gs, cams):
            gb.append(g0)
            rb.append(r0)
            g0 += g.n
            r0 += grid_dims(c)[2]
        key = arena.bucket(g0, r0)
        layout = BatchLayout(TILES_X, key[1], key[0], gb, rb)
        t_launch = time.perf_counter()
        with torch.cuda.stream(arena.stream):
            arena.stream.wait_event(arena.ready)
            outs = []
            for c in cams:
                hs, ws, _, _ = grid_dims(c)
                outs.append((torch.empty((4 + self.c_sem, hs, ws), device=dev), torch.empty((hs, ws), device=dev),
                             torch.empty((hs, ws), dtype=torch.int32, device=dev)))
            table = batch_table([(g, c, *o) for g, c, o in zip(gs, cams, outs)], layout)
            xgs_batch_check(table, len(batch), layout, self.c_sem)
            full = arena.empty_table(key)             # unused slots: no Gaussians, no tile rows
            ctypes.memmove(full, table, ctypes.sizeof(XgsBatchSlot) * len(batch))
            ctypes.memmove(arena.h_table.data_ptr(), full, ctypes.sizeof(full))
            arena.d_table.copy_(arena.h_table, non_blocking=True)
            if self.use_graphs and arena.uses[key] > 0:
                if key not in arena.graphs:
                    # captured on the arena's stream on the bucket's second
                    # batch; the capture does not synchronise the device, so
                    # the other arena keeps running
                    arena.graphs[key] = self._capture(lambda: arena.body(key))
                    self.graphs_captured += 1
                arena.graphs[key].replay()
            else:
                arena.body(key)
            arena.status_host.copy_(arena.binning.status, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(arena.stream)
        arena.uses[key] += 1
        arena.batches += 1
        self.batches += 1
        self.batched_requests += len(batch)
        ob = sum(self._out_nbytes(r.res) for r in batch)
        self._out_bytes += ob
        self.peak_ledger_bytes = max(self.peak_ledger_bytes, self.ledger_bytes + self._out_bytes)
        arena.busy = (batch, layout, outs, ev, t_launch, ob)

    def _finish(self, arena: _Arena):
        batch, layout, outs, ev, t_launch, ob = arena.busy
        arena.busy = None
        self._out_bytes -= ob
        if int(arena.status_host.item()) != 0:
            # Instance overflow: measure each slot's instances from the
            # projection the arena still holds, raise the estimates, grow the
            # arena if one request alone needs more, and requeue the batch.
            self.overflows += 1
            need = [int(arena.proj.tiles_touched[gb:gb + self.scenes[r.scene].n].to(torch.int64).sum().item())
                    for r, gb in zip(batch, layout.gauss_base)]
            for r, m in zip(batch, need):
                self._est[(r.scene, r.res)] = max(self._estimate(r), int(1.25 * m) + 1024)
            if max(need) > arena.max_instances:
                self._grow(int(1.25 * max(need)) + 1024)
            self._pending.extendleft(reversed(batch))
            return
        t = time.perf_counter()
        for r, (img, fT, _) in zip(batch, outs):
            if r.discard:
                img = fT = None
            res = RenderResult(img, fT, t - r.t_arrival, t_launch - r.t_arrival)
            self.completed.append((res.latency_s, res.queued_s))
            r.future.set_result(res)

    def _grow(self, instances: int):
        """Raises the arenas' instance capacity; idle arenas below it are
        rebuilt before their next batch (_refresh)."""
        cap, rows, inst = self._arena_args
        self._arena_args = (cap, rows, max(instances, inst))

    def _refresh(self, i: int):
        arena = self.arenas[i]
        if arena.busy is not None or arena.max_instances >= self._arena_args[2]:
            return
        torch.cuda.current_stream().wait_stream(arena.stream)
        self.ledger_bytes -= arena.nbytes
        self.arenas[i] = None
        del arena
        new = _Arena(self, *self._arena_args)
        self._charge(new.nbytes)
        self.arenas[i] = new
        self.arena_growths += 1
        if self.use_graphs:
            self._precapture(new)

    def _loop(self):
        self._ensure_arenas()
        while not (self._stop.is_set() and self._queue.empty() and not self._pending
                   and not any(a.busy for a in self.arenas)):
            try:
                while True:
                    self._pending.append(self._queue.get_nowait())
            except queue.Empty:
                pass
            # retire finished batches, then fill every free arena
            for a in list(self.arenas):
                if a.busy is not None and a.busy[3].query():
                    self._finish(a)
            for i in range(len(self.arenas)):
                if self.arenas[i].busy is None and self._pending:
                    self._refresh(i)
                    a = self.arenas[i]
                    batch = self._form_batch(a)
                    if batch:
                        try:
                            self._launch(a, batch)
                        except Exception as e:  # surface launch errors on the requests
                            for r in batch:
                                r.future.set_exception(e)
            if not self._pending and not any(a.busy for a in self.arenas):
                try:
                    self._pending.append(self._queue.get(timeout=0.001))
                except queue.Empty:
                    pass
            else:
                time.sleep(0)


def poisson_load(server: Server, requests: list, qps: float, seed: int = 48, discard: bool = False) -> list[Future]:
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
        futures.append(server.submit(scene, vm, res, discard=discard))
    return futures
