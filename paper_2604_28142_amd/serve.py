"""Encode service: assigns and PQ-encodes newly arriving documents against a
resident token-aware index (centroids, centroid offsets and PQ codebooks stay
in HBM).

Continuous batching.  A scheduler thread admits waiting requests into the next
batch while the earlier batches are still on the GPU: a batch is formed as soon
as a stream slot is free, from every admitted request that fits (at most
`max_docs` documents and `max_rows` vectors), and a ledger of device memory
bounds what the batches in flight hold: the executor charges each batch the
device bytes it occupies (its rows' buffers and the assignment's workspace for
that many rows), and a request that does not fit the remaining budget waits,
it is never dropped.  Each slot owns a libtac context on its own HIP stream and
pinned staging buffers, so the copies and kernels of consecutive batches
overlap.  A completion thread waits for batches in launch order, splits their
outputs per document and resolves the futures.

Graph replay (optional, `graphs=True`).  A batch's assignment and encoding are
a fixed sequence of about twenty kernels.  The GPU executor can capture, per
slot, one HIP graph of those kernels per row bucket (powers of two up to the
slot's capacity) and replay the graph of the smallest bucket that holds the
batch; measured on an MI355X it was no faster than launching the kernels (a
one-slot batch of 8 documents 0.545 vs 0.532 ms, of 512 documents 3.82 vs
3.60 ms): the dependent kernels' dispatch gaps stay inside the graph, and the
padded rows cost sorting time, so eager launches are the default.
The copies stay outside the graph, sized to the batch: its rows in, its
results out, and the bucket's token ids, whose rows past the batch carry id -1,
which the assignment marks unassigned and the encoder skips, so the batch's own
rows are computed exactly as in an eager launch.

Every output row is the canonical argmin for that row alone (assignment and
PQ codes), so a document's result is bitwise the same alone or in any batch.
A document with a token that has no centroid (or an id outside [0, T)) fails
on its own with TacError(TAC_E_UNSEEN_TOKEN); the rest of its batch succeeds.

Garbage collection.  Every request allocates a future, a request and a result
record; with Python's default thresholds the cyclic collector then runs full
collections over every long-lived object of the process (the caller's data
included) in the middle of serving, which showed as tail latencies of tens of
milliseconds.  By default the first running service therefore freezes the
objects alive at its start (gc.freeze) and raises the collector's first
threshold; the last one to close restores both.
"""
from __future__ import annotations

import gc
import queue
import threading
import time
from collections import deque
from concurrent.futures import Future
from dataclasses import dataclass, field

import numpy as np

ROW_BYTES = 128 * 4 + 4 + 4 + 32 + 4   # staged per vector: x, token, assignment, codes, norm

GC_THRESHOLD0 = 50_000                 # first-generation threshold while a service runs

_gc_lock = threading.Lock()
_gc_users = 0
_gc_saved = None


def _gc_acquire():
    global _gc_users, _gc_saved
    with _gc_lock:
        if _gc_users == 0:
            _gc_saved = gc.get_threshold()
            gc.collect()
            gc.freeze()
            gc.set_threshold(max(GC_THRESHOLD0, _gc_saved[0]), *_gc_saved[1:])
        _gc_users += 1


def _gc_release():
    global _gc_users
    with _gc_lock:
        _gc_users -= 1
        if _gc_users == 0:
            gc.set_threshold(*_gc_saved)
            gc.unfreeze()


@dataclass
class ResidentIndex:
    """What the service keeps in HBM: centroids [K, 128], centroid offsets
    [T + 1] and PQ codebooks [M, 256, 4] (torch tensors on the GPU)."""
    T: int
    K: int
    C: object
    cent_off: object
    codebooks: object


@dataclass
class Request:
    x: np.ndarray            # float32[n_d, 128]
    tok: np.ndarray          # int32[n_d]
    future: Future
    t_arrival: float
    t_done: float = 0.0
    rid: int = 0


@dataclass
class Result:
    assign: np.ndarray       # int32[n_d]: global centroid id
    codes: np.ndarray        # uint8[n_d, M]
    rnorm: np.ndarray        # float32[n_d]: residual norm
    latency: float = 0.0     # seconds from submit to completion


@dataclass
class ServiceStats:
    latencies: list = field(default_factory=list)     # seconds, per completed request
    batches: int = 0
    docs: int = 0
    vectors: int = 0
    failed: int = 0
    batch_sizes: list = field(default_factory=list)

    def percentile(self, q: float) -> float:
        return float(np.percentile(np.asarray(self.latencies), q)) if self.latencies else float("nan")


def row_buckets(max_rows: int, smallest: int = 1024) -> list:
    """Row counts of the replayed graphs: powers of two from `smallest`, and max_rows last."""
    out, b = [], smallest
    while b < max_rows:
        out.append(b)
        b *= 2
    out.append(max_rows)
    return out


class GpuExecutor:
    """Runs batches on the GPU through libtac; one context, stream and set of
    staging buffers per slot.  Each context holds the resident index's
    centroids prepared once (tac_ctx_set_static_centroids), so a batch's
    assignment does not re-derive norms and 16-bit rows from all K centroids.
    With `graphs`, every slot replays a captured graph per row bucket
    (see row_buckets) instead of launching the batch's kernels one by one."""

    def __init__(self, index, n_slots: int = 3, max_rows: int = 512 * 180, device: int = 0,
                 precision: int | None = None, graphs: bool = False, buckets: list | None = None):
        import torch

        from . import _lib as L
        self.L, self.torch = L, torch
        self.index = index
        self.n_slots = n_slots
        self.max_rows = max_rows
        self.precision = L.TAC_BF16 if precision is None else precision
        dev = torch.device("cuda", device)
        M = index.codebooks.shape[0]
        self.M = M
        self.buckets = sorted(buckets) if buckets else row_buckets(max_rows)
        if self.buckets[-1] != max_rows:
            raise ValueError("the largest bucket must be max_rows")
        self.graphs = graphs
        self.slots = []
        for _ in range(n_slots):
            s = torch.cuda.Stream(device=dev)
            ctx = L.Context(device, stream=s)
            ctx.set_static_centroids(index.C, self.precision)
            self.slots.append(dict(
                stream=s, ctx=ctx, event=torch.cuda.Event(), graph={},
                x_h=torch.zeros((max_rows, 128), dtype=torch.float32, pin_memory=True),
                tok_h=torch.full((max_rows,), -1, dtype=torch.int32, pin_memory=True),
                a_h=torch.empty(max_rows, dtype=torch.int32, pin_memory=True),
                c_h=torch.empty((max_rows, M), dtype=torch.uint8, pin_memory=True),
                r_h=torch.empty(max_rows, dtype=torch.float32, pin_memory=True),
                x_d=torch.empty((max_rows, 128), dtype=torch.float32, device=dev),
                tok_d=torch.empty(max_rows, dtype=torch.int32, device=dev),
                a_d=torch.empty(max_rows, dtype=torch.int32, device=dev),
                dist_d=torch.empty(max_rows, dtype=torch.float32, device=dev),
                c_d=torch.empty((max_rows, M), dtype=torch.uint8, device=dev),
                r_d=torch.empty(max_rows, dtype=torch.float32, device=dev)))
        # device bytes of one staged row: x, token, assignment, distance, codes, norm
        self.row_device_bytes = 128 * 4 + 4 + 4 + 4 + M + 4
        self._ws = {}
        if graphs:
            self._capture()

    def _compute(self, S, b: int):
        """Assignment and PQ encoding of the slot's first b device rows (on the current stream)."""
        L, ix = self.L, self.index
        L.tac_assign(S["ctx"], S["x_d"][:b], ix.C, ix.cent_off, S["a_d"][:b], tok=S["tok_d"][:b],
                     precision=self.precision, dist=S["dist_d"][:b])
        L.pq_encode(S["ctx"], S["x_d"][:b], S["a_d"][:b], ix.C, ix.codebooks, S["c_d"][:b], rnorm=S["r_d"][:b])

    def _capture(self):
        """Per slot: one eager run of the largest bucket (it sizes the context's
        workspace, so no capture allocates), then one graph per bucket."""
        torch = self.torch
        for S in self.slots:
            S["x_d"].zero_()
            S["tok_d"].fill_(-1)
            with torch.cuda.stream(S["stream"]):
                self._compute(S, self.max_rows)
            S["stream"].synchronize()
            for b in self.buckets:
                g = torch.cuda.CUDAGraph()
                with torch.cuda.graph(g, stream=S["stream"]):
                    self._compute(S, b)
                S["graph"][b] = g
            S["stream"].synchronize()

    def bucket(self, rows: int) -> int:
        """Rows a batch of `rows` rows occupies: its graph's bucket (or itself without graphs)."""
        if not self.graphs:
            return rows
        for b in self.buckets:
            if rows <= b:
                return b
        raise ValueError("batch exceeds the slot's staging rows")

    def batch_bytes(self, rows: int) -> int:
        """Device bytes a batch of `rows` rows holds while in flight: the staged
        rows of its bucket and the assignment's workspace for that many rows."""
        b = self.bucket(rows)
        if b not in self._ws:
            ix = self.index
            self._ws[b] = self.L.tac_assign_workspace_bytes(self.slots[0]["ctx"], b, ix.T, ix.C, ix.K,
                                                            self.precision, with_tok=True, with_dist=True)
        return b * self.row_device_bytes + self._ws[b]

    def launch(self, slot: int, xs: list, toks: list) -> int:
        """Stage the rows of a batch into the slot's pinned buffers and enqueue
        copy-in, assignment, PQ encoding and copy-out on the slot's stream (the
        replay of the bucket's graph, or the calls themselves)."""
        S = self.slots[slot]
        n = sum(x.shape[0] for x in xs)
        if n > self.max_rows:
            raise ValueError("batch exceeds the slot's staging rows")
        if n:
            np.concatenate(xs, axis=0, out=S["x_h"].numpy()[:n])
            np.concatenate(toks, axis=0, out=S["tok_h"].numpy()[:n])
        torch = self.torch
        b = self.bucket(n)
        if b > n:
            S["tok_h"].numpy()[n:b] = -1           # the bucket's other rows: unassigned, not encoded
        with torch.cuda.stream(S["stream"]):
            S["x_d"][:n].copy_(S["x_h"][:n], non_blocking=True)
            S["tok_d"][:b].copy_(S["tok_h"][:b], non_blocking=True)
            if self.graphs:
                S["graph"][b].replay()
            else:
                self._compute(S, n)
            S["a_h"][:n].copy_(S["a_d"][:n], non_blocking=True)
            S["c_h"][:n].copy_(S["c_d"][:n], non_blocking=True)
            S["r_h"][:n].copy_(S["r_d"][:n], non_blocking=True)
            S["event"].record(S["stream"])
        return n

    def wait(self, slot: int, n: int):
        S = self.slots[slot]
        S["event"].synchronize()
        return S["a_h"].numpy()[:n], S["c_h"].numpy()[:n], S["r_h"].numpy()[:n]

    def close(self):
        for S in self.slots:
            S["graph"].clear()
            S["ctx"].close()


class EncodeService:
    """Continuous-batching encode service over an executor (GpuExecutor, or a
    stand-in with the same launch / wait interface)."""

    def __init__(self, executor, max_docs: int = 512, ledger_bytes: int | None = None, idle_wait: float = 0.0005,
                 tune_gc: bool = True):
        """ledger_bytes: device memory the batches in flight may hold together
        (default: what every slot holds at its capacity).  The executor's
        batch_bytes(rows) is a batch's charge; an executor without it is
        charged ROW_BYTES per row."""
        self.ex = executor
        self._tune_gc = tune_gc
        if tune_gc:
            _gc_acquire()
        self.n_slots = executor.n_slots
        self.max_docs = max_docs
        self.max_rows = executor.max_rows
        self._bytes = getattr(executor, "batch_bytes", None) or (lambda rows: rows * ROW_BYTES)
        self.ledger_cap = ledger_bytes if ledger_bytes is not None else self.n_slots * self._bytes(self.max_rows)
        self.max_ledger_used = 0
        self.ledger_used = 0
        self.idle_wait = idle_wait
        self.stats = ServiceStats()
        self._in = queue.Queue()
        self._pending: deque[Request] = deque()
        self._free = list(range(self.n_slots))
        self._inflight = queue.Queue()
        self._lock = threading.Condition()
        self._stop = False
        self._next_id = 0
        self._sched = threading.Thread(target=self._schedule, name="tac-scheduler", daemon=True)
        self._done = threading.Thread(target=self._complete, name="tac-completion", daemon=True)
        self._sched.start()
        self._done.start()

    # ---- public -------------------------------------------------------------
    def submit(self, x: np.ndarray, tok: np.ndarray) -> Future:
        x = np.ascontiguousarray(x, dtype=np.float32)
        tok = np.ascontiguousarray(tok, dtype=np.int32)
        if x.ndim != 2 or x.shape[1] != 128 or tok.shape != (x.shape[0],):
            raise ValueError("a document is x float32[n, 128] with tok int32[n]")
        if x.shape[0] > self.max_rows or x.shape[0] == 0 or self._bytes(x.shape[0]) > self.ledger_cap:
            raise ValueError(f"a document holds 1..{self.max_rows} vectors (and fits the memory ledger)")
        f = Future()
        r = Request(x, tok, f, time.perf_counter())
        with self._lock:
            r.rid = self._next_id
            self._next_id += 1
        self._in.put(r)
        return f

    def close(self):
        with self._lock:
            self._stop = True
            self._lock.notify_all()
        self._in.put(None)
        self._sched.join()
        self._inflight.put(None)
        self._done.join()
        if self._tune_gc:
            self._tune_gc = False
            _gc_release()

    # ---- scheduler ----------------------------------------------------------
    def _take_arrivals(self, block: bool):
        try:
            r = self._in.get(timeout=self.idle_wait) if block else self._in.get_nowait()
        except queue.Empty:
            return
        while r is not None:
            self._pending.append(r)
            try:
                r = self._in.get_nowait()
            except queue.Empty:
                return

    def _schedule(self):
        while True:
            with self._lock:
                stop = self._stop
            self._take_arrivals(block=not self._pending)
            if stop and not self._pending and self._in.empty():
                return
            if not self._pending:
                continue
            with self._lock:
                while not self._free and not self._stop:
                    self._lock.wait()
                if not self._free:
                    continue
                slot = self._free.pop(0)
                # admit in arrival order while the batch and the ledger have room
                batch, rows, nbytes = [], 0, 0
                while self._pending and len(batch) < self.max_docs:
                    r = self._pending[0]
                    k = r.x.shape[0]
                    if rows + k > self.max_rows:
                        break
                    b = self._bytes(rows + k)
                    if self.ledger_used + b > self.ledger_cap:
                        break
                    batch.append(self._pending.popleft())
                    rows += k
                    nbytes = b
                if not batch:            # nothing fits until memory is released
                    self._free.insert(0, slot)
                    self._lock.wait()
                    continue
                self.ledger_used += nbytes
                self.max_ledger_used = max(self.max_ledger_used, self.ledger_used)
            try:
                n = self.ex.launch(slot, [r.x for r in batch], [r.tok for r in batch])
                self._inflight.put((slot, batch, n, nbytes, None))
            except Exception as e:  # the batch fails as a whole; the loop continues
                self._inflight.put((slot, batch, 0, nbytes, e))

    # ---- completion ---------------------------------------------------------
    def _complete(self):
        from ._lib import TAC_E_UNSEEN_TOKEN, TacError
        while True:
            item = self._inflight.get()
            if item is None:
                return
            slot, batch, n, nbytes, err = item
            lens = np.fromiter((r.x.shape[0] for r in batch), dtype=np.int64, count=len(batch))
            offs = np.zeros(len(batch) + 1, dtype=np.int64)
            np.cumsum(lens, out=offs[1:])
            if err is None:
                try:
                    # one copy of the batch's outputs (the staging buffers are reused);
                    # each document's result holds views into it
                    a, c, rho = (np.array(v, copy=True) for v in self.ex.wait(slot, n))
                    bad = np.minimum.reduceat(a, offs[:-1]) < 0 if len(batch) else np.zeros(0, bool)
                except Exception as e:
                    err = e
            now = time.perf_counter()
            for i, r in enumerate(batch):
                r.t_done = now
                if err is not None:
                    r.future.set_exception(err)
                    self.stats.failed += 1
                elif bad[i]:
                    r.future.set_exception(TacError(TAC_E_UNSEEN_TOKEN, "a token of this document has no centroid"))
                    self.stats.failed += 1
                else:
                    o0, o1 = offs[i], offs[i + 1]
                    r.future.set_result(Result(a[o0:o1], c[o0:o1], rho[o0:o1], now - r.t_arrival))
                    self.stats.latencies.append(now - r.t_arrival)
            off = int(offs[-1])
            self.stats.batches += 1
            self.stats.docs += len(batch)
            self.stats.vectors += off
            self.stats.batch_sizes.append(len(batch))
            with self._lock:
                self.ledger_used -= nbytes
                self._free.append(slot)
                self._lock.notify_all()


def run_load(service: EncodeService, docs: list, arrivals: np.ndarray | None):
    """Submit documents at the given arrival times (seconds from now; None = all
    at once) and wait for every result.  Returns (results, wall seconds)."""
    t0 = time.perf_counter()
    futs = []
    for i, (x, t) in enumerate(docs):
        if arrivals is not None:
            delay = t0 + arrivals[i] - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
        futs.append(service.submit(x, t))
    out = []
    for f in futs:
        try:
            out.append(f.result())
        except Exception as e:  # failed documents are reported as their exception
            out.append(e)
    return out, time.perf_counter() - t0
