"""Measured launch tuning of tac_assign, cached per workload.

The assignment kernel's launch has five knobs (``tac_tuning`` in the C ABI).
Two of them together pick the 16-bit screens' compiled kernel (the ``tile``
knob here): the occupancy (``waves_per_simd``: one or two 256-thread
work-groups per compute unit) and the tile shape (``tile_blocks``: column
blocks of 16 rows per wave, i.e. 192-, 256- or 320-row work items; two
work-groups per CU take 192).  The others choose which tokens skip the
matrix-core screen (``direct_max_kappa``),
which tokens the persistent work queue hands out first (``heavy_kappa``), and
how many persistent work-groups share a compute unit (``groups_per_cu``).
None of them changes a result, only the time, and the best values depend on
the segment structure (how rows and centroids spread over tokens) and on the
device.  A larger tile restages each centroid for more rows; a smaller one
holds fewer registers and spreads a token's rows over more compute units; two
work-groups per CU hide one's memory waits and vector work under the other's
matrix work, with half the registers and LDS each.

``tune_assign`` measures candidate settings on the caller's resident buffers by
coordinate search (one knob at a time, the others held at their best so far),
timing whole ``tac_assign`` calls with HIP events on the context's stream, and
checks on the way that every candidate returns bitwise the same assignments.
Results are cached in a JSON file keyed by a fingerprint of the workload, the
precision, the device and the library build, so a later build of the same
shape reuses them without measuring.
"""
from __future__ import annotations

import hashlib
import json
import os
import time

import numpy as np
import torch

from . import _lib as L

DEFAULT = {"waves_per_simd": 2, "tile_blocks": 3, "direct_max_kappa": 4, "heavy_kappa": 1024, "groups_per_cu": 0}
# the 16-bit screens' compiled kernels: (occupancy, tile) pairs
TILES = [{"waves_per_simd": 2, "tile_blocks": 3}, {"waves_per_simd": 1, "tile_blocks": 5},
         {"waves_per_simd": 1, "tile_blocks": 4}, {"waves_per_simd": 1, "tile_blocks": 3}]
SPACE = {
    "tile": TILES,
    "direct_max_kappa": [0, 2, 4, 8, 16],
    "heavy_kappa": [128, 512, 1024, 2048, 4096, 8192, 16384, 1 << 30],  # 2^30: no token queued first
    "groups_per_cu": [0, 1],
}
CACHE_ENV = "TAC_AUTOTUNE_CACHE"


def default_cache_path() -> str:
    return os.environ.get(CACHE_ENV) or os.path.join(os.path.expanduser("~"), ".cache", "tac_autotune.json")


def _library_id() -> str:
    st = os.stat(L.LIB_PATH)
    return f"{st.st_size}:{int(st.st_mtime)}"


def workload_key(seg_off: np.ndarray, cent_off: np.ndarray, precision: int, device: int = 0) -> str:
    """Fingerprint of the segment structure (rows and centroids per token), precision, device and build."""
    n = np.diff(np.asarray(seg_off, dtype=np.int64))
    k = np.diff(np.asarray(cent_off, dtype=np.int64))
    h = hashlib.sha1()
    h.update(np.ascontiguousarray(n).tobytes())
    h.update(np.ascontiguousarray(k).tobytes())
    name = torch.cuda.get_device_name(device) if torch.cuda.is_available() else "cpu"
    return f"p{precision}:N{int(n.sum())}:T{n.size}:K{int(k.sum())}:{h.hexdigest()[:16]}:{name}:{_library_id()}"


def _load(path: str) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path: str, data: dict):
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = f"{path}.{os.getpid()}.tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _time_assign(ctx: L.Context, xs, C, cent_off, seg_off, precision, assign, dist, reps: int) -> float:
    """Median ms of `reps` tac_assign calls (after one untimed call), HIP events on the context's stream."""
    stream = ctx.stream
    L.tac_assign(ctx, xs, C, cent_off, assign, seg_off=seg_off, precision=precision, dist=dist)
    times = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        L.tac_assign(ctx, xs, C, cent_off, assign, seg_off=seg_off, precision=precision, dist=dist)
        b.record(stream)
        b.synchronize()
        times.append(a.elapsed_time(b))
    return float(np.median(times))


def tune_assign(ctx: L.Context, xs: torch.Tensor, C: torch.Tensor, cent_off: torch.Tensor, seg_off: torch.Tensor,
                precision: int = L.TAC_BF16, reps: int = 3, cache_path: str | None = None,
                space: dict | None = None, host_seg_off=None, host_cent_off=None, apply: bool = True,
                verbose: bool = False) -> dict:
    """Pick the fastest tac_tuning for this workload; returns {"tuning", "ms", "default_ms", "cached", "trials"}.

    The chosen tuning is set on `ctx` when `apply` is true.  Candidates whose
    assignments differ from the first candidate's raise RuntimeError (the
    tuning must never change a result)."""
    space = dict(space or SPACE)
    if precision == L.TAC_FP32:
        space.pop("tile", None)  # the FP32 screen has one tile shape
    cache_path = cache_path or default_cache_path()
    so = np.asarray(host_seg_off if host_seg_off is not None else seg_off.cpu().numpy())
    co = np.asarray(host_cent_off if host_cent_off is not None else cent_off.cpu().numpy())
    key = workload_key(so, co, precision, ctx.device)
    cache = _load(cache_path)
    if key in cache:
        entry = dict(cache[key], cached=True)
        if apply:
            ctx.set_tuning(**entry["tuning"])
        return entry

    before = ctx.get_tuning()
    N = xs.shape[0]
    assign = torch.empty(max(N, 1), dtype=torch.int32, device=xs.device)[:N]
    dist = torch.empty(max(N, 1), dtype=torch.float32, device=xs.device)[:N]
    ref = None
    trials = []
    best = dict(DEFAULT)
    measured = {}

    def measure(t: dict) -> float:
        nonlocal ref
        tk = tuple(sorted(t.items()))
        if tk in measured:
            return measured[tk]
        ctx.set_tuning(**t)
        ms = _time_assign(ctx, xs, C, cent_off, seg_off, precision, assign, dist, reps)
        if ref is None:
            ref = assign.clone()
        elif not torch.equal(assign, ref):
            raise RuntimeError(f"tuning {t} changed the assignments")
        measured[tk] = ms
        trials.append({"tuning": dict(t), "ms": ms})
        if verbose:
            print(f"  autotune {t}: {ms:.3f} ms", flush=True)
        return ms

    t0 = time.time()
    default_ms = measure(best)
    best_ms = default_ms
    for knob, values in space.items():
        for v in values:
            cand = dict(best, **(v if isinstance(v, dict) else {knob: v}))
            ms = measure(cand)
            if ms < best_ms:
                best, best_ms = cand, ms
    entry = {"tuning": best, "ms": best_ms, "default_ms": default_ms, "trials": trials,
             "seconds": round(time.time() - t0, 3)}
    cache[key] = entry
    _store(cache_path, cache)
    ctx.set_tuning(**(best if apply else before))
    return dict(entry, cached=False)
