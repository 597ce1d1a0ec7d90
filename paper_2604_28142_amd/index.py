"""Index-build driver: chains the libtac calls of the token-aware clustering path.

group + budget (tac_budget) -> seeded initial centroids -> Lloyd iterations
(tac_assign + tac_update, optionally captured once into a HIP graph and
replayed) -> final assignment -> PQ training on normalised residuals of a
seeded sample -> fused residual + PQ encoding of every vector.  Device buffers
are torch tensors; all arithmetic runs in libtac.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import torch

from . import _lib as L


@dataclass
class Index:
    """Device state of a built (or partly built) index, token-sorted order."""
    T: int
    K: int
    xs: torch.Tensor            # [N, 128] float32 token-sorted vectors
    perm: torch.Tensor          # [N] int32 sorted row -> input row
    seg_off: torch.Tensor       # [T+1] int64
    cent_off: torch.Tensor      # [T+1] int64
    C: torch.Tensor             # [K, 128] float32 centroids
    host: dict = field(default_factory=dict)   # seg_off, counts, spread, kappa, cent_off (numpy)
    assign: torch.Tensor | None = None
    dist: torch.Tensor | None = None
    codebooks: torch.Tensor | None = None
    codes: torch.Tensor | None = None
    rnorm: torch.Tensor | None = None


def group_and_budget(ctx: L.Context, x: torch.Tensor, tok: torch.Tensor, T: int, K: int,
                     params: L.BudgetParams | None = None, spread_override=None, keep_x: bool = True) -> Index:
    N = x.shape[0]
    dev = x.device
    perm = torch.empty(N, dtype=torch.int32, device=dev)
    xs = torch.empty_like(x)
    seg = torch.empty(T + 1, dtype=torch.int64, device=dev)
    coff = torch.empty(T + 1, dtype=torch.int64, device=dev)
    host = L.tac_budget(ctx, x, tok, T, K, params, spread_override=spread_override, perm=perm, xs=xs,
                        seg_off=seg, cent_off=coff)
    C = torch.empty((K, x.shape[1]), dtype=torch.float32, device=dev)
    return Index(T=T, K=K, xs=xs, perm=perm, seg_off=seg, cent_off=coff, C=C, host=host)


def init_centroids(ctx: L.Context, idx: Index, picks: np.ndarray):
    L.tac_init_centroids(ctx, idx.xs, idx.seg_off, idx.cent_off, torch.from_numpy(picks).to(idx.xs.device), idx.C)


class LloydLoop:
    """`iters` Lloyd iterations (assign + update) over resident buffers.

    run() enqueues them eagerly; capture() records the same sequence into a HIP
    graph once (after one eager run has sized the workspace) and replay() relaunches
    it.  Centroids ping-pong between two buffers; the result is always left in
    idx.C (an even number of swaps, with a copy when `iters` is odd)."""

    def __init__(self, ctx: L.Context, idx: Index, iters: int = 10, precision: int = L.TAC_BF16):
        self.ctx, self.idx, self.iters, self.precision = ctx, idx, iters, precision
        N = idx.xs.shape[0]
        dev = idx.xs.device
        self.assign = torch.empty(N, dtype=torch.int32, device=dev)
        self.dist = torch.empty(N, dtype=torch.float32, device=dev)
        self.inertia = torch.zeros(iters + 1, dtype=torch.float64, device=dev)
        self.counts = torch.empty(idx.K, dtype=torch.int64, device=dev)
        self.other = torch.empty_like(idx.C)
        self.graph = None

    def _enqueue(self):
        idx = self.idx
        cur, nxt = idx.C, self.other
        for t in range(self.iters):
            L.tac_assign(self.ctx, idx.xs, cur, idx.cent_off, self.assign, seg_off=idx.seg_off,
                         precision=self.precision, dist=self.dist, inertia=self.inertia[t:t + 1])
            L.tac_update(self.ctx, idx.xs, idx.seg_off, self.assign, cur, nxt, self.counts)
            cur, nxt = nxt, cur
        if cur is not idx.C:
            idx.C.copy_(cur)

    def run(self):
        self._enqueue()

    def capture(self):
        """Record the loop into a HIP graph on a side stream (timing must be off)."""
        s = torch.cuda.Stream(device=self.idx.xs.device)
        prev = self.ctx.stream
        s.wait_stream(torch.cuda.current_stream())
        g = torch.cuda.CUDAGraph()
        self.ctx.set_stream(s)
        try:
            with torch.cuda.graph(g, stream=s):
                self._enqueue()
        finally:
            self.ctx.set_stream(prev)
        torch.cuda.current_stream().wait_stream(s)
        self.graph = g

    def replay(self):
        self.graph.replay()


def final_assign(ctx: L.Context, idx: Index, precision: int = L.TAC_BF16):
    N = idx.xs.shape[0]
    dev = idx.xs.device
    idx.assign = torch.empty(N, dtype=torch.int32, device=dev)
    idx.dist = torch.empty(N, dtype=torch.float32, device=dev)
    L.tac_assign(ctx, idx.xs, idx.C, idx.cent_off, idx.assign, seg_off=idx.seg_off, precision=precision,
                 dist=idx.dist)


def train_pq(ctx: L.Context, idx: Index, sample_rows: np.ndarray, init_rows: np.ndarray, M: int = 32,
             ksub: int = 256, iters: int = 10):
    """Codebooks from the normalised residuals of the sampled (token-sorted) rows.

    The initial codebook of subspace m holds the m-th 4-d slices of the training
    rows `init_rows` (positions inside the sample)."""
    dev = idx.xs.device
    rows = torch.from_numpy(np.ascontiguousarray(sample_rows, dtype=np.int64)).to(dev)
    R = torch.empty((rows.shape[0], idx.xs.shape[1]), dtype=torch.float32, device=dev)
    L.tac_residuals(ctx, idx.xs, idx.assign, idx.C, R, rows=rows)
    dsub = idx.xs.shape[1] // M
    init = R[torch.from_numpy(np.asarray(init_rows, dtype=np.int64)).to(dev)]
    init = init.view(ksub, M, dsub).transpose(0, 1).contiguous()
    idx.codebooks = torch.empty((M, ksub, dsub), dtype=torch.float32, device=dev)
    L.pq_train(ctx, R, init, idx.codebooks, iters=iters)
    return R


def encode_all(ctx: L.Context, idx: Index, normalize: bool = True):
    N = idx.xs.shape[0]
    dev = idx.xs.device
    M = idx.codebooks.shape[0]
    idx.codes = torch.empty((N, M), dtype=torch.uint8, device=dev)
    idx.rnorm = torch.empty(N, dtype=torch.float32, device=dev)
    L.pq_encode(ctx, idx.xs, idx.assign, idx.C, idx.codebooks, idx.codes, normalize=normalize, rnorm=idx.rnorm)
