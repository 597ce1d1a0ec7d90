"""Independent per-token Lloyd k-means (oracle; test infrastructure only).

Sect. 2.1: after the budget, TAC runs kappa_j-means independently inside the
vectors of every token j, minimising the within-cluster sum of squares
(the inertia equation of Sect. 2.1); Sect. 3.1 fixes 10 iterations, and the
clustering time there includes assigning every vector to its final centroid.

Definitions used (readings listed in the design notes):
* distance: squared Euclidean distance, in float64;
* assignment: argmin over the token's own centroids, lowest centroid index on
  equal distances;
* update: every centroid becomes the float64 mean of its members, rounded to
  float32; a centroid with no members keeps its previous value;
* initialisation: seeded distinct rows of the segment (supplied as data).

The float64 distance matrix of a segment is formed with the identity
||x - c||^2 = ||x||^2 - 2 x.c + ||c||^2 through one matrix product (a library
primitive); the distance reported for the chosen centroid is recomputed
directly as sum_i (x_i - c_i)^2.

Pinned by: brute-force optimal partitions on tiny 1-D inputs, the closed form
for one centroid per token (one step gives the token means and inertia
sum_j n_j s_j), fixed points when every row is its own centroid, monotone
inertia, and agreement with the direct float64 definition
(tests/test_oracle_lloyd.py, tests/test_oracle_bruteforce.py).
"""
from __future__ import annotations

import numpy as np

from . import dist32 as _d32

# dist32 differs from the exact distance by at most about (d+2) * 2^-24
# relative (< 1e-5 for d = 128).  Centroids farther than this margin above the
# float64 minimum can never be the float32 argmin, so the fp32 decision mode
# evaluates the canonical distance only on the others.
_FP32_MARGIN_ABS = 1e-4
_FP32_MARGIN_REL = 1e-4
_ROW_CHUNK = 2048


def _d64_matrix(X: np.ndarray, C: np.ndarray) -> np.ndarray:
    xx = np.einsum("ij,ij->i", X, X)
    cc = np.einsum("ij,ij->i", C, C)
    return xx[:, None] - 2.0 * (X @ C.T) + cc[None, :]


def _smallest_k(D: np.ndarray, kk: int) -> np.ndarray:
    """int64[n, kk]: per row the column indices of the kk smallest entries in
    ascending order, equal values by lower index -- the first kk entries of a
    stable argsort of the row, found without sorting the whole row."""
    n, k = D.shape
    if kk >= k or k <= 64:
        return np.argsort(D, axis=1, kind="stable")[:, :kk]
    # every entry not above the row's kk-th smallest value is a candidate
    kth = np.partition(D, kk - 1, axis=1)[:, kk - 1]
    out = np.empty((n, kk), dtype=np.int64)
    for i in range(n):
        cand = np.nonzero(D[i] <= kth[i])[0]
        order = np.lexsort((cand, D[i, cand]))
        out[i] = cand[order[:kk]]
    return out


def _assign_block(X32, C32, decide, topk, full_fp32=False):
    """Assign rows X32 to centroids C32 (both float32 arrays of one token).

    Returns (local argmin int64[n], D64 of the chosen float64[n],
    d32 of the chosen float32[n], top-k local idx int64[n,topk], top-k D64)."""
    n, k = X32.shape[0], C32.shape[0]
    X = X32.astype(np.float64)
    C = C32.astype(np.float64)
    D = _d64_matrix(X, C)
    if decide == "fp64":
        a = np.argmin(D, axis=1)
    elif decide == "fp32":
        if full_fp32:
            d32 = _d32.pairwise(X32, C32)
            a = np.argmin(d32, axis=1)
        else:
            dmin = D.min(axis=1)
            thr = dmin + _FP32_MARGIN_ABS + _FP32_MARGIN_REL * np.abs(dmin)
            r, c = np.nonzero(D <= thr[:, None])
            d32 = _d32.rowwise(X32[r], C32[c])
            order = np.lexsort((c, d32, r))
            r, c = r[order], c[order]
            first = np.ones(r.shape[0], dtype=bool)
            first[1:] = r[1:] != r[:-1]
            a = np.empty(n, dtype=np.int64)
            a[r[first]] = c[first]
    else:
        raise ValueError(decide)
    a = a.astype(np.int64)
    diff = X - C[a]
    D_chosen = np.einsum("ij,ij->i", diff, diff)
    d32_chosen = _d32.rowwise(X32, C32[a])
    if topk:
        kk = min(topk, k)
        idx = _smallest_k(D, kk)
        tD = np.take_along_axis(D, idx, axis=1)
        if kk < topk:
            idx = np.pad(idx, ((0, 0), (0, topk - kk)), constant_values=-1)
            tD = np.pad(tD, ((0, 0), (0, topk - kk)), constant_values=np.inf)
    else:
        idx = tD = None
    return a, D_chosen, d32_chosen, idx, tD


def assign(xs, seg_off, C, cent_off, decide="fp64", topk=0, full_fp32=False):
    """Assign every token-sorted row to the nearest centroid of its own token.

    Returns a dict with ``a`` (int64[N], global centroid id), ``D`` (float64[N],
    distance to the chosen centroid), ``d32`` (float32[N], canonical FP32
    distance to the chosen centroid), ``J`` (float64 inertia = sum of D) and,
    when ``topk`` > 0, ``top_idx`` / ``top_D`` (the ``topk`` nearest centroids
    of each row in float64, global ids, -1 / inf padded)."""
    N = xs.shape[0]
    T = seg_off.shape[0] - 1
    a = np.full(N, -1, dtype=np.int64)
    D = np.zeros(N, dtype=np.float64)
    d32 = np.zeros(N, dtype=np.float32)
    top_idx = np.full((N, topk), -1, dtype=np.int64) if topk else None
    top_D = np.full((N, topk), np.inf) if topk else None
    for j in range(T):
        lo, hi = int(seg_off[j]), int(seg_off[j + 1])
        c0, c1 = int(cent_off[j]), int(cent_off[j + 1])
        if hi == lo:
            continue
        if c1 == c0:
            raise ValueError(f"token {j} has vectors but no centroids")
        Cj = C[c0:c1]
        for r0 in range(lo, hi, _ROW_CHUNK):
            r1 = min(hi, r0 + _ROW_CHUNK)
            la, lD, l32, ti, tD = _assign_block(xs[r0:r1], Cj, decide, topk, full_fp32)
            a[r0:r1] = la + c0
            D[r0:r1] = lD
            d32[r0:r1] = l32
            if topk:
                top_idx[r0:r1] = np.where(ti >= 0, ti + c0, -1)
                top_D[r0:r1] = tD
    out = {"a": a, "D": D, "d32": d32, "J": float(D.sum())}
    if topk:
        out["top_idx"] = top_idx
        out["top_D"] = top_D
    return out


def assign_rows(xs, rows, seg_off, C, cent_off, decide="fp64", topk=0):
    """Assignment of selected token-sorted rows only (a row's assignment depends
    only on its own token's centroids, so a sample loses no exactness)."""
    rows = np.asarray(rows, dtype=np.int64)
    seg = np.searchsorted(seg_off, rows, side="right") - 1
    a = np.empty(rows.shape[0], dtype=np.int64)
    D = np.empty(rows.shape[0], dtype=np.float64)
    d32 = np.empty(rows.shape[0], dtype=np.float32)
    top_idx = np.full((rows.shape[0], topk), -1, dtype=np.int64) if topk else None
    top_D = np.full((rows.shape[0], topk), np.inf) if topk else None
    for j in np.unique(seg):
        sel = np.nonzero(seg == j)[0]
        c0, c1 = int(cent_off[j]), int(cent_off[j + 1])
        for s0 in range(0, sel.shape[0], _ROW_CHUNK):
            s = sel[s0:s0 + _ROW_CHUNK]
            la, lD, l32, ti, tD = _assign_block(xs[rows[s]], C[c0:c1], decide, topk)
            a[s] = la + c0
            D[s] = lD
            d32[s] = l32
            if topk:
                top_idx[s] = np.where(ti >= 0, ti + c0, -1)
                top_D[s] = tD
    out = {"a": a, "D": D, "d32": d32}
    if topk:
        out["top_idx"] = top_idx
        out["top_D"] = top_D
    return out


def update(xs, a, C_old):
    """New centroids: float64 mean of each cluster's members, rounded to float32;
    empty clusters keep C_old.  Returns (C_new float32[K, d], counts int64[K])."""
    K, d = C_old.shape
    a = np.asarray(a, dtype=np.int64)
    counts = np.bincount(a, minlength=K).astype(np.int64)
    sums = np.empty((K, d), dtype=np.float64)
    for i in range(d):
        sums[:, i] = np.bincount(a, weights=xs[:, i].astype(np.float64), minlength=K)
    C_new = C_old.astype(np.float32).copy()
    nz = counts > 0
    C_new[nz] = (sums[nz] / counts[nz, None]).astype(np.float32)
    return C_new, counts


def inertia(xs, a, C) -> float:
    """Within-cluster sum of squares (Sect. 2.1) of assignment ``a``, float64."""
    diff = xs.astype(np.float64) - C[np.asarray(a)].astype(np.float64)
    return float(np.einsum("ij,ij->", diff, diff))


def init_centroids(xs, seg_off, cent_off, picks) -> np.ndarray:
    """float32[K, d]: centroid cent_off_j + l is row seg_off_j + picks[cent_off_j + l]."""
    T = seg_off.shape[0] - 1
    K = int(cent_off[-1])
    C = np.empty((K, xs.shape[1]), dtype=np.float32)
    for j in range(T):
        c0, c1 = int(cent_off[j]), int(cent_off[j + 1])
        if c1 > c0:
            C[c0:c1] = xs[int(seg_off[j]) + picks[c0:c1]]
    return C


def lloyd(xs, seg_off, cent_off, C0, iters=10, decide="fp64", topk=0):
    """Run ``iters`` Lloyd steps (assign, update) then a final assign.

    Returns a list of per-step dicts: step t holds the centroids C it started
    from, its assignment output and the updated centroids/counts; the last
    entry is the final assignment (no update)."""
    C = C0.astype(np.float32).copy()
    steps = []
    for _ in range(iters):
        r = assign(xs, seg_off, C, cent_off, decide=decide, topk=topk)
        C_new, counts = update(xs, r["a"], C)
        r.update(C=C, C_new=C_new, counts=counts)
        steps.append(r)
        C = C_new
    r = assign(xs, seg_off, C, cent_off, decide=decide, topk=topk)
    r.update(C=C)
    steps.append(r)
    return steps
