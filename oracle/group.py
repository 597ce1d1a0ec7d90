"""Grouping by token and per-token spread (oracle; test infrastructure only).

Sect. 2.1 splits the clustering into independent per-token subproblems: the
vectors sharing a token id form one segment.  Phase 2 of the budget needs, for
every token j, the spread s_j = (1/n_j) * sum_i ||t_{j,i} - mean_j||^2
(the "component-wise variance" equation of Sect. 2.1).

Pinned by: closed forms of the spread (unit vectors: s = 1 - ||mean||^2;
two orthonormal vectors: s = 1/2; identical vectors: s = 0) and a stable-sort
invariant on the permutation (tests/test_oracle_group.py).
"""
from __future__ import annotations

import numpy as np


def group_by_token(tok: np.ndarray, T: int):
    """Stable grouping of rows by token id.

    Returns (perm int64[N], seg_off int64[T+1], counts int64[T]).  Row
    ``perm[i]`` of the input is row ``i`` of the token-sorted order; segments
    are in ascending token id and, inside a segment, in ascending original
    row index.  Token j owns sorted rows [seg_off[j], seg_off[j+1]).
    """
    tok = np.asarray(tok)
    if tok.size and (tok.min() < 0 or tok.max() >= T):
        raise ValueError("token id out of range")
    perm = np.argsort(tok, kind="stable").astype(np.int64)
    counts = np.bincount(tok, minlength=T).astype(np.int64)
    seg_off = np.zeros(T + 1, dtype=np.int64)
    seg_off[1:] = np.cumsum(counts)
    return perm, seg_off, counts


def spreads(xs: np.ndarray, seg_off: np.ndarray) -> np.ndarray:
    """float64[T] spread per token, two-pass in float64 (Sect. 2.1, Phase 2).

    ``xs`` are the token-sorted vectors.  Absent tokens (n_j = 0) get 0.
    """
    T = seg_off.shape[0] - 1
    out = np.zeros(T, dtype=np.float64)
    for j in range(T):
        lo, hi = int(seg_off[j]), int(seg_off[j + 1])
        n = hi - lo
        if n == 0:
            continue
        X = xs[lo:hi].astype(np.float64)
        mean = X.sum(axis=0) / n
        dev = X - mean
        out[j] = float((dev * dev).sum()) / n
    return out
