"""Residual compression with product quantisation (oracle; test infrastructure only).

Sect. 2.1 ("Residuals Compression"): after clustering, every vector's residual
r = x - c_{a(x)} is normalised, its norm is stored separately, and the
normalised residual is compressed with PQ; Sect. 3.1 fixes M = 32 subspaces
with 8-bit codes (256 codes per subspace).

Readings (listed in the design notes): subspace m is the contiguous block of
d/M coordinates starting at m*d/M, with no rotation; a zero residual has
u = 0; codebooks are trained by Lloyd iterations per subspace (lowest code
index on ties, empty codes keep their value, float64 means rounded to
float32), starting from the subspace slices of seeded training rows.

``mode="fp32"`` evaluates the residual, its norm and the code distances with
the canonical FP32 operation sequence of the kernels (each op rounded once,
no fused multiply-add): r_i = x_i - c_i; rho = sqrt(sum_i r_i * r_i)
(sequential); u_i = r_i / rho; code distance = sequential sum over the d/M
coordinates of (u_i - B_i)^2.

Pinned by: ||u|| = 1 (or 0), x = c + rho * u, zero reconstruction error when
the codebook holds every training row, brute-force argmin equality, and the
scalar-quantiser special case d/M = 1 (tests/test_oracle_pq.py).
"""
from __future__ import annotations

import numpy as np

from . import dist32 as _d32


def residuals(x, c_rows, normalize=True, mode="fp64"):
    """Normalised residuals of rows ``x`` against their assigned centroids
    ``c_rows`` (same shape).  Returns (u, rho): float64 in mode "fp64",
    float32 (canonical kernel sequence) in mode "fp32"."""
    if mode == "fp64":
        r = x.astype(np.float64) - c_rows.astype(np.float64)
        rho = np.sqrt(np.einsum("ij,ij->i", r, r))
        if not normalize:
            return r, rho
        u = np.zeros_like(r)
        nz = rho > 0
        u[nz] = r[nz] / rho[nz, None]
        return u, rho
    if mode == "fp32":
        x32 = np.ascontiguousarray(x, dtype=np.float32)
        c32 = np.ascontiguousarray(c_rows, dtype=np.float32)
        r = x32 - c32
        rho = np.sqrt(_d32.sqnorm(r)).astype(np.float32)
        if not normalize:
            return r, rho
        u = np.zeros_like(r)
        nz = rho > 0
        u[nz] = r[nz] / rho[nz, None]
        return u, rho
    raise ValueError(mode)


def _sub(u, m, dsub):
    return u[:, m * dsub:(m + 1) * dsub]


def pq_encode(u, codebooks, decide="fp64", topk=0, chunk=8192):
    """Codes uint8[n, M]: per subspace, argmin over codes of the squared
    distance, lowest code on ties.  With ``topk`` also returns the ``topk``
    nearest codes and their float64 distances per (row, subspace)."""
    M, ksub, dsub = codebooks.shape
    n = u.shape[0]
    codes = np.empty((n, M), dtype=np.uint8 if ksub <= 256 else np.int32)
    t_idx = np.empty((n, M, topk), dtype=np.int64) if topk else None
    t_D = np.empty((n, M, topk), dtype=np.float64) if topk else None
    for m in range(M):
        Bm32 = codebooks[m].astype(np.float32)
        Bm = Bm32.astype(np.float64)
        for r0 in range(0, n, chunk):
            r1 = min(n, r0 + chunk)
            S = _sub(u[r0:r1], m, dsub)
            if decide == "fp64" or topk:
                S64 = S.astype(np.float64)
                D = np.zeros((r1 - r0, ksub))
                for i in range(dsub):
                    t = S64[:, i, None] - Bm[None, :, i]
                    D += t * t
            if decide == "fp64":
                codes[r0:r1, m] = np.argmin(D, axis=1)
            elif decide == "fp32":
                codes[r0:r1, m] = np.argmin(_d32.pairwise(S.astype(np.float32), Bm32), axis=1)
            else:
                raise ValueError(decide)
            if topk:
                idx = np.argsort(D, axis=1, kind="stable")[:, :topk]
                t_idx[r0:r1, m] = idx
                t_D[r0:r1, m] = np.take_along_axis(D, idx, axis=1)
    if topk:
        return codes, t_idx, t_D
    return codes


def pq_train(R, M, ksub, iters, init_rows=None, decide="fp64", init_codebooks=None):
    """Codebooks float32[M, ksub, d/M]: Lloyd per subspace on the training rows
    R (float32[n, d]), starting from the slices of rows ``init_rows`` (or from
    ``init_codebooks`` when given)."""
    n, d = R.shape
    dsub = d // M
    R = np.asarray(R)
    if init_codebooks is not None:
        cb = np.asarray(init_codebooks, dtype=np.float32).copy()
    else:
        cb = np.stack([_sub(R[np.asarray(init_rows)], m, dsub) for m in range(M)]).astype(np.float32)
    for _ in range(iters):
        codes = pq_encode(R, cb, decide=decide)
        new = cb.copy()
        for m in range(M):
            c = codes[:, m].astype(np.int64)
            cnt = np.bincount(c, minlength=ksub)
            S = _sub(R, m, dsub).astype(np.float64)
            for i in range(dsub):
                s = np.bincount(c, weights=S[:, i], minlength=ksub)
                nz = cnt > 0
                new[m, nz, i] = (s[nz] / cnt[nz]).astype(np.float32)
        cb = new
    return cb


def pq_decode(codes, codebooks) -> np.ndarray:
    """float32[n, d]: concatenation of the selected code vectors."""
    M = codebooks.shape[0]
    return np.concatenate([codebooks[m][codes[:, m].astype(np.int64)] for m in range(M)], axis=1)
