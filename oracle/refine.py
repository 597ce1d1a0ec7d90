"""Oracle for the refine phase of retrieval: MaxSim over candidate documents
from their centroid ids, PQ codes and residual norms (Sect. 2.2, "Refine
Phase: PQ-Optimized MaxSim Computation", with the document layout of the same
section and the distance-table layout of Figure 1).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The score of document d for a query q of n_q token vectors is

    S(q, d) = sum_i max_{t in d} <q_i, x_t>,   x_t = c_{a_t} + rho_t * u_t,

where c_{a_t} is the token's centroid, rho_t its stored residual norm and u_t
the decoded normalised residual: the concatenation of the codewords
B[m, code_{t,m}] (residuals are normalised and their norms kept apart,
Sect. 2.1 "Residuals Compression").  MaxSim uses inner products.

``maxsim_scores`` evaluates it in the paper's order.  The distance tables
T[m][b][i] = <q_{i,m}, B[m, b]> are laid out as macro-blocks per subspace m,
centroid blocks per code b and micro-blocks of the n_q query tokens.  Each
document is read from its layout block: first the centroid contributions
<q_i, c_{a_t}> of all of its tokens, then the residual contributions, one
micro-block per (token, subspace).

Readings (where the paper is silent):
* a document with no token, or whose tokens all carry a centroid id outside
  [0, K), scores -inf (the maximum over an empty set);
* tokens whose centroid id is outside [0, K) are skipped;
* a candidate id outside [0, D) names no document and scores NaN;
* rho is indexed like the layout's tokens: token t of document d is entry
  doc_off[d] + t.

Arithmetic is float64; the final sum over query tokens is sequential in i.
Pins: a hand-worked example, a brute-force decode and invariants in
``tests/test_oracle_refine.py``.
"""
import numpy as np


def distance_tables(Q, codebooks):
    """T float64 [M, ksub, n_q]: T[m, b, i] = <q_{i,m}, B[m, b]>, the
    three-level layout (subspace, code, query-token micro-block)."""
    Q = np.asarray(Q, dtype=np.float64)
    B = np.asarray(codebooks, dtype=np.float64)
    M, ksub, dsub = B.shape
    T = np.empty((M, ksub, Q.shape[0]))
    for m in range(M):
        T[m] = B[m] @ Q[:, m * dsub:(m + 1) * dsub].T
    return T


def doc_block(layout, doc_off, d, M):
    """(centroid ids int64 [n_d], codes uint8 [n_d, M]) of document d, read
    from its layout block: n_d 4-byte little-endian ids, then n_d x M codes."""
    lay = np.asarray(layout, dtype=np.uint8)
    t0, t1 = int(doc_off[d]), int(doc_off[d + 1])
    n = t1 - t0
    base = t0 * (4 + M)
    ids = lay[base:base + 4 * n].view("<i4").astype(np.int64)
    codes = lay[base + 4 * n:base + 4 * n + n * M].reshape(n, M)
    return ids, codes


def maxsim_scores(Q, C, codebooks, layout, doc_off, rnorm, cand):
    """float64 [len(cand)]: S(q, d) for each candidate document d of one query
    Q [n_q, dim]; C [K, dim] centroids, codebooks [M, ksub, dim / M], layout
    and doc_off as produced by ``doc_layout``, rnorm [N] residual norms."""
    Q = np.asarray(Q, dtype=np.float64)
    C = np.asarray(C, dtype=np.float64)
    rnorm = np.asarray(rnorm, dtype=np.float64)
    K = C.shape[0]
    M = np.asarray(codebooks).shape[0]
    nq = Q.shape[0]
    T = distance_tables(Q, codebooks)
    D = len(doc_off) - 1
    out = np.empty(len(cand))
    for j, d in enumerate(np.asarray(cand).tolist()):
        if not 0 <= d < D:
            out[j] = np.nan
            continue
        ids, codes = doc_block(layout, doc_off, d, M)
        keep = (ids >= 0) & (ids < K)
        ids, codes = ids[keep], codes[keep]
        rho = rnorm[int(doc_off[d]):int(doc_off[d + 1])][keep]
        if ids.size == 0:
            out[j] = -np.inf
            continue
        # first pass: centroid contributions of every token
        sim = C[ids] @ Q.T
        # second pass: residual contributions, one micro-block per (token, subspace)
        res = np.zeros((ids.size, nq))
        for m in range(M):
            res += T[m, codes[:, m], :]
        sim = sim + rho[:, None] * res
        best = sim.max(axis=0)
        s = 0.0
        for i in range(nq):
            s += best[i]
        out[j] = s
    return out
