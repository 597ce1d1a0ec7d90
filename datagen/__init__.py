"""Seeded synthetic inputs for the token-aware clustering (TAC) build path.

This module holds only random-number draws and their reshaping into inputs:
token ids, token vectors, the seeded initial-centroid picks, the PQ training
sample and serving requests.  It contains none of the method's arithmetic
(no grouping, statistics, budget, distances, means or quantisation), so both
the CPU oracle and the GPU path may import it.

The paper evaluates on ColBERTv2 token embeddings of MS MARCO v1 and LoTTE
(Sect. 3), which are not available here; these generators stand in for them
with the shapes the paper states: 128-d L2-normalised token vectors carrying a
token id from a BERT-sized vocabulary, with a heavy-tailed (Zipf) token
frequency so that the most frequent ~100 ids hold a large share of all
vectors (Sect. 2.1 reports 41-45%).

Every draw comes from ``numpy.random.default_rng([seed, stream, ...])`` with a
fixed stream number, and large arrays are drawn in fixed chunks of
``CHUNK`` rows, each chunk with its own key, so the result does not depend on
how many threads generate it.

Streams: 0 token uniforms, 1 per-token means, 2 per-token sub-centres,
3 vector noise, 4 initial-centroid picks, 5 PQ sample, 6 PQ initial rows,
7 id permutation, 8 serving documents, 9 serving arrivals, 10 sub-centre pick
and document lengths, 11 queries.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

CHUNK = 1 << 18  # rows per independently keyed chunk
DIM = 128


@dataclass(frozen=True)
class Workload:
    """One synthetic workload: sizes and distribution parameters."""
    name: str
    n: int                 # number of token vectors
    vocab: int             # number of token ids
    zipf_s: float          # Zipf exponent of token frequencies
    subcentres: int        # sub-clusters per token (1 = one mean per token)
    sigma: float           # total noise norm before renormalisation
    k: int                 # total centroid budget
    iters: int = 10        # Lloyd iterations
    pq_m: int = 32         # PQ subspaces
    pq_ksub: int = 256     # codes per subspace
    pq_sample: int = 0     # PQ training sample (0 = no PQ)
    seed: int = 0
    extra: dict = field(default_factory=dict)


# The workloads the build is measured and checked on.
WORKLOADS = {
    # CPU-finishable: 200k vectors, 2,000 ids, Zipf 1.1, one mean per token.
    "c0": Workload("c0", 200_000, 2_000, 1.1, 1, 0.30, 8_192, pq_sample=50_000),
    # 10M vectors, 30,522 ids, Zipf 1.0, four sub-centres per token.
    "c1": Workload("c1", 10_000_000, 30_522, 1.0, 4, 0.25, 262_144, pq_sample=1_000_000),
    # 50M vectors with the c1 generator and 2^21 centroids.
    "c3": Workload("c3", 50_000_000, 30_522, 1.0, 4, 0.25, 2_097_152, pq_sample=1_000_000),
    # Small cases for unit and parity tests.
    "tiny": Workload("tiny", 6_000, 40, 1.1, 2, 0.30, 300, pq_sample=2_000),
    "small": Workload("small", 60_000, 400, 1.0, 4, 0.25, 2_048, pq_sample=20_000),
}


def _threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def zipf_cdf(vocab: int, s: float) -> np.ndarray:
    """CDF of the finite Zipf law p_k ~ k^-s over ranks 1..vocab (last entry exactly 1)."""
    p = np.arange(1, vocab + 1, dtype=np.float64) ** (-s)
    cdf = np.cumsum(p)
    cdf /= cdf[-1]
    cdf[-1] = 1.0
    return cdf


def id_permutation(vocab: int, seed: int) -> np.ndarray:
    """Seeded map from frequency rank (0-based) to token id, so id order != frequency order."""
    return np.random.default_rng([seed, 7]).permutation(vocab).astype(np.int32)


def tokens(n: int, vocab: int, s: float, seed: int) -> np.ndarray:
    """int32[n] token ids drawn from the finite Zipf law, ids permuted by stream 7."""
    cdf = zipf_cdf(vocab, s)
    perm = id_permutation(vocab, seed)
    out = np.empty(n, dtype=np.int32)

    def chunk(c):
        lo, hi = c * CHUNK, min(n, (c + 1) * CHUNK)
        u = np.random.default_rng([seed, 0, c]).random(hi - lo)
        rank = np.searchsorted(cdf, u, side="right")
        out[lo:hi] = perm[rank]

    nchunks = (n + CHUNK - 1) // CHUNK
    with ThreadPoolExecutor(_threads()) as ex:
        list(ex.map(chunk, range(nchunks)))
    return out


def centres(vocab: int, sub: int, seed: int, dim: int = DIM) -> np.ndarray:
    """float32[vocab, sub, dim] random unit vectors (stream 1 when sub == 1, else stream 2)."""
    stream = 1 if sub == 1 else 2
    g = np.random.default_rng([seed, stream]).standard_normal((vocab, sub, dim))
    g /= np.linalg.norm(g, axis=-1, keepdims=True)
    return g.astype(np.float32)


def vectors(tok: np.ndarray, cen: np.ndarray, sigma: float, seed: int,
            noise_stream: int = 3, pick_stream: int = 10) -> np.ndarray:
    """float32[n, dim]: x = normalise(centre + (sigma / sqrt(dim)) * z), z ~ N(0, I).

    The centre is the token's mean, or one of its sub-centres picked uniformly.
    """
    n = tok.shape[0]
    sub, dim = cen.shape[1], cen.shape[2]
    scale = np.float32(sigma / np.sqrt(dim))
    out = np.empty((n, dim), dtype=np.float32)

    def chunk(c):
        lo, hi = c * CHUNK, min(n, (c + 1) * CHUNK)
        z = np.random.default_rng([seed, noise_stream, c]).standard_normal((hi - lo, dim), dtype=np.float32)
        if sub > 1:
            pick = np.random.default_rng([seed, pick_stream, c]).integers(0, sub, hi - lo)
            base = cen[tok[lo:hi], pick]
        else:
            base = cen[tok[lo:hi], 0]
        v = base + scale * z
        nrm = np.sqrt(np.einsum("ij,ij->i", v, v, dtype=np.float64)).astype(np.float32)
        out[lo:hi] = v / nrm[:, None]

    nchunks = (n + CHUNK - 1) // CHUNK
    with ThreadPoolExecutor(_threads()) as ex:
        list(ex.map(chunk, range(nchunks)))
    return out


def make(w: Workload | str, n: int | None = None):
    """(x float32[n,128], tok int32[n]) for a workload; ``n`` truncates the row count."""
    if isinstance(w, str):
        w = WORKLOADS[w]
    n = w.n if n is None else n
    tok = tokens(n, w.vocab, w.zipf_s, w.seed)
    cen = centres(w.vocab, w.subcentres, w.seed)
    x = vectors(tok, cen, w.sigma, w.seed)
    return x, tok


def init_picks(counts: np.ndarray, kappa: np.ndarray, seed: int) -> np.ndarray:
    """int32[sum kappa]: for each token j in ascending id order, kappa_j distinct
    segment-local row indices in [0, n_j), drawn by default_rng([seed, 4, j]).

    Initial centroid cent_off_j + l is row seg_off_j + pick[cent_off_j + l] of
    the token-sorted vectors (the paper does not state an initialisation).
    """
    out = np.empty(int(kappa.sum()), dtype=np.int32)
    pos = 0
    for j in range(counts.shape[0]):
        k = int(kappa[j])
        if k == 0:
            continue
        rng = np.random.default_rng([seed, 4, j])
        out[pos:pos + k] = rng.choice(int(counts[j]), size=k, replace=False)
        pos += k
    return out


def pq_sample(n: int, size: int, seed: int) -> np.ndarray:
    """int64[size]: sorted distinct positions of the PQ training rows (stream 5)."""
    size = min(size, n)
    return np.sort(np.random.default_rng([seed, 5]).choice(n, size=size, replace=False))


def pq_init_rows(size: int, ksub: int, seed: int) -> np.ndarray:
    """int64[ksub]: which training rows seed every subspace's codebook (stream 6)."""
    return np.random.default_rng([seed, 6]).permutation(size)[:ksub]


def build_doc_offsets(n: int, seed: int = 0, lo: int = 30, hi: int = 180) -> np.ndarray:
    """int64[D + 1]: the build's vectors, in input order, cut into documents of
    U{lo..hi} consecutive vectors (the last one shorter; stream 10)."""
    rng = np.random.default_rng([seed, 10])
    lens = rng.integers(lo, hi + 1, size=n // lo + 1)
    off = np.concatenate([[0], np.cumsum(lens)])
    D = int(np.searchsorted(off, n, side="left"))
    off = off[:D + 1].copy()
    off[-1] = n
    return off.astype(np.int64)


def serving_docs(w: Workload | str, ndocs: int, seed: int = 0, lo: int = 30, hi: int = 180):
    """Documents for the encode service: n_d ~ U{lo..hi} vectors each, token ids
    from the workload's Zipf law and vectors around the same centres with fresh
    noise (stream 8).  Returns (doc_len int32[ndocs], x float32[sum,128], tok int32[sum])."""
    if isinstance(w, str):
        w = WORKLOADS[w]
    rng = np.random.default_rng([seed, 8])
    lens = rng.integers(lo, hi + 1, size=ndocs).astype(np.int32)
    total = int(lens.sum())
    cdf = zipf_cdf(w.vocab, w.zipf_s)
    perm = id_permutation(w.vocab, w.seed)
    tok = perm[np.searchsorted(cdf, rng.random(total), side="right")].astype(np.int32)
    cen = centres(w.vocab, w.subcentres, w.seed)
    x = vectors(tok, cen, w.sigma, seed + 1000, noise_stream=8, pick_stream=8)
    return lens, x, tok


def poisson_arrivals(rate: float, count: int, seed: int = 0) -> np.ndarray:
    """float64[count] arrival times (s) of a Poisson process of the given rate (stream 9)."""
    gaps = np.random.default_rng([seed, 9]).exponential(1.0 / rate, size=count)
    return np.cumsum(gaps)


def queries(w: Workload | str, count: int, nq: int = 32, seed: int = 0) -> np.ndarray:
    """float32[count, nq, 128]: query token vectors, token ids from the workload's
    Zipf law and vectors around the same centres with fresh noise (stream 11).
    nq = 32 is the fixed query length of ColBERTv2-style encoders."""
    if isinstance(w, str):
        w = WORKLOADS[w]
    rng = np.random.default_rng([seed, 11])
    cdf = zipf_cdf(w.vocab, w.zipf_s)
    perm = id_permutation(w.vocab, w.seed)
    tok = perm[np.searchsorted(cdf, rng.random(count * nq), side="right")].astype(np.int32)
    cen = centres(w.vocab, w.subcentres, w.seed)
    x = vectors(tok, cen, w.sigma, seed + 2000, noise_stream=11, pick_stream=11)
    return x.reshape(count, nq, -1)

