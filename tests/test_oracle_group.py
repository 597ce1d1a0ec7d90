"""Pins for the oracle's grouping and per-token spread (Sect. 2.1, Phase 2)."""
import numpy as np

import datagen
from oracle.group import group_by_token, spreads


def test_stable_grouping():
    rng = np.random.default_rng(1)
    tok = rng.integers(0, 50, 5000).astype(np.int32)
    perm, seg_off, counts = group_by_token(tok, 60)
    # ascending token, and inside a token ascending original row
    keys = tok[perm].astype(np.int64) * 10**6 + perm
    assert np.all(np.diff(keys) > 0)
    for j in range(60):
        rows = [i for i in range(tok.shape[0]) if tok[i] == j]
        assert perm[seg_off[j]:seg_off[j + 1]].tolist() == rows
        assert counts[j] == len(rows)
    assert seg_off[-1] == tok.shape[0]


def test_spread_closed_forms():
    d = 128
    e = np.eye(d, dtype=np.float32)
    xs = np.stack([e[0], e[1], e[5], e[5], e[5]])
    seg_off = np.array([0, 2, 5, 5])
    s = spreads(xs, seg_off)
    assert s[0] == 0.5          # two orthonormal vectors
    assert s[1] == 0.0          # identical vectors
    assert s[2] == 0.0          # absent token


def test_spread_unit_vectors_identity():
    """For unit vectors, (1/n) sum ||x - m||^2 = 1 - ||m||^2."""
    x, tok = datagen.make("tiny")
    perm, seg_off, counts = group_by_token(tok, 40)
    xs = x[perm]
    s = spreads(xs, seg_off)
    for j in range(40):
        if counts[j] == 0:
            continue
        X = xs[seg_off[j]:seg_off[j + 1]].astype(np.float64)
        nrm2 = np.einsum("ij,ij->i", X, X)
        m = X.mean(axis=0)
        expect = nrm2.mean() - m @ m
        assert abs(s[j] - expect) <= 1e-13 * max(1.0, expect)
        assert abs(s[j] - (1.0 - m @ m)) <= 1e-6


def test_generator_statistics():
    """Synthetic stand-in check: a heavy head (Sect. 2.1 reports 41-45% of all
    vectors in the 100 most frequent tokens on the real collections)."""
    w = datagen.WORKLOADS["c1"]
    tok = datagen.tokens(400_000, w.vocab, w.zipf_s, 0)
    c = np.sort(np.bincount(tok, minlength=w.vocab))[::-1]
    share = c[:100].sum() / c.sum()
    assert 0.44 < share < 0.51
    x, tok0 = datagen.make("c0")
    assert x.shape == (200_000, 128) and x.dtype == np.float32
    assert np.allclose(np.linalg.norm(x[:1000], axis=1), 1.0, atol=1e-6)
    c0 = np.sort(np.bincount(tok0, minlength=2000))[::-1]
    assert 0.68 < c0[:100].sum() / c0.sum() < 0.76
