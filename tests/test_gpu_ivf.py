"""Inverted lists and document layout on the GPU (Sect. 2.2) against the
oracle, bit for bit: documents in row order and in any order, tokens without
a centroid, empty lists and empty documents, word and byte code widths."""
import numpy as np
import pytest
import torch

import oracle

from gpu_common import dev, host

pytestmark = pytest.mark.gpu

tac = pytest.importorskip("paper_2604_28142_amd")


@pytest.fixture(scope="module")
def ctx():
    c = tac.Context(0)
    yield c
    c.close()


def _ivf(ctx, assign, doc, K, D):
    off = torch.empty(K + 1, dtype=torch.int64, device="cuda")
    docs = torch.full((max(assign.size, 1),), -7, dtype=torch.int32, device="cuda")
    tac.tac_ivf_build(ctx, dev(assign.astype(np.int32)), dev(doc.astype(np.int32)), K, D, off, docs)
    off_h = host(off)
    return off_h, host(docs)[:off_h[-1]]


@pytest.mark.parametrize("ordered", [True, False])
def test_inverted_lists(ctx, ordered):
    rng = np.random.default_rng(30 + ordered)
    n, K, D = 50_000, 3_000, 400
    assign = rng.integers(-1, K, n)
    assign[(assign >= 100) & (assign < 200)] = -1          # centroids 100..199 keep empty lists
    assign[rng.random(n) < 0.01] = K + 5                  # out of range: no list
    doc = np.sort(rng.integers(0, D, n)) if ordered else rng.integers(-2, D + 2, n)
    off, docs = _ivf(ctx, assign, doc, K, D)
    ok = (doc >= 0) & (doc < D)
    ro, rd = oracle.inverted_lists(np.where(ok, assign, -1), doc, K)
    assert np.array_equal(off, ro) and np.array_equal(docs, rd)
    assert (np.diff(off) == 0).any()                        # some lists are empty


def test_inverted_lists_c1_scale(ctx):
    """One C1-sized call (10M tokens, 262,144 lists), checked against invariants
    that hold at any size, plus 2,000 lists checked entry by entry."""
    rng = np.random.default_rng(32)
    n, K = 10_000_000, 262_144
    lens = rng.integers(30, 181, n // 30)
    doc_off = np.concatenate([[0], np.cumsum(lens)])
    D = int(np.searchsorted(doc_off, n, side="right"))
    doc = (np.searchsorted(doc_off, np.arange(n), side="right") - 1).astype(np.int32)
    assign = rng.integers(0, K, n).astype(np.int32)
    off, docs = _ivf(ctx, assign, doc, K, D)
    pairs = np.unique(assign.astype(np.int64) * D + doc)
    assert off[-1] == pairs.size and np.array_equal(docs, (pairs % D).astype(np.int32))
    assert np.array_equal(np.diff(off), np.bincount(pairs // D, minlength=K))


@pytest.mark.parametrize("M", [32, 6])
def test_doc_layout(ctx, M):
    rng = np.random.default_rng(33 + M)
    lens = rng.integers(0, 181, 300)
    lens[:3] = 0                                            # empty documents
    doc_off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    n = int(doc_off[-1])
    assign = rng.integers(-1, 1 << 21, n).astype(np.int32)
    codes = rng.integers(0, 256, (n, M)).astype(np.uint8)
    lay = torch.empty(n * (4 + M), dtype=torch.uint8, device="cuda")
    tac.tac_doc_layout(ctx, dev(assign), dev(codes), dev(doc_off), lay)
    assert np.array_equal(host(lay), oracle.doc_layout(assign, codes, doc_off))


def test_empty_and_bad_sizes(ctx):
    off, docs = _ivf(ctx, np.zeros(0, np.int64), np.zeros(0, np.int64), 5, 3)
    assert np.array_equal(off, np.zeros(6, np.int64)) and docs.size == 0
    with pytest.raises(tac.TacError):
        tac.tac_ivf_build(ctx, dev(np.zeros(4, np.int32)), dev(np.zeros(4, np.int32)), 0, 3,
                          torch.empty(1, dtype=torch.int64, device="cuda"),
                          torch.empty(4, dtype=torch.int32, device="cuda"))
