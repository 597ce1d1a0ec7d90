"""Pins of the inverted-list and document-layout oracle (Sect. 2.2): a
hand-worked example, and invariants checked by independent computations."""
import json
import os

import numpy as np

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


def test_hand_example():
    fx = json.load(open(os.path.join(HERE, "golden", "ivf_example.json")))
    off, docs = oracle.inverted_lists(fx["assign"], fx["doc"], fx["K"])
    assert off.tolist() == fx["list_off"] and docs.tolist() == fx["list_docs"]
    lay = oracle.doc_layout(fx["assign"], np.asarray(fx["codes"], np.uint8), fx["doc_off"])
    assert lay.tolist() == fx["layout"]


def test_lists_match_distinct_pairs():
    rng = np.random.default_rng(0)
    n, K, D = 3000, 50, 200
    assign = rng.integers(-1, K, n)
    doc = rng.integers(0, D, n)                       # documents in any order
    off, docs = oracle.inverted_lists(assign, doc, K)
    assert off[0] == 0 and np.all(np.diff(off) >= 0) and off[-1] == docs.size
    valid = assign >= 0
    pairs = np.unique(np.stack([assign[valid], doc[valid]], 1), axis=0)   # sorted by (centroid, doc)
    assert docs.size == pairs.shape[0]
    assert np.array_equal(np.repeat(np.arange(K), np.diff(off)), pairs[:, 0])
    assert np.array_equal(docs, pairs[:, 1])
    for k in range(K):                                # strictly increasing ids per list
        assert np.all(np.diff(docs[off[k]:off[k + 1]]) > 0)


def test_every_token_is_found_from_its_centroid():
    rng = np.random.default_rng(1)
    n, K = 2000, 17
    assign = rng.integers(0, K, n)
    doc = np.sort(rng.integers(0, 300, n))
    off, docs = oracle.inverted_lists(assign, doc, K)
    for t in range(n):
        assert doc[t] in set(docs[off[assign[t]]:off[assign[t] + 1]].tolist())


def test_layout_round_trip_and_offsets():
    rng = np.random.default_rng(2)
    lens = rng.integers(30, 181, 40)
    doc_off = np.concatenate([[0], np.cumsum(lens)])
    n, M = int(doc_off[-1]), 32
    assign = rng.integers(-1, 1 << 20, n)
    codes = rng.integers(0, 256, (n, M)).astype(np.uint8)
    lay = oracle.doc_layout(assign, codes, doc_off)
    assert lay.size == n * (4 + M)
    a2, c2 = oracle.decode_layout(lay, doc_off, M)
    assert np.array_equal(a2, assign) and np.array_equal(c2, codes)
    # document d starts at doc_off[d] * (4 + M): its first centroid id sits there
    for d in range(len(lens)):
        b = int(doc_off[d]) * (4 + M)
        assert int.from_bytes(bytes(lay[b:b + 4]), "little", signed=True) == assign[doc_off[d]]
