"""Oracle for the index structures built from the clustering (Sect. 2.2).

TEST INFRASTRUCTURE ONLY (see the package docstring).

* ``inverted_lists`` follows "Index Structure": every centroid keeps an inverted
  list of the ids of the documents whose tokens are assigned to it.  Readings:
  a document appears once per list however many of its tokens the centroid
  holds, ids are in increasing order, and tokens without a centroid (assignment
  -1) enter no list.
* ``doc_layout`` follows "Document Layout": per document, the centroid ids of all
  of its tokens stored contiguously, followed by all of their PQ codes.  Reading:
  the codes are token-major (the M codes of the first token, then of the
  second, ...), the order of the [N, M] code array; centroid ids are 4-byte
  little-endian integers, so document d starts at byte doc_off[d] * (4 + M).

Both are written out directly from those definitions with Python sets and
byte strings.  Pins: a hand-worked example and invariants in
``tests/test_oracle_ivf.py``.
"""
import numpy as np


def inverted_lists(assign, doc, K):
    """Returns (list_off int64[K + 1], list_docs int32[total]): list k is
    list_docs[list_off[k]:list_off[k + 1]]."""
    assign = np.asarray(assign, dtype=np.int64)
    doc = np.asarray(doc, dtype=np.int64)
    lists = [set() for _ in range(K)]
    for a, d in zip(assign.tolist(), doc.tolist()):
        if 0 <= a < K:
            lists[a].add(d)
    off = [0]
    docs = []
    for k in range(K):
        docs.extend(sorted(lists[k]))
        off.append(len(docs))
    return np.asarray(off, dtype=np.int64), np.asarray(docs, dtype=np.int32)


def doc_layout(assign, codes, doc_off):
    """Returns the layout bytes (uint8[N * (4 + M)]) of the documents whose
    tokens are rows doc_off[d] .. doc_off[d + 1] - 1."""
    assign = np.asarray(assign, dtype=np.int64)
    codes = np.asarray(codes, dtype=np.uint8)
    out = bytearray()
    for d in range(len(doc_off) - 1):
        b, e = int(doc_off[d]), int(doc_off[d + 1])
        for t in range(b, e):
            out += int(assign[t]).to_bytes(4, "little", signed=True)
        for t in range(b, e):
            out += bytes(codes[t])
    return np.frombuffer(bytes(out), dtype=np.uint8).copy()


def decode_layout(layout, doc_off, M):
    """Inverse of doc_layout: (assign int64[N], codes uint8[N, M])."""
    n = int(doc_off[-1])
    assign = np.empty(n, dtype=np.int64)
    codes = np.empty((n, M), dtype=np.uint8)
    for d in range(len(doc_off) - 1):
        b, e = int(doc_off[d]), int(doc_off[d + 1])
        base = b * (4 + M)
        for i in range(e - b):
            assign[b + i] = int.from_bytes(bytes(layout[base + 4 * i: base + 4 * i + 4]), "little", signed=True)
        cb = base + 4 * (e - b)
        for i in range(e - b):
            codes[b + i] = layout[cb + M * i: cb + M * (i + 1)]
    return assign, codes
