"""Oracle for the gather phase of retrieval (Sect. 2.3, "Gather Phase:
Centroid-based Document Scoring").

TEST INFRASTRUCTURE ONLY (see the package docstring).

For a query of n_q token vectors, with the inverted lists of the index
(``inverted_lists``):
1. every query token q_i takes the kappa_c centroids of largest inner product
   <q_i, c_j>;
2. for every such centroid it visits the documents of its inverted list;
3. a document reached through several of q_i's centroids keeps the largest
   similarity: s_i(d) = max_{j : d in L_j} <q_i, c_j>;
4. the partial scores add up over the query tokens: S(q, d) = sum_i s_i(d).
The candidates are then the kappa_d documents of largest S.

Readings (where the paper is silent or approximate):
* step 1 is exact here: the paper finds the centroids with an HNSW graph, an
  approximation of this set; ties go to the lower centroid id;
* a query token that reaches no list of d adds nothing to S(q, d);
* the candidates are ordered by S descending, ties to the lower document id;
  when fewer than kappa_d documents are reached, the rest of the output is
  (-1, -inf);
* the adaptive candidate pruning the paper borrows from other work (its
  parameter alpha) is not part of this function.

Arithmetic is float64; the sum over query tokens is sequential in i.  Pins: a
hand-worked example, brute force over all documents and invariants in
``tests/test_oracle_gather.py``.
"""
import numpy as np


def top_centroids(Q, C, kc):
    """(ids int64 [n_q, kc], sims float64 [n_q, kc]): per query token the kc
    centroids of largest inner product, in that order (ties: lower id first)."""
    Q = np.asarray(Q, dtype=np.float64)
    C = np.asarray(C, dtype=np.float64)
    kc = min(int(kc), C.shape[0])
    sims = Q @ C.T
    ids = np.empty((Q.shape[0], kc), dtype=np.int64)
    for i in range(Q.shape[0]):
        order = np.lexsort((np.arange(C.shape[0]), -sims[i]))   # by -sim, then by id
        ids[i] = order[:kc]
    return ids, np.take_along_axis(sims, ids, axis=1)


def document_scores(Q, C, list_off, list_docs, kc):
    """{document id: S(q, d)} for every document some query token reaches."""
    ids, sims = top_centroids(Q, C, kc)
    S = {}
    for i in range(ids.shape[0]):
        best = {}                                   # s_i(d): the largest similarity reaching d
        for j, s in zip(ids[i].tolist(), sims[i].tolist()):
            for d in np.asarray(list_docs[int(list_off[j]):int(list_off[j + 1])]).tolist():
                if d not in best or s > best[d]:
                    best[d] = s
        for d, s in best.items():                   # query tokens in order i = 0, 1, ...
            S[d] = S.get(d, 0.0) + s
    return S


def gather(Q, C, list_off, list_docs, kc, kd):
    """(docs int32 [kd], scores float64 [kd]): the kd documents of largest S
    (ties: lower id first), padded with (-1, -inf)."""
    S = document_scores(Q, C, list_off, list_docs, kc)
    items = sorted(S.items(), key=lambda t: (-t[1], t[0]))[:kd]
    docs = np.full(kd, -1, dtype=np.int32)
    scores = np.full(kd, -np.inf)
    for r, (d, s) in enumerate(items):
        docs[r] = d
        scores[r] = s
    return docs, scores
