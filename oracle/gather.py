"""Oracle for the gather phase of retrieval (Sect. 2.2, "Gather Phase:
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


def document_score_bounds(Q, C, list_off, list_docs, kc, tol):
    """Admissible scores when every similarity may carry an error of up to ``tol``.

    An implementation that computes <q_i, c_j> with an error of at most tol and
    then takes its own top-kc per query token can pick any centroid whose exact
    similarity lies within 2 tol of the kc-th largest one (``v_i``): a centroid
    above v_i + 2 tol is always taken, one below v_i - 2 tol never (at least kc
    centroids stay above it).  Over every such choice, s_i(d) (the largest
    similarity among the chosen centroids that reach d, absent when none does)
    lies between the bounds below, so S(q, d) lies in [lo(d), hi(d)], with each
    similarity itself exact here and the rounding allowance left to the caller.

    Returns (sure, lo, hi): ``sure`` the set of documents every choice reaches,
    ``lo`` / ``hi`` dicts over every document some choice reaches (absent
    tokens count 0).  With tol = 0 and no equal similarities across any cut,
    lo = hi = document_scores.
    """
    Q = np.asarray(Q, dtype=np.float64)
    C = np.asarray(C, dtype=np.float64)
    K = C.shape[0]
    kc = min(int(kc), K)
    sims = Q @ C.T
    lo, hi = {}, {}
    sure = None
    for i in range(Q.shape[0]):
        v = np.sort(sims[i])[::-1][kc - 1]
        if kc >= K:
            must = np.arange(K)
            maybe = np.zeros(0, dtype=np.int64)
        else:
            must = np.nonzero(sims[i] > v + 2 * tol)[0]
            maybe = np.nonzero((sims[i] >= v - 2 * tol) & (sims[i] <= v + 2 * tol))[0]
            if must.size + maybe.size == kc:         # no choice left: every optional centroid is taken
                must = np.concatenate([must, maybe])
                maybe = maybe[:0]
        sure_i = {}                                  # d -> max similarity over the centroids always taken
        for j in must.tolist():
            s = sims[i, j]
            for d in np.asarray(list_docs[int(list_off[j]):int(list_off[j + 1])]).tolist():
                if d not in sure_i or s > sure_i[d]:
                    sure_i[d] = s
        amb_min, amb_max = {}, {}                    # d -> min / max similarity over the optional centroids
        for j in maybe.tolist():
            s = sims[i, j]
            for d in np.asarray(list_docs[int(list_off[j]):int(list_off[j + 1])]).tolist():
                amb_min[d] = min(amb_min.get(d, s), s)
                amb_max[d] = max(amb_max.get(d, s), s)
        for d in set(sure_i) | set(amb_max):
            if d in sure_i:
                l_i = sure_i[d]
                h_i = max(sure_i[d], amb_max.get(d, -np.inf))
            else:                                    # reached or not, depending on the choice
                l_i = min(0.0, amb_min[d])
                h_i = max(0.0, amb_max[d])
            lo[d] = lo.get(d, 0.0) + l_i
            hi[d] = hi.get(d, 0.0) + h_i
        sure = set(sure_i) if sure is None else sure | set(sure_i)
    return (sure or set()), lo, hi
