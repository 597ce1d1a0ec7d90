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

The centroid graph the GPU path searches instead of the paper's HNSW
(``knn_graph``), its best-first search (``beam_search``) and steps 2-4 from
given top lists (``gather_from_top``) follow at the end; their pins (a
hand-worked graph, the search reaching the exact set when the beam covers
every centroid, greedy walks on a path graph, agreement with ``gather``) are
in ``tests/test_oracle_graph.py``.
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


# ---- the centroid graph (Sect. 2.2, "Index Structure") ---------------------------
# The paper searches the centroids with an HNSW graph (M = 32 neighbours); the GPU
# path builds a flat neighbour graph instead and searches it best-first.  These
# functions state that graph and that search plainly, in float64, so that the
# GPU's can be checked against them.

def _key_order(sims, ids):
    """Positions of (sims, ids) by similarity descending, then id ascending."""
    return np.lexsort((np.asarray(ids), -np.asarray(sims)))


def knn_graph(C, deg=32):
    """Neighbour table int64 [K, 2 deg]: row i lists the deg centroids j != i of
    largest <c_i, c_j> (ties: lower id), then up to deg reverse edges: the
    centroids j whose own list holds i and that i does not list, largest <c_i,
    c_j> first (ties: lower id); -1 fills the rest."""
    C = np.asarray(C, dtype=np.float64)
    K = C.shape[0]
    S = C @ C.T
    nbr = np.full((K, 2 * deg), -1, dtype=np.int64)
    fwd = []
    for i in range(K):
        others = np.array([j for j in range(K) if j != i], dtype=np.int64)
        order = others[_key_order(S[i, others], others)][:deg]
        nbr[i, :order.size] = order
        fwd.append(set(order.tolist()))
    for i in range(K):
        cands = np.array([j for j in range(K) if i in fwd[j] and j not in fwd[i]], dtype=np.int64)
        if cands.size:
            order = cands[_key_order(S[i, cands], cands)][:deg]
            nbr[i, deg:deg + order.size] = order
    return nbr


def beam_search(q, C, nbr, entry, ef, kc):
    """Best-first search of the neighbour graph for one query token q.

    The ef entry centroids of largest <q, c> (ties: lower id) start the beam;
    while the beam holds an entry not yet expanded, its best such entry is
    expanded: each neighbour (in column order) not seen before is scored, and
    the beam keeps the ef best of its entries and the new ones.  Returns (ids,
    sims) of the kc best, padded with (-1, -inf)."""
    q = np.asarray(q, dtype=np.float64)
    C = np.asarray(C, dtype=np.float64)
    entry = np.asarray(entry, dtype=np.int64)
    es = C[entry] @ q
    start = entry[_key_order(es, entry)][:ef]
    seen = set(start.tolist())
    beam = [(float(C[j] @ q), int(j), False) for j in start.tolist()]

    def top(items):
        items = sorted(items, key=lambda t: (-t[0], t[1]))
        return items[:ef]

    beam = top(beam)
    while True:
        open_ = [t for t in beam if not t[2]]
        if not open_:
            break
        s, j, _ = open_[0]
        beam = [(a, b, True) if b == j else (a, b, c) for a, b, c in beam]
        new = []
        for n in np.asarray(nbr[j]).tolist():
            if n < 0 or n in seen:
                continue
            seen.add(n)
            new.append((float(C[n] @ q), int(n), False))
        beam = top(beam + new)
    ids = np.full(kc, -1, dtype=np.int64)
    sims = np.full(kc, -np.inf)
    for r, (s, j, _) in enumerate(beam[:kc]):
        ids[r] = j
        sims[r] = s
    return ids, sims


def gather_from_top(ids, sims, list_off, list_docs, kd):
    """Steps 2-4 of the gather for one query whose per-token top lists are given
    (ids [n_q, kc], -1 for an empty slot; sims [n_q, kc]): (docs int32 [kd],
    scores float64 [kd]) as ``gather`` returns them."""
    S = {}
    for i in range(ids.shape[0]):
        best = {}
        for j, s in zip(np.asarray(ids[i]).tolist(), np.asarray(sims[i], dtype=np.float64).tolist()):
            if j < 0:
                continue
            for d in np.asarray(list_docs[int(list_off[j]):int(list_off[j + 1])]).tolist():
                if d not in best or s > best[d]:
                    best[d] = s
        for d, s in best.items():
            S[d] = S.get(d, 0.0) + s
    items = sorted(S.items(), key=lambda t: (-t[1], t[0]))[:kd]
    docs = np.full(kd, -1, dtype=np.int32)
    scores = np.full(kd, -np.inf)
    for r, (d, s) in enumerate(items):
        docs[r] = d
        scores[r] = s
    return docs, scores
