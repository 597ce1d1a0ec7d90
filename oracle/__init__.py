"""CPU oracle for the token-aware clustering (TAC) build path.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, deliberately simple
NumPy implementation of what the GPU library computes, written from the paper
(Sect. 2.1: tail handling, damped scoring, bounding, budget reconciliation,
per-token k-means, residual compression with product quantisation), the
inverted lists and document layout built from it (Sect. 2.2), and the two
phases of retrieval over that index (Sect. 2.2, its Gather and Refine phases).  Only the
test suite, the smoke check and the CPU-baseline leg of the benchmark may
import it; the product path never does, and it imports nothing from the
product package.

Arithmetic is IEEE float64 unless a function says otherwise.  Where a float
comparison decides an integer (an argmin that picks a centroid or a PQ code),
the oracle offers two decision modes:

* ``"fp64"``: the method's own definition evaluated in float64 -- the
  reference result, compared with a distance-gap tie allowance;
* ``"fp32"``: the same argmin taken on the FP32 distance the kernels define
  as canonical (``oracle.dist32``), so that both sides take the decision in
  the same precision and integer outputs can be compared bit for bit.

Parity status of each function is stated in its module header.
"""
from .group import group_by_token, spreads
from .budget import BudgetParams, budget, cent_offsets
from .lloyd import (assign, update, inertia, init_centroids, lloyd,
                    assign_rows)
from .pq import residuals, pq_encode, pq_train, pq_decode
from .ivf import inverted_lists, doc_layout, decode_layout
from . import dist32

__all__ = [
    "group_by_token", "spreads", "BudgetParams", "budget", "cent_offsets",
    "assign", "update", "inertia", "init_centroids", "lloyd", "assign_rows",
    "residuals", "pq_encode", "pq_train", "pq_decode", "dist32",
    "inverted_lists", "doc_layout", "decode_layout",
]
from .refine import distance_tables, doc_block, maxsim_scores
from .gather import top_centroids, document_scores, document_score_bounds, gather
