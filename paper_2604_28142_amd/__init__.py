"""MI355X (gfx950) token-aware clustering: the index-build hot path of Tachiom.

The work runs in libtac.so (HIP kernels behind the C ABI of include/tac.h);
this package holds the ctypes binding (``_lib``), the in-tree build script
(``build``) and the drivers that chain the calls (``index``, ``serve``).
"""
from ._lib import (TAC_BF16, TAC_F16, TAC_FP32, TAC_THETA_FILL_THEN_RELAX, TAC_THETA_SOFT, BudgetParams, Context,
                   TacError, Tuning, load, pq_encode, pq_train, tac_assign, tac_assign_noalloc, tac_assign_stats, tac_budget,
                   tac_budget_from_stats, tac_centroid_topk, tac_doc_layout, tac_gather, tac_gather_lists,
                   tac_graph_build, tac_graph_search, tac_init_centroids, tac_ivf_build, tac_maxsim, tac_residuals,
                   tac_update)

__all__ = ["TAC_BF16", "TAC_F16", "TAC_FP32", "TAC_THETA_FILL_THEN_RELAX", "TAC_THETA_SOFT", "BudgetParams", "Context",
           "TacError", "Tuning", "load", "pq_encode", "pq_train", "tac_assign", "tac_assign_noalloc", "tac_assign_stats", "tac_budget",
           "tac_budget_from_stats", "tac_centroid_topk", "tac_doc_layout", "tac_gather", "tac_gather_lists",
           "tac_graph_build", "tac_graph_search", "tac_init_centroids", "tac_ivf_build", "tac_maxsim", "tac_residuals",
           "tac_update"]
