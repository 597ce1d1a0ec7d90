"""ctypes binding of libtac (C ABI declared in include/tac.h).

Argument marshalling only: device arrays are torch tensors on the context's
GPU (their ``data_ptr()`` is passed), host arrays are NumPy arrays, and every
computation happens in the HIP kernels of libtac.so.  A missing or unloadable
library raises immediately; there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libtac.so")

TAC_OK, TAC_E_INVAL, TAC_E_INFEASIBLE, TAC_E_NOMEM, TAC_E_HIP, TAC_E_UNSEEN_TOKEN = 0, -1, -2, -3, -4, -5
TAC_FP32, TAC_BF16, TAC_F16 = 0, 1, 2
TAC_THETA_FILL_THEN_RELAX, TAC_THETA_SOFT = 0, 1

_STATUS = {TAC_E_INVAL: "TAC_E_INVAL", TAC_E_INFEASIBLE: "TAC_E_INFEASIBLE", TAC_E_NOMEM: "TAC_E_NOMEM",
           TAC_E_HIP: "TAC_E_HIP", TAC_E_UNSEEN_TOKEN: "TAC_E_UNSEEN_TOKEN"}

EXPORTS = ["tac_ctx_create", "tac_ctx_set_stream", "tac_ctx_destroy", "tac_last_error", "tac_budget", "tac_assign_noalloc",
           "tac_budget_from_stats",
           "tac_init_centroids", "tac_assign", "tac_assign_stats", "tac_update", "tac_residuals", "pq_train",
           "pq_encode", "tac_ctx_enable_timing", "tac_kernel_ms", "tac_ctx_set_tuning", "tac_ctx_get_tuning",
           "tac_ivf_build", "tac_doc_layout", "tac_maxsim", "tac_gather", "tac_ctx_set_static_centroids",
           "tac_assign_workspace_bytes", "tac_graph_build", "tac_graph_search", "tac_gather_lists",
           "tac_centroid_topk"]
TAC_SLOT_ASSIGN, TAC_SLOT_UPDATE, TAC_SLOT_ENCODE = 0, 1, 2


class TacError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class BudgetParams(C.Structure):
    """tac_budget_params; fields left out take the defaults of Sect. 2.1's
    settings (mu 128, tau 256, eps 4, theta 39, fill-then-relax)."""
    _fields_ = [("mu", C.c_int64), ("tau", C.c_int64), ("eps", C.c_int64), ("theta", C.c_double),
                ("theta_policy", C.c_int32)]

    def __init__(self, mu: int = 128, tau: int = 256, eps: int = 4, theta: float = 39.0, theta_policy: int = 0):
        super().__init__(mu, tau, eps, theta, theta_policy)


class Tuning(C.Structure):
    """Launch tuning of tac_assign (results do not depend on it)."""
    _fields_ = [("direct_max_kappa", C.c_int32), ("heavy_kappa", C.c_int32), ("groups_per_cu", C.c_int32),
                ("tile_blocks", C.c_int32), ("waves_per_simd", C.c_int32)]

    def as_dict(self) -> dict:
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


class AssignCounters(C.Structure):
    _fields_ = [("rows", C.c_int64), ("screened", C.c_int64), ("fallback", C.c_int64), ("unassigned", C.c_int64)]


_P = C.c_void_p
_I64 = C.c_int64
_I32 = C.c_int32

_SIGS = {
    "tac_ctx_create": (C.c_int, [C.c_int, _P, C.c_size_t, C.POINTER(_P)]),
    "tac_ctx_set_stream": (C.c_int, [_P, _P]),
    "tac_ctx_destroy": (None, [_P]),
    "tac_ctx_enable_timing": (C.c_int, [_P, C.c_int]),
    "tac_kernel_ms": (C.c_int, [_P, C.c_int, C.POINTER(C.c_float)]),
    "tac_ctx_set_tuning": (C.c_int, [_P, C.POINTER(Tuning)]),
    "tac_ctx_set_static_centroids": (C.c_int, [_P, _P, C.c_int64, C.c_int32]),
    "tac_ctx_get_tuning": (C.c_int, [_P, C.POINTER(Tuning)]),
    "tac_last_error": (C.c_char_p, []),
    "tac_budget": (C.c_int, [_P, _P, _P, _I64, _I32, _I32, _I64, C.POINTER(BudgetParams), _P, _P, _P, _P, _P, _P,
                             _P, _P, _P, _P]),
    "tac_budget_from_stats": (C.c_int, [_P, _P, _I32, _I64, C.POINTER(BudgetParams), _P, _P]),
    "tac_init_centroids": (C.c_int, [_P, _P, _P, _P, _I32, _I32, _P, _I64, _P]),
    "tac_assign": (C.c_int, [_P, _P, _P, _P, _I64, _I32, _I32, _P, _P, _I64, _I32, _P, _P, _P]),
    "tac_assign_noalloc": (C.c_int, [_P, _P, _P, _P, _I64, _I32, _I32, _P, _P, _I64, _I32, _P, _P, _P]),
    "tac_assign_stats": (C.c_int, [_P, C.POINTER(AssignCounters)]),
    "tac_graph_build": (C.c_int, [_P, _P, _I64, _I32, _P]),
    "tac_centroid_topk": (C.c_int, [_P, _P, _I64, _I32, _P, _I64, _I32, _P, _P]),
    "tac_graph_search": (C.c_int, [_P, _P, _I64, _I32, _P, _I64, _P, _P, _I64, _I32, _I32, _P, _P]),
    "tac_gather_lists": (C.c_int, [_P, _P, _P, _I64, _I32, _I32, _P, _P, _I64, _I64, _I32, _P, _P]),
    "tac_assign_workspace_bytes": (C.c_int, [_P, _I64, _I32, _P, _I64, _I32, C.c_int, C.c_int,
                                             C.POINTER(C.c_size_t)]),
    "tac_update": (C.c_int, [_P, _P, _P, _I32, _I64, _I32, _P, _P, _I64, _P, _P]),
    "tac_residuals": (C.c_int, [_P, _P, _P, _P, _I64, _P, _I64, _I32, C.c_int, _P, _P]),
    "pq_train": (C.c_int, [_P, _P, _I64, _I32, _I32, _I32, _I32, _P, _P]),
    "pq_encode": (C.c_int, [_P, _P, _P, _P, _I64, _I64, _I32, _P, _I32, _I32, C.c_int, _P, _P]),
    "tac_ivf_build": (C.c_int, [_P, _P, _P, _I64, _I64, _I64, _P, _P]),
    "tac_doc_layout": (C.c_int, [_P, _P, _P, _I32, _P, _I64, _I64, _P]),
    "tac_maxsim": (C.c_int, [_P, _P, _I64, _I32, _I32, _P, _I64, _P, _I32, _I32, _P, _P, _I64, _I64, _P, _P,
                             _I64, _P]),
    "tac_gather": (C.c_int, [_P, _P, _I64, _I32, _I32, _P, _I64, _P, _P, _I64, _I32, _I32, _P, _P]),
}

_lib = None


def load(path: str = LIB_PATH) -> C.CDLL:
    """Load libtac.so (torch is imported first so both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2604_28142_amd.build`")
    lib = C.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status: int):
    if status != TAC_OK:
        raise TacError(status, load().tac_last_error().decode())


def _dptr(t):
    """Device pointer of a contiguous torch tensor on the GPU (None -> NULL)."""
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("device arguments must be torch tensors on the GPU")
    if not t.is_contiguous():
        raise ValueError("device tensors must be contiguous")
    return t.data_ptr()


def _hptr(a, dtype):
    """Host pointer of a contiguous NumPy array of the given dtype (None -> NULL)."""
    if a is None:
        return None
    if not (isinstance(a, np.ndarray) and a.dtype == dtype and a.flags.c_contiguous):
        raise TypeError(f"host arguments must be C-contiguous numpy {np.dtype(dtype).name} arrays")
    return a.ctypes.data


def _check_dtype(t, dtype, name):
    if t is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}")


class Context:
    """A libtac context on one GPU, enqueueing on a torch stream."""

    def __init__(self, device: int = 0, stream: torch.cuda.Stream | None = None, max_workspace: int = 0):
        lib = load()
        torch.cuda.init()
        self.device = device
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        h = _P()
        _check(lib.tac_ctx_create(device, self.stream.cuda_stream, max_workspace, C.byref(h)))
        self.handle = h
        self.timing_enabled = False

    def set_stream(self, stream: torch.cuda.Stream):
        _check(load().tac_ctx_set_stream(self.handle, stream.cuda_stream))
        self.stream = stream

    def enable_timing(self, on: bool = True):
        _check(load().tac_ctx_enable_timing(self.handle, int(on)))
        self.timing_enabled = bool(on)

    def kernel_ms(self, slot: int) -> float:
        """Elapsed ms of the last recording of a timing slot (HIP events on the context's stream)."""
        v = C.c_float()
        _check(load().tac_kernel_ms(self.handle, slot, C.byref(v)))
        return float(v.value)

    def set_tuning(self, direct_max_kappa: int | None = None, heavy_kappa: int | None = None,
                   groups_per_cu: int | None = None, tile_blocks: int | None = None,
                   waves_per_simd: int | None = None):
        """Change some fields of the context's tac_assign tuning; returns the new tuning as a dict."""
        t = Tuning()
        _check(load().tac_ctx_get_tuning(self.handle, C.byref(t)))
        if direct_max_kappa is not None:
            t.direct_max_kappa = direct_max_kappa
        if heavy_kappa is not None:
            t.heavy_kappa = heavy_kappa
        if groups_per_cu is not None:
            t.groups_per_cu = groups_per_cu
        if tile_blocks is not None:
            t.tile_blocks = tile_blocks
        if waves_per_simd is not None:
            t.waves_per_simd = waves_per_simd
        _check(load().tac_ctx_set_tuning(self.handle, C.byref(t)))
        return t.as_dict()

    def set_static_centroids(self, C_cent, precision: int):
        """Declare C_cent [K, d] float32 unchanging for tac_assign at this precision
        (prepared once; None clears).  C_cent must stay alive and unchanged meanwhile."""
        if C_cent is None:
            _check(load().tac_ctx_set_static_centroids(self.handle, None, 0, 0))
            self._static = None
            return
        _check_dtype(C_cent, torch.float32, "C_cent")
        _check(load().tac_ctx_set_static_centroids(self.handle, _dptr(C_cent), C_cent.shape[0], precision))
        self._static = C_cent          # keeps the tensor alive while declared

    def get_tuning(self) -> dict:
        t = Tuning()
        _check(load().tac_ctx_get_tuning(self.handle, C.byref(t)))
        return t.as_dict()

    def close(self):
        if getattr(self, "handle", None):
            load().tac_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def tac_budget(ctx: Context, x, tok, T: int, K: int, params: BudgetParams | None = None, spread_override=None,
               perm=None, xs=None, seg_off=None, cent_off=None):
    """Group by token and budget.  Returns a dict of host arrays
    (seg_off, counts, spread, kappa, cent_off); device outputs are written in place."""
    N, d = x.shape
    _check_dtype(x, torch.float32, "x")
    _check_dtype(tok, torch.int32, "tok")
    _check_dtype(perm, torch.int32, "perm")
    _check_dtype(seg_off, torch.int64, "seg_off")
    _check_dtype(cent_off, torch.int64, "cent_off")
    out = {"seg_off": np.zeros(T + 1, np.int64), "counts": np.zeros(T, np.int64),
           "spread": np.zeros(T, np.float64), "kappa": np.zeros(T, np.int64), "cent_off": np.zeros(T + 1, np.int64)}
    so = None
    if spread_override is not None:
        spread_override = np.ascontiguousarray(spread_override, dtype=np.float64)
        so = _hptr(spread_override, np.float64)
    _check(load().tac_budget(ctx.handle, _dptr(x), _dptr(tok), N, d, T, K, C.byref(params) if params else None, so,
                             _dptr(perm), _dptr(xs), _dptr(seg_off), _hptr(out["seg_off"], np.int64),
                             _hptr(out["counts"], np.int64), _hptr(out["spread"], np.float64),
                             _hptr(out["kappa"], np.int64), _dptr(cent_off), _hptr(out["cent_off"], np.int64)))
    return out


def tac_budget_from_stats(counts, spread, K: int, params: BudgetParams | None = None):
    """Host-only budget from per-token counts and spreads; returns (kappa int64[T], tier-2 units)."""
    counts = np.ascontiguousarray(counts, dtype=np.int64)
    spread = np.ascontiguousarray(spread, dtype=np.float64)
    T = counts.shape[0]
    kappa = np.zeros(T, np.int64)
    tier2 = np.zeros(1, np.int64)
    _check(load().tac_budget_from_stats(_hptr(counts, np.int64), _hptr(spread, np.float64), T, K,
                                        C.byref(params) if params else None, _hptr(kappa, np.int64),
                                        _hptr(tier2, np.int64)))
    return kappa, int(tier2[0])


def tac_init_centroids(ctx: Context, xs, seg_off, cent_off, picks, C_out):
    T = seg_off.shape[0] - 1
    _check_dtype(picks, torch.int32, "picks")
    _check(load().tac_init_centroids(ctx.handle, _dptr(xs), _dptr(seg_off), _dptr(cent_off), T, xs.shape[1],
                                     _dptr(picks), C_out.shape[0], _dptr(C_out)))


def tac_assign(ctx: Context, x, C_cent, cent_off, assign, seg_off=None, tok=None, precision: int = TAC_FP32,
               dist=None, inertia=None):
    N, d = x.shape
    T = cent_off.shape[0] - 1
    _check_dtype(assign, torch.int32, "assign")
    _check_dtype(dist, torch.float32, "dist")
    _check_dtype(inertia, torch.float64, "inertia")
    _check_dtype(tok, torch.int32, "tok")
    _check(load().tac_assign(ctx.handle, _dptr(x), _dptr(seg_off), _dptr(tok), N, d, T, _dptr(C_cent),
                             _dptr(cent_off), C_cent.shape[0], precision, _dptr(assign), _dptr(dist),
                             _dptr(inertia)))


def tac_assign_noalloc(ctx: Context, x, C_cent, cent_off, assign, seg_off=None, tok=None,
                       precision: int = TAC_FP32, dist=None, inertia=None):
    """tac_assign with the library's fixed per-device scratch instead of the
    context's workspace: allocates nothing (TacError TAC_E_NOMEM when the call
    needs more than the scratch holds)."""
    N, d = x.shape
    T = cent_off.shape[0] - 1
    _check_dtype(assign, torch.int32, "assign")
    _check_dtype(dist, torch.float32, "dist")
    _check_dtype(inertia, torch.float64, "inertia")
    _check_dtype(tok, torch.int32, "tok")
    _check(load().tac_assign_noalloc(ctx.handle, _dptr(x), _dptr(seg_off), _dptr(tok), N, d, T, _dptr(C_cent),
                                     _dptr(cent_off), C_cent.shape[0], precision, _dptr(assign), _dptr(dist),
                                     _dptr(inertia)))


def tac_assign_workspace_bytes(ctx: Context, N: int, T: int, C_cent, K: int, precision: int,
                               with_tok: bool = True, with_dist: bool = True) -> int:
    """Device workspace bytes tac_assign takes on `ctx` for such a call (C_cent
    matters only when the context holds it prepared)."""
    out = C.c_size_t()
    _check(load().tac_assign_workspace_bytes(ctx.handle, N, T, _dptr(C_cent), K,
                                             precision, int(with_tok), int(with_dist), C.byref(out)))
    return int(out.value)


def tac_assign_stats(ctx: Context) -> dict:
    c = AssignCounters()
    _check(load().tac_assign_stats(ctx.handle, C.byref(c)))
    return {"rows": c.rows, "screened": c.screened, "fallback": c.fallback, "unassigned": c.unassigned}


def tac_update(ctx: Context, xs, seg_off, assign, C_old, C_new, count=None):
    N, d = xs.shape
    T = seg_off.shape[0] - 1
    _check_dtype(count, torch.int64, "count")
    _check(load().tac_update(ctx.handle, _dptr(xs), _dptr(seg_off), T, N, d, _dptr(assign), _dptr(C_old),
                             C_old.shape[0], _dptr(C_new), _dptr(count)))


def tac_residuals(ctx: Context, x, assign, C_cent, R, rows=None, normalize: bool = True, rnorm=None):
    n = R.shape[0]
    _check_dtype(rows, torch.int64, "rows")
    _check(load().tac_residuals(ctx.handle, _dptr(x), _dptr(assign), _dptr(C_cent), C_cent.shape[0], _dptr(rows),
                                n, x.shape[1], int(normalize), _dptr(R), _dptr(rnorm)))


def pq_train(ctx: Context, R, init, codebooks, iters: int = 10):
    n, d = R.shape
    M, ksub, _ = init.shape
    _check(load().pq_train(ctx.handle, _dptr(R), n, d, M, ksub, iters, _dptr(init), _dptr(codebooks)))


def pq_encode(ctx: Context, x, assign, C_cent, codebooks, codes, normalize: bool = True, rnorm=None):
    n, d = x.shape
    M, ksub, _ = codebooks.shape
    _check_dtype(codes, torch.uint8, "codes")
    _check(load().pq_encode(ctx.handle, _dptr(x), _dptr(assign), _dptr(C_cent), C_cent.shape[0], n, d,
                            _dptr(codebooks), M, ksub, int(normalize), _dptr(codes), _dptr(rnorm)))


def tac_ivf_build(ctx: Context, assign, doc, K: int, D: int, list_off, list_docs):
    """Inverted lists (Sect. 2.2): list k = list_docs[list_off[k]:list_off[k + 1]], unique increasing
    document ids; list_off[K] entries in all.  assign, doc: int32 [N]; list_off int64 [K + 1];
    list_docs int32 with room for N."""
    N = assign.shape[0]
    _check_dtype(assign, torch.int32, "assign")
    _check_dtype(doc, torch.int32, "doc")
    _check_dtype(list_off, torch.int64, "list_off")
    _check_dtype(list_docs, torch.int32, "list_docs")
    if doc.shape[0] != N or list_off.shape[0] != K + 1 or list_docs.shape[0] < N:
        raise ValueError("tac_ivf_build: inconsistent shapes")
    _check(load().tac_ivf_build(ctx.handle, _dptr(assign), _dptr(doc), N, K, D, _dptr(list_off), _dptr(list_docs)))


def tac_doc_layout(ctx: Context, assign, codes, doc_off, layout):
    """Document layout (Sect. 2.2): per document its centroid ids (int32 LE), then its PQ codes.
    assign int32 [N], codes uint8 [N, M], doc_off int64 [D + 1], layout uint8 [N * (4 + M)]."""
    N, M = codes.shape
    D = doc_off.shape[0] - 1
    _check_dtype(assign, torch.int32, "assign")
    _check_dtype(codes, torch.uint8, "codes")
    _check_dtype(doc_off, torch.int64, "doc_off")
    _check_dtype(layout, torch.uint8, "layout")
    if assign.shape[0] != N or layout.numel() != N * (4 + M):
        raise ValueError("tac_doc_layout: inconsistent shapes")
    _check(load().tac_doc_layout(ctx.handle, _dptr(assign), _dptr(codes), M, _dptr(doc_off), D, N, _dptr(layout)))


def tac_maxsim(ctx: Context, Q, C_cent, codebooks, layout, doc_off, rnorm, cand, scores):
    """Refine phase (Sect. 2.2): MaxSim of every candidate document for its query.
    Q float32 [B, nq, 128]; C_cent [K, 128]; codebooks [32, ksub, 4]; layout uint8 and
    doc_off int64 [D + 1] from tac_doc_layout; rnorm float32 [N] in layout token order;
    cand int32 [B, nc]; scores float32 [B, nc] (output)."""
    B, nq, d = Q.shape
    M, ksub, _ = codebooks.shape
    D = doc_off.shape[0] - 1
    N = rnorm.shape[0]
    _check_dtype(Q, torch.float32, "Q")
    _check_dtype(layout, torch.uint8, "layout")
    _check_dtype(doc_off, torch.int64, "doc_off")
    _check_dtype(rnorm, torch.float32, "rnorm")
    _check_dtype(cand, torch.int32, "cand")
    _check_dtype(scores, torch.float32, "scores")
    if cand.dim() != 2 or cand.shape[0] != B or tuple(scores.shape) != tuple(cand.shape):
        raise ValueError("tac_maxsim: cand and scores must be [B, nc]")
    if layout.shape[0] < N * (4 + M):
        raise ValueError("tac_maxsim: layout is smaller than N * (4 + M) bytes")
    _check(load().tac_maxsim(ctx.handle, _dptr(Q), B, nq, d, _dptr(C_cent), C_cent.shape[0], _dptr(codebooks), M,
                             ksub, _dptr(layout), _dptr(doc_off), D, N, _dptr(rnorm), _dptr(cand), cand.shape[1],
                             _dptr(scores)))


def tac_gather(ctx: Context, Q, C_cent, list_off, list_docs, D: int, kc: int, cand, scores):
    """Gather phase (Sect. 2.2): the kd = cand.shape[1] documents of largest centroid-level
    score per query.  Q float32 [B, nq, 128]; C_cent [K, 128]; list_off int64 [K + 1] and
    list_docs int32 from tac_ivf_build; cand int32 [B, kd] and scores float32 [B, kd] (output).
    Synchronous."""
    B, nq, d = Q.shape
    K = C_cent.shape[0]
    _check_dtype(Q, torch.float32, "Q")
    _check_dtype(list_off, torch.int64, "list_off")
    _check_dtype(list_docs, torch.int32, "list_docs")
    _check_dtype(cand, torch.int32, "cand")
    _check_dtype(scores, torch.float32, "scores")
    if list_off.shape[0] != K + 1 or cand.dim() != 2 or cand.shape[0] != B or tuple(scores.shape) != tuple(cand.shape):
        raise ValueError("tac_gather: inconsistent shapes")
    _check(load().tac_gather(ctx.handle, _dptr(Q), B, nq, d, _dptr(C_cent), K, _dptr(list_off), _dptr(list_docs),
                             D, kc, cand.shape[1], _dptr(cand), _dptr(scores)))


def tac_graph_build(ctx: Context, C_cent, nbr):
    """Neighbour table nbr [K, 64] int32 of the centroid graph (32 nearest, then up to 32 reverse edges)."""
    _check_dtype(nbr, torch.int32, "nbr")
    K, d = C_cent.shape
    if tuple(nbr.shape) != (K, 64):
        raise ValueError("nbr must be [K, 64]")
    _check(load().tac_graph_build(ctx.handle, _dptr(C_cent), K, d, _dptr(nbr)))


def tac_graph_search(ctx: Context, Q, C_cent, nbr, entry, ef: int, kc: int, top_id, top_sim):
    """Top-kc centroids per query-token row of Q [R, 128] by beam search on the graph from the routers `entry`."""
    R, d = Q.shape
    _check(load().tac_graph_search(ctx.handle, _dptr(Q), R, d, _dptr(C_cent), C_cent.shape[0], _dptr(nbr),
                                   _dptr(entry), entry.shape[0], ef, kc, _dptr(top_id), _dptr(top_sim)))


def tac_gather_lists(ctx: Context, top_id, top_sim, list_off, list_docs, K: int, D: int, kd: int, cand, scores):
    """Steps 2-4 of the gather from given top lists top_id / top_sim [B, nq, kc]."""
    B, nq, kc = top_id.shape
    _check(load().tac_gather_lists(ctx.handle, _dptr(top_id), _dptr(top_sim), B, nq, kc, _dptr(list_off),
                                   _dptr(list_docs), K, D, kd, _dptr(cand), _dptr(scores)))


def tac_centroid_topk(ctx: Context, Q, C_cent, kc: int, top_id, top_sim):
    """Exact top-kc centroids by inner product per query-token row of Q [R, 128]."""
    R, d = Q.shape
    _check(load().tac_centroid_topk(ctx.handle, _dptr(Q), R, d, _dptr(C_cent), C_cent.shape[0], kc, _dptr(top_id),
                                    _dptr(top_sim)))
