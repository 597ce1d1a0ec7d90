"""Shared helpers for the GPU parity tests (inputs from datagen, expectations from oracle)."""
import numpy as np
import torch

import datagen
import oracle
from oracle.budget import BudgetParams as OParams

TIE_GAP = 1e-5   # an FP32 pick may differ from the float64 argmin only on a smaller distance gap
REL_TOL = 1e-5   # centroids, inertia and codebooks: relative tolerance

# Budget parameters per workload: the paper's values (Sect. 3.1) for the larger
# cases, scaled down for the tiny one so that it has tail and active tokens.
PARAMS = {
    "tiny": dict(mu=20, tau=60, eps=2, theta=10.0),
    "small": dict(mu=128, tau=256, eps=4, theta=39.0),
    "c0": dict(mu=128, tau=256, eps=4, theta=39.0),
    "c1": dict(mu=128, tau=256, eps=4, theta=39.0),
}


def lib_params(name, policy=0):
    import paper_2604_28142_amd as tac
    p = PARAMS[name]
    return tac.BudgetParams(p["mu"], p["tau"], p["eps"], p["theta"], policy)


def oracle_params(name, policy=0):
    p = PARAMS[name]
    return OParams(mu=p["mu"], tau=p["tau"], eps=p["eps"], theta=p["theta"], policy=policy)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.cpu().numpy()


class Case:
    """One workload grouped and budgeted by the oracle, with its seeded initial centroids."""

    def __init__(self, name, n=None):
        w = datagen.WORKLOADS[name]
        self.name = name
        self.w = w
        self.x, self.tok = datagen.make(w, n)
        self.T = w.vocab
        self.K = w.k
        self.perm, self.seg_off, self.counts = oracle.group_by_token(self.tok, self.T)
        self.xs = self.x[self.perm]
        self.spread = oracle.spreads(self.xs, self.seg_off)
        self.kappa = oracle.budget(self.counts, self.spread, self.K, oracle_params(name))
        self.cent_off = oracle.cent_offsets(self.kappa)
        self.picks = datagen.init_picks(self.counts, self.kappa, w.seed)
        self.C0 = oracle.init_centroids(self.xs, self.seg_off, self.cent_off, self.picks)

    def device(self):
        return dict(xs=dev(self.xs), seg_off=dev(self.seg_off), cent_off=dev(self.cent_off))


def check_assign(xs, seg_off, C, cent_off, a_gpu, d_gpu, rows=None, fp64=True):
    """Compare GPU assignments with both oracle decision modes.

    Bit-exact against the FP32-decision oracle (same canonical distance); against
    the float64 oracle a different pick is a counted tie only if its float64
    distance is within TIE_GAP of the minimum.  Returns the tie count."""
    if rows is None:
        r32 = oracle.assign(xs, seg_off, C, cent_off, decide="fp32")
        r64 = oracle.assign(xs, seg_off, C, cent_off, decide="fp64", topk=8)
    else:
        r32 = oracle.assign_rows(xs, rows, seg_off, C, cent_off, decide="fp32")
        r64 = oracle.assign_rows(xs, rows, seg_off, C, cent_off, decide="fp64", topk=8)
    a_gpu = np.asarray(a_gpu, dtype=np.int64)
    bad = np.nonzero(a_gpu != r32["a"])[0]
    assert bad.size == 0, f"{bad.size} assignments differ from the FP32-decision oracle, first rows {bad[:8]}"
    assert np.array_equal(np.asarray(d_gpu, dtype=np.float32), r32["d32"]), "canonical distances differ"
    if not fp64:
        return 0, r64
    diff = np.nonzero(a_gpu != r64["a"])[0]
    for i in diff:
        hit = np.nonzero(r64["top_idx"][i] == a_gpu[i])[0]
        assert hit.size == 1, f"row {i}: pick {a_gpu[i]} not among the 8 nearest"
        gap = r64["top_D"][i, hit[0]] - r64["top_D"][i, 0]
        assert gap < TIE_GAP, f"row {i}: distance gap {gap} is not a tie"
    return int(diff.size), r64


def check_centroids(C_gpu, C_ref):
    nrm = np.linalg.norm(C_ref.astype(np.float64), axis=1)
    err = np.linalg.norm(C_gpu.astype(np.float64) - C_ref.astype(np.float64), axis=1)
    tol = np.where(nrm < 1e-3, 1e-8, REL_TOL * nrm)
    bad = np.nonzero(err > tol)[0]
    assert bad.size == 0, f"{bad.size} centroids off, worst rel {np.max(err / np.maximum(nrm, 1e-30))}"
