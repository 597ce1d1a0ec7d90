"""GPU parity of the HIP path against the oracle, judged per Lloyd step.

Every call goes through the C ABI (libtac.so via the ctypes binding).  Inputs
come from the seeded generators; every expected value comes from the oracle.
"""
import numpy as np
import pytest
import torch

import datagen
import oracle

from gpu_common import (Case, check_assign, check_centroids, dev, host, lib_params, REL_TOL)

pytestmark = pytest.mark.gpu

tac = pytest.importorskip("paper_2604_28142_amd")


@pytest.fixture(scope="module")
def ctx():
    c = tac.Context(0)
    yield c
    c.close()


_CASES = {}


def case(name):
    if name not in _CASES:
        _CASES[name] = Case(name)
    return _CASES[name]


@pytest.mark.parametrize("name", ["tiny", "small", "c0"])
def test_budget(ctx, name):
    c = case(name)
    N = c.x.shape[0]
    x, tok = dev(c.x), dev(c.tok)
    perm = torch.empty(N, dtype=torch.int32, device="cuda")
    xs = torch.empty_like(x)
    seg = torch.empty(c.T + 1, dtype=torch.int64, device="cuda")
    cent = torch.empty(c.T + 1, dtype=torch.int64, device="cuda")
    out = tac.tac_budget(ctx, x, tok, c.T, c.K, lib_params(name), spread_override=c.spread, perm=perm, xs=xs,
                         seg_off=seg, cent_off=cent)
    assert np.array_equal(host(perm), c.perm)
    assert np.array_equal(host(xs), c.xs)
    assert np.array_equal(host(seg), c.seg_off) and np.array_equal(out["seg_off"], c.seg_off)
    assert np.array_equal(out["counts"], c.counts)
    s = out["spread"]
    err = np.abs(s - c.spread)
    assert np.all(err <= 1e-12 * np.maximum(np.abs(c.spread), 1e-6)), err.max()
    assert np.array_equal(out["kappa"], c.kappa)
    assert np.array_equal(out["cent_off"], c.cent_off) and np.array_equal(host(cent), c.cent_off)
    # with the GPU's own spreads the budget still satisfies every invariant
    out2 = tac.tac_budget(ctx, x, tok, c.T, c.K, lib_params(name), perm=perm)
    assert out2["kappa"].sum() == c.K and np.all(out2["kappa"] <= c.counts)
    # the host-only budget agrees with the oracle given the same statistics
    k, _ = tac.tac_budget_from_stats(c.counts, c.spread, c.K, lib_params(name))
    assert np.array_equal(k, c.kappa)


@pytest.mark.parametrize("name", ["tiny", "small"])
def test_init_centroids(ctx, name):
    c = case(name)
    d = c.device()
    C = torch.empty((c.K, 128), dtype=torch.float32, device="cuda")
    tac.tac_init_centroids(ctx, d["xs"], d["seg_off"], d["cent_off"], dev(c.picks), C)
    assert np.array_equal(host(C), c.C0)
    bad = c.picks.copy()
    bad[0] = c.counts[np.searchsorted(c.cent_off, 0, side="right") - 1]
    with pytest.raises(tac.TacError):
        tac.tac_init_centroids(ctx, d["xs"], d["seg_off"], d["cent_off"], dev(bad), C)


def _gpu_assign(ctx, d, C, prec):
    N = d["xs"].shape[0]
    a = torch.empty(N, dtype=torch.int32, device="cuda")
    dist = torch.empty(N, dtype=torch.float32, device="cuda")
    J = torch.zeros(1, dtype=torch.float64, device="cuda")
    tac.tac_assign(ctx, d["xs"], dev(C), d["cent_off"], a, seg_off=d["seg_off"], precision=prec, dist=dist,
                   inertia=J)
    return host(a), host(dist), float(host(J)[0])


@pytest.mark.parametrize("name,steps", [("tiny", 10), ("small", 4), ("c0", 3)])
def test_lloyd_per_step(ctx, name, steps):
    """Each step starts from the oracle's centroids: assignments bit-exact with the
    FP32-decision oracle (ties only vs float64), inertia within 1e-5, and the update
    fed the oracle's assignments within 1e-5 per centroid with exact counts."""
    c = case(name)
    d = c.device()
    traj = oracle.lloyd(c.xs, c.seg_off, c.cent_off, c.C0, iters=steps, decide="fp32")
    for t, st in enumerate(traj):
        for prec in (tac.TAC_FP32, tac.TAC_BF16, tac.TAC_F16):
            a, dist, J = _gpu_assign(ctx, d, st["C"], prec)
            ties, r64 = check_assign(c.xs, c.seg_off, st["C"], c.cent_off, a, dist)
            assert abs(J - r64["J"]) <= REL_TOL * r64["J"]
            stats = tac.tac_assign_stats(ctx)
            assert stats["rows"] == c.xs.shape[0] and stats["unassigned"] == 0
        if "C_new" not in st:
            continue
        C_new = torch.empty((c.K, 128), dtype=torch.float32, device="cuda")
        cnt = torch.empty(c.K, dtype=torch.int64, device="cuda")
        tac.tac_update(ctx, d["xs"], d["seg_off"], dev(st["a"].astype(np.int32)), dev(st["C"]), C_new, cnt)
        assert np.array_equal(host(cnt), st["counts"])
        check_centroids(host(C_new), st["C_new"])
        empty = st["counts"] == 0
        assert np.array_equal(host(C_new)[empty], st["C"][empty])


def test_determinism_and_precision_identity(ctx):
    c = case("small")
    d = c.device()
    a1, d1, J1 = _gpu_assign(ctx, d, c.C0, tac.TAC_FP32)
    a2, d2, J2 = _gpu_assign(ctx, d, c.C0, tac.TAC_FP32)
    a3, d3, J3 = _gpu_assign(ctx, d, c.C0, tac.TAC_BF16)
    a4, d4, J4 = _gpu_assign(ctx, d, c.C0, tac.TAC_F16)
    assert np.array_equal(a1, a2) and np.array_equal(d1, d2) and J1 == J2
    assert np.array_equal(a1, a3) and np.array_equal(d1, d3) and J1 == J3
    assert np.array_equal(a1, a4) and np.array_equal(d1, d4) and J1 == J4
    C1 = torch.empty((c.K, 128), dtype=torch.float32, device="cuda")
    C2 = torch.empty_like(C1)
    ad = dev(a1)
    tac.tac_update(ctx, d["xs"], d["seg_off"], ad, dev(c.C0), C1)
    tac.tac_update(ctx, d["xs"], d["seg_off"], ad, dev(c.C0), C2)
    assert torch.equal(C1, C2)


@pytest.mark.parametrize("name", ["tiny", "small"])
def test_pq(ctx, name):
    c = case(name)
    d = c.device()
    r = oracle.assign(c.xs, c.seg_off, c.C0, c.cent_off, decide="fp32")
    a = r["a"]
    n = c.xs.shape[0]
    ad, Cd = dev(a.astype(np.int32)), dev(c.C0)
    # residuals: bit-exact with the canonical FP32 sequence
    R = torch.empty((n, 128), dtype=torch.float32, device="cuda")
    rho = torch.empty(n, dtype=torch.float32, device="cuda")
    tac.tac_residuals(ctx, d["xs"], ad, Cd, R, rnorm=rho)
    u32, rho32 = oracle.residuals(c.xs, c.C0[a], mode="fp32")
    assert np.array_equal(host(R), u32) and np.array_equal(host(rho), rho32)
    u64, rho64 = oracle.residuals(c.xs, c.C0[a])
    assert np.allclose(host(rho), rho64, rtol=2e-6, atol=1e-7)
    # training, judged per step from the oracle's codebooks
    ns = min(n, c.w.pq_sample)
    sample = datagen.pq_sample(n, ns, c.w.seed)
    Rs = u32[sample]
    init_rows = datagen.pq_init_rows(ns, 256, c.w.seed)
    cb0 = oracle.pq_train(Rs, 32, 256, 0, init_rows)
    cb = cb0
    Rd = dev(Rs)
    for t in range(3):
        ref = oracle.pq_train(Rs, 32, 256, 1, decide="fp32", init_codebooks=cb)
        out = torch.empty((32, 256, 4), dtype=torch.float32, device="cuda")
        tac.pq_train(ctx, Rd, dev(cb), out, iters=1)
        check_centroids(host(out).reshape(-1, 4), ref.reshape(-1, 4))
        cb = ref
    # several iterations in one call agree with the oracle run the same way
    out = torch.empty((32, 256, 4), dtype=torch.float32, device="cuda")
    tac.pq_train(ctx, Rd, dev(cb0), out, iters=3)
    ref3 = oracle.pq_train(Rs, 32, 256, 3, init_rows, decide="fp32")
    check_centroids(host(out).reshape(-1, 4), ref3.reshape(-1, 4))
    # encoding: fused residual + normalise + argmin, bit-exact with the FP32-decision oracle
    codes = torch.empty((n, 32), dtype=torch.uint8, device="cuda")
    rho2 = torch.empty(n, dtype=torch.float32, device="cuda")
    tac.pq_encode(ctx, d["xs"], ad, Cd, dev(ref3), codes, rnorm=rho2)
    exp32 = oracle.pq_encode(u32, ref3, decide="fp32")
    assert np.array_equal(host(codes), exp32)
    assert np.array_equal(host(rho2), rho32)
    exp64, ti, tD = oracle.pq_encode(u64, ref3, topk=4)
    g = host(codes).astype(np.int64)
    diff = np.nonzero(g != exp64)
    for i, m in zip(*diff):
        hit = np.nonzero(ti[i, m] == g[i, m])[0]
        assert hit.size == 1 and tD[i, m, hit[0]] - tD[i, m, 0] < 1e-5

