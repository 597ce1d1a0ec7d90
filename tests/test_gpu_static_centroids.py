"""Centroids declared unchanging (tac_ctx_set_static_centroids): tac_assign with
the declared (C, K, precision) uses the prepared norms, bounds and 16-bit rows
and must return exactly what a call that prepares its own returns; any other
call (another precision, another centroid array, after clearing) prepares its
own and stays exact."""
import numpy as np
import pytest
import torch

import oracle

from gpu_common import dev, host

pytestmark = pytest.mark.gpu

tac = pytest.importorskip("paper_2604_28142_amd")


def problem(seed):
    rng = np.random.default_rng(seed)
    shapes = [(300, 40), (50, 2500), (900, 700), (7, 3), (120, 0)]
    C = rng.standard_normal((sum(k for _, k in shapes), 128)).astype(np.float32)
    C /= np.linalg.norm(C, axis=1, keepdims=True)
    cent_off = np.concatenate([[0], np.cumsum([k for _, k in shapes])]).astype(np.int64)
    xs, tok = [], []
    for j, (n, k) in enumerate(shapes):
        base = C[cent_off[j] + rng.integers(0, k, n)] if k else rng.standard_normal((n, 128))
        xs.append(base + 0.5 * rng.standard_normal((n, 128)) / np.sqrt(128))
        tok.append(np.full(n, j, np.int32))
    x = np.concatenate(xs).astype(np.float32)
    t = np.concatenate(tok)
    order = rng.permutation(x.shape[0])
    return x[order], t[order], C, cent_off


def run(ctx, x, t, C_d, cent_off, prec):
    a = torch.empty(x.shape[0], dtype=torch.int32, device="cuda")
    d = torch.empty(x.shape[0], dtype=torch.float32, device="cuda")
    tac.tac_assign(ctx, dev(x), C_d, dev(cent_off), a, tok=dev(t), precision=prec, dist=d)
    return host(a), host(d), tac.tac_assign_stats(ctx)


def expected(x, t, C, cent_off):
    """The oracle's assignment in input order; rows of a token without centroids get -1."""
    keep = np.nonzero(cent_off[t + 1] > cent_off[t])[0]
    perm, seg_off, _ = oracle.group_by_token(t[keep], len(cent_off) - 1)
    ref = oracle.assign(x[keep][perm], seg_off, C, cent_off, decide="fp32")
    a = np.full(x.shape[0], -1, np.int64)
    a[keep[perm]] = ref["a"]
    return a


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_prepared_equals_per_call(prec):
    x, t, C, cent_off = problem(50 + prec)
    ctx = tac.Context(0)
    try:
        C_d = dev(C)
        a0, d0, s0 = run(ctx, x, t, C_d, cent_off, prec)
        ctx.set_static_centroids(C_d, prec)
        a1, d1, s1 = run(ctx, x, t, C_d, cent_off, prec)
        assert np.array_equal(a0, a1) and np.array_equal(d0.view(np.uint32), d1.view(np.uint32))
        assert s0 == s1
        assert np.array_equal(a1, expected(x, t, C, cent_off))
        other = (prec + 1) % 3                     # not the declared precision: prepares its own
        a2, d2, _ = run(ctx, x, t, C_d, cent_off, other)
        assert np.array_equal(a2, a1) and np.array_equal(d2.view(np.uint32), d1.view(np.uint32))
        ctx.set_static_centroids(None, 0)
        a3, d3, _ = run(ctx, x, t, C_d, cent_off, prec)
        assert np.array_equal(a3, a1) and np.array_equal(d3.view(np.uint32), d1.view(np.uint32))
    finally:
        ctx.close()


def test_declaration_follows_the_array():
    """A call with another centroid array of the same size does not use the
    declared one's preparation; redeclaring replaces it."""
    x, t, C, cent_off = problem(60)
    C2 = np.ascontiguousarray(C[::-1])
    ctx = tac.Context(0)
    try:
        C_d, C2_d = dev(C), dev(C2)
        ctx.set_static_centroids(C_d, tac.TAC_BF16)
        a2, _, _ = run(ctx, x, t, C2_d, cent_off, tac.TAC_BF16)
        assert np.array_equal(a2, expected(x, t, C2, cent_off))
        ctx.set_static_centroids(C2_d, tac.TAC_BF16)
        a2b, _, _ = run(ctx, x, t, C2_d, cent_off, tac.TAC_BF16)
        assert np.array_equal(a2b, a2)
        a1, _, _ = run(ctx, x, t, C_d, cent_off, tac.TAC_BF16)
        assert np.array_equal(a1, expected(x, t, C, cent_off))
        with pytest.raises(tac.TacError):
            tac._lib._check(tac._lib.load().tac_ctx_set_static_centroids(ctx.handle, tac._lib._dptr(C_d), 0, 1))
    finally:
        ctx.close()
