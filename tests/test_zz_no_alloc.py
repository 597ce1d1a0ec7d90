"""tac_assign_noalloc (the assignment without any allocation, for callers that
cannot allocate) through the C ABI: its assignments, canonical distances and
inertia equal tac_assign's bit for bit on two calls in a row, the second with
a smaller input, on sorted segments and on the serving path; a call whose
workspace would not fit the fixed scratch is refused before anything runs,
and preparing the centroids once brings a large index within it."""
import numpy as np
import pytest
import torch

from gpu_common import Case, dev, host

pytestmark = pytest.mark.gpu

tac = pytest.importorskip("paper_2604_28142_amd")


@pytest.fixture(scope="module")
def ctx():
    c = tac.Context(0)
    yield c
    c.close()


def run(fn, ctx, x, C, cent_off, prec, seg_off=None, tok=None):
    N = x.shape[0]
    a = torch.full((N,), -7, dtype=torch.int32, device="cuda")
    d = torch.full((N,), -7.0, dtype=torch.float32, device="cuda")
    J = torch.full((1,), -7.0, dtype=torch.float64, device="cuda")
    fn(ctx, x, C, cent_off, a, seg_off=seg_off, tok=tok, precision=prec, dist=d, inertia=J)
    torch.cuda.synchronize()
    return host(a), host(d), host(J)


def same(r1, r2):
    assert np.array_equal(r1[0], r2[0]), "assignments differ"
    assert np.array_equal(r1[1].view(np.uint32), r2[1].view(np.uint32)), "distances differ"
    assert np.array_equal(r1[2].view(np.uint64), r2[2].view(np.uint64)), "inertia differs"
    assert np.all(r1[0] >= 0)


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_sorted_segments_two_calls(ctx, prec):
    """The 60k-row, 400-token case: all rows, then only the rows of the first
    150 tokens (a smaller input on the same scratch)."""
    c = Case("small")
    xs, seg, coff, C = dev(c.xs), dev(c.seg_off), dev(c.cent_off), dev(c.C0)
    n2 = int(c.seg_off[150])
    seg2 = dev(np.minimum(c.seg_off, n2))
    for x_d, s_d in ((xs, seg), (xs[:n2], seg2)):
        ref = run(tac.tac_assign, ctx, x_d, C, coff, prec, seg_off=s_d)
        got = run(tac.tac_assign_noalloc, ctx, x_d, C, coff, prec, seg_off=s_d)
        same(got, ref)


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_serving_path_two_calls(ctx, prec):
    """Unsorted rows with token ids (grouped inside the call): 5,000 rows, then
    1,200 rows of other tokens."""
    c = Case("small")
    rng = np.random.default_rng(70)
    coff, C = dev(c.cent_off), dev(c.C0)
    for n in (5000, 1200):
        rows = rng.choice(c.x.shape[0], n, replace=False)
        x_d, tok_d = dev(c.x[rows]), dev(c.tok[rows])
        ref = run(tac.tac_assign, ctx, x_d, C, coff, prec, tok=tok_d)
        got = run(tac.tac_assign_noalloc, ctx, x_d, C, coff, prec, tok=tok_d)
        same(got, ref)


def test_large_index_needs_prepared_centroids(ctx):
    """200,000 BF16 centroids over 3,000 tokens: staging their 16-bit rows per
    call needs more than the scratch holds, so the call is refused and its
    outputs stay untouched; with the centroids prepared once on the context the
    same call runs, twice (4,000 then 900 rows), and equals tac_assign."""
    rng = np.random.default_rng(71)
    T, K = 3000, 200_000
    kap = np.full(T, (K - 20_000) // (T - 1), dtype=np.int64)
    kap[0] = 20_000
    kap[-1] += K - kap.sum()
    cent_off = np.concatenate([[0], np.cumsum(kap)]).astype(np.int64)
    Cn = rng.standard_normal((K, 128))
    C = (Cn / np.linalg.norm(Cn, axis=1, keepdims=True)).astype(np.float32)
    C_d, coff = dev(C), dev(cent_off)
    prec = tac.TAC_BF16

    def batch(n):
        tok = np.where(rng.random(n) < 0.3, 0, rng.integers(0, T, n)).astype(np.int32)
        k = cent_off[tok] + (rng.random(n) * kap[tok]).astype(np.int64)
        x = C[k] + 0.3 * rng.standard_normal((n, 128)) / np.sqrt(128)
        return dev((x / np.linalg.norm(x, axis=1, keepdims=True)).astype(np.float32)), dev(tok)

    x_d, tok_d = batch(4000)
    a = torch.full((4000,), -7, dtype=torch.int32, device="cuda")
    with pytest.raises(tac.TacError, match="scratch"):
        tac.tac_assign_noalloc(ctx, x_d, C_d, coff, a, tok=tok_d, precision=prec)
    torch.cuda.synchronize()
    assert torch.all(a == -7)
    ctx.set_static_centroids(C_d, prec)
    try:
        for n in (4000, 900):
            x_d, tok_d = batch(n)
            ref = run(tac.tac_assign, ctx, x_d, C_d, coff, prec, tok=tok_d)
            got = run(tac.tac_assign_noalloc, ctx, x_d, C_d, coff, prec, tok=tok_d)
            same(got, ref)
    finally:
        ctx.set_static_centroids(None, prec)
