"""The 16-bit screens' split route through the C ABI: a token of at most 8,192
rows and at least 2,048 centroids (a serving batch's frequent token) is
screened as (320-row tile, 1,024-centroid chunk) work items spread over the
device, and the chunks' exact minima meet per row.  Its results must equal the oracle's FP32-decision assignment
bit for bit, like every other route: across chunk edges, with ties between
chunks, with certificates that fail in several chunks, and on the serving path."""
import numpy as np
import pytest
import torch

import oracle

from gpu_common import check_assign, dev, host

pytestmark = pytest.mark.gpu

tac = pytest.importorskip("paper_2604_28142_amd")


@pytest.fixture(scope="module")
def ctx():
    c = tac.Context(0)
    yield c
    c.close()


def run_assign(ctx, xs, seg_off, C, cent_off, prec):
    N = xs.shape[0]
    a = torch.empty(N, dtype=torch.int32, device="cuda")
    d = torch.empty(N, dtype=torch.float32, device="cuda")
    tac.tac_assign(ctx, dev(xs), dev(C), dev(cent_off), a, seg_off=dev(seg_off), precision=prec, dist=d)
    return host(a), host(d)


def unit(rng, n):
    v = rng.standard_normal((n, 128))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def token_data(rng, n, k):
    """n rows near k random centroids (rows drawn around the centroids, so the
    nearest centroid is usually clear but not always the one a row was drawn at)."""
    C = unit(rng, k)
    x = C[rng.integers(0, k, n)] + 0.6 * rng.standard_normal((n, 128)) / np.sqrt(128)
    return x.astype(np.float32), C.astype(np.float32)


def build(tokens):
    xs = np.concatenate([x for x, _ in tokens])
    C = np.concatenate([c for _, c in tokens])
    seg_off = np.concatenate([[0], np.cumsum([x.shape[0] for x, _ in tokens])]).astype(np.int64)
    cent_off = np.concatenate([[0], np.cumsum([c.shape[0] for _, c in tokens])]).astype(np.int64)
    return xs, seg_off, C, cent_off


@pytest.mark.parametrize("prec", [1, 2])
def test_split_tokens_match_oracle(ctx, prec):
    """Split tokens at the route's limits (8,192 rows in 26 ragged tiles; 2,048
    centroids; partial last chunks) beside tokens just outside it (8,193 rows;
    2,047 centroids) and a direct token, all in one call: every row equals the
    FP32 path bit for bit, and a sample of rows (all of the small tokens) the
    oracle."""
    rng = np.random.default_rng(40)
    shapes = [(80, 5000), (1, 2048), (3, 2047), (8193, 2048), (10, 4), (321, 2100), (8192, 1025 + 2048)]
    xs, seg_off, C, cent_off = build([token_data(rng, n, k) for n, k in shapes])
    a, d = run_assign(ctx, xs, seg_off, C, cent_off, prec)
    st = tac.tac_assign_stats(ctx)
    assert st["rows"] == xs.shape[0] and st["screened"] == xs.shape[0] - 10    # the direct token is not screened
    a32, d32 = run_assign(ctx, xs, seg_off, C, cent_off, tac.TAC_FP32)
    assert np.array_equal(a, a32) and np.array_equal(d.view(np.uint32), d32.view(np.uint32))
    big = [3, 6]
    rows = np.concatenate([np.arange(seg_off[j], seg_off[j + 1]) for j in range(len(shapes)) if j not in big] +
                          [rng.choice(np.arange(seg_off[j], seg_off[j + 1]), 400, replace=False) for j in big])
    rows = np.sort(rows)
    check_assign(xs, seg_off, C, cent_off, a[rows], d[rows], rows=rows)


@pytest.mark.parametrize("prec", [1, 2])
def test_exact_ties_across_chunks(ctx, prec):
    """Copies of one centroid in three different chunks, and rows equal to it:
    every chunk finds the same distance, and the lowest index must win."""
    rng = np.random.default_rng(41)
    x, C = token_data(rng, 60, 3500)
    for src, copies in ((5, (1030, 2100)), (1500, (3400,)), (2047, (2048, 3071))):
        for c in copies:
            C[c] = C[src]
    x[:10] = C[5]
    x[10:20] = C[1500]
    x[20:30] = C[2047]
    xs, seg_off, Cc, cent_off = build([(x, C)])
    a, d = run_assign(ctx, xs, seg_off, Cc, cent_off, prec)
    check_assign(xs, seg_off, Cc, cent_off, a, d)
    assert np.all(a[:10] == 5) and np.all(a[10:20] == 1500) and np.all(a[20:30] == 2047)


@pytest.mark.parametrize("prec", [1, 2])
def test_certificate_fails_in_many_chunks(ctx, prec):
    """Centroids nearly equidistant from every row defeat the certificate in
    every chunk of both row tiles; each row is queued once (at most one
    fallback per row) and the token-wide rescoring returns the exact argmin."""
    rng = np.random.default_rng(42)
    k, n = 3000, 400
    C = (unit(rng, k) * (1.0 + 1e-7 * rng.standard_normal((k, 1)))).astype(np.float32)
    x = (1e-7 * rng.standard_normal((n, 128))).astype(np.float32)
    xs, seg_off, Cc, cent_off = build([(x, C)])
    a, d = run_assign(ctx, xs, seg_off, Cc, cent_off, prec)
    fb = tac.tac_assign_stats(ctx)["fallback"]
    assert 0 < fb <= n
    check_assign(xs, seg_off, Cc, cent_off, a, d, fp64=False)


@pytest.mark.parametrize("prec", [1, 2])
def test_serving_path_with_split_tokens(ctx, prec):
    """Token ids in any order (the serving path groups them): three split tokens
    and two ordinary ones, checked against the sorted oracle."""
    rng = np.random.default_rng(43)
    shapes = [(700, 4100), (20, 300), (5, 2600), (200, 2500), (2100, 2200)]
    toks = [token_data(rng, n, k) for n, k in shapes]
    xs, seg_off, C, cent_off = build(toks)
    tok = np.repeat(np.arange(len(shapes), dtype=np.int32), [n for n, _ in shapes])
    order = rng.permutation(xs.shape[0])
    x_u, t_u = xs[order].copy(), tok[order].copy()
    a = torch.empty(xs.shape[0], dtype=torch.int32, device="cuda")
    d = torch.empty(xs.shape[0], dtype=torch.float32, device="cuda")
    tac.tac_assign(ctx, dev(x_u), dev(C), dev(cent_off), a, tok=dev(t_u), precision=prec, dist=d)
    ref = oracle.assign(xs, seg_off, C, cent_off, decide="fp32")
    assert np.array_equal(host(a), ref["a"][order])
    assert np.array_equal(host(d), ref["d32"][order])
