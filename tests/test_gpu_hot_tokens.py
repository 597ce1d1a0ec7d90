"""The persistent assignment kernel at the token shapes that dominate the 10M-row
workload (30,522 Zipf(1.0) ids, 262,144 centroids): tokens of more than 8,192
rows (so the 16-bit screens keep them on the persistent kernel rather than the
split route) with 4,097, 8,192 and 23,485 centroids -- 5 to 23 epochs of 1,024
centroids, ragged last stages and epochs, ragged last row tiles -- in all three
screens, plus a check of the whole 10M-row workload on a row sample that holds
rows of every one of its five largest tokens.

Rows are drawn like the workload's (four sub-centres per token, noise norm
0.25, renormalised).  Centroids are the seeded initial rows, or one float64
Lloyd step of the oracle from them, which packs them closer together (more
near-ties for the certificates).  Every expected value comes from the oracle:
assignments and canonical distances bit-exact against its FP32-decision mode,
float64 differences only as ties below 1e-5."""
import numpy as np
import pytest
import torch

import datagen
import oracle

from gpu_common import TIE_GAP, check_centroids, dev, host, oracle_params

pytestmark = pytest.mark.gpu

tac = pytest.importorskip("paper_2604_28142_amd")

PRECS = (tac.TAC_FP32, tac.TAC_BF16, tac.TAC_F16) if hasattr(tac, "TAC_F16") else ()


@pytest.fixture(scope="module")
def ctx():
    c = tac.Context(0)
    yield c
    c.close()


def token_rows(rng, n):
    """n rows of one token: four random unit sub-centres, noise norm 0.25."""
    cen = rng.standard_normal((4, 128))
    cen /= np.linalg.norm(cen, axis=1, keepdims=True)
    x = cen[rng.integers(0, 4, n)] + (0.25 / np.sqrt(128)) * rng.standard_normal((n, 128))
    return (x / np.linalg.norm(x, axis=1, keepdims=True)).astype(np.float32)


def gpu_assign(ctx, xs_d, seg_d, C, cent_off, prec):
    N = xs_d.shape[0]
    a = torch.empty(N, dtype=torch.int32, device="cuda")
    d = torch.empty(N, dtype=torch.float32, device="cuda")
    tac.tac_assign(ctx, xs_d, dev(C), dev(cent_off), a, seg_off=seg_d, precision=prec, dist=d)
    return host(a).astype(np.int64), host(d)


def compare(rows, a, d, r32, r64):
    """Bit-exact against the FP32-decision oracle; float64 differences only as ties."""
    bad = np.nonzero(a[rows] != r32["a"])[0]
    assert bad.size == 0, f"{bad.size} of {rows.size} sampled rows differ, first rows {rows[bad[:8]]}"
    assert np.array_equal(d[rows].view(np.uint32), r32["d32"].view(np.uint32)), "canonical distances differ"
    diff = np.nonzero(a[rows] != r64["a"])[0]
    for i in diff:
        hit = np.nonzero(r64["top_idx"][i] == a[rows][i])[0]
        assert hit.size == 1, f"row {rows[i]}: pick not among the 8 nearest"
        assert r64["top_D"][i, hit[0]] - r64["top_D"][i, 0] < TIE_GAP
    return int(diff.size)


# (rows, centroids): > 8,192 rows each; 23,485 = 22 epochs + 957 (the largest
# token's budget in the 10M-row workload), 8,192 = 8 whole epochs, 4,097 = 4
# epochs + one centroid; 5,000 and 2,500 centroids beside them
HOT = [(30_000, 23_485), (12_001, 8_192), (9_000, 4_097), (8_193, 5_000), (9_001, 2_500)]


def hot_case(seed, trained):
    rng = np.random.default_rng(seed)
    xs = np.concatenate([token_rows(rng, n) for n, _ in HOT])
    seg_off = np.concatenate([[0], np.cumsum([n for n, _ in HOT])]).astype(np.int64)
    cent_off = np.concatenate([[0], np.cumsum([k for _, k in HOT])]).astype(np.int64)
    C = np.concatenate([xs[seg_off[j] + rng.choice(n, k, replace=False)] for j, (n, k) in enumerate(HOT)])
    if trained:
        r = oracle.assign(xs, seg_off, C, cent_off)
        C, _ = oracle.update(xs, r["a"], C)
    rows = np.concatenate([np.sort(rng.choice(np.arange(seg_off[j], seg_off[j + 1]), 2_000, replace=False))
                           for j in range(len(HOT))])
    # the last rows of every token (its ragged last tile) are always in the sample
    tails = np.concatenate([np.arange(seg_off[j + 1] - 40, seg_off[j + 1]) for j in range(len(HOT))])
    rows = np.unique(np.concatenate([rows, tails]))
    return xs, seg_off, C, cent_off, rows


@pytest.mark.parametrize("trained", [False, True])
def test_hot_tokens_persistent_route(ctx, trained):
    """Five tokens of 8,193-30,000 rows and 2,500-23,485 centroids in one call
    per screen: sampled rows (2,000 per token plus each token's last 40) are
    bit-exact against the FP32-decision oracle, and all rows agree across the
    three screens bit for bit."""
    xs, seg_off, C, cent_off, rows = hot_case(50 + int(trained), trained)
    r32 = oracle.assign_rows(xs, rows, seg_off, C, cent_off, decide="fp32")
    r64 = oracle.assign_rows(xs, rows, seg_off, C, cent_off, decide="fp64", topk=8)
    xs_d, seg_d = dev(xs), dev(seg_off)
    ref = None
    for prec in PRECS:
        a, d = gpu_assign(ctx, xs_d, seg_d, C, cent_off, prec)
        st = tac.tac_assign_stats(ctx)
        # every row went through the persistent screen: none is left unassigned
        assert st["rows"] == xs.shape[0] and st["screened"] == xs.shape[0] and st["unassigned"] == 0
        print(f"prec {prec} trained {trained}: {st['fallback']} certificate fallbacks")
        compare(rows, a, d, r32, r64)
        if ref is None:
            ref = (a, d)
        else:
            assert np.array_equal(a, ref[0]) and np.array_equal(d.view(np.uint32), ref[1].view(np.uint32))


@pytest.fixture(scope="module")
def c1():
    """The 10M-row workload grouped, budgeted and initialised by the oracle."""
    w = datagen.WORKLOADS["c1"]
    x, tok = datagen.make(w)
    perm, seg_off, counts = oracle.group_by_token(tok, w.vocab)
    del tok
    xs = x[perm]
    del x, perm
    s = oracle.spreads(xs, seg_off)
    kappa = oracle.budget(counts, s, w.k, oracle_params("c1"))
    cent_off = oracle.cent_offsets(kappa)
    C0 = oracle.init_centroids(xs, seg_off, cent_off, datagen.init_picks(counts, kappa, w.seed))
    out = dict(w=w, xs=xs, seg_off=seg_off, counts=counts, kappa=kappa, cent_off=cent_off, C0=C0,
               xs_d=dev(xs), seg_d=dev(seg_off))
    yield out
    out.clear()
    torch.cuda.empty_cache()


def test_c1_sampled_assign(ctx, c1):
    """The whole 10M-row, 262,144-centroid workload assigned on the GPU from
    the seeded initial centroids in all three screens.  About 175k rows are
    compared with the oracle: 15,000 of each of the five largest tokens (up to
    23,485 centroids), every row of 50 random tokens and 80,000 uniform rows;
    all 10M rows agree across the screens."""
    xs, seg_off, cent_off, C0, counts = c1["xs"], c1["seg_off"], c1["cent_off"], c1["C0"], c1["counts"]
    rng = np.random.default_rng(60)
    top5 = np.argsort(-counts, kind="stable")[:5]
    assert c1["kappa"][top5].max() == 23_485
    parts = [rng.choice(np.arange(seg_off[j], seg_off[j + 1]), 15_000, replace=False) for j in top5]
    present = np.nonzero(counts)[0]
    for j in rng.choice(present, 50, replace=False):
        parts.append(np.arange(seg_off[j], seg_off[j + 1]))
    parts.append(rng.choice(xs.shape[0], 80_000, replace=False))
    rows = np.unique(np.concatenate(parts))
    r32 = oracle.assign_rows(xs, rows, seg_off, C0, cent_off, decide="fp32")
    r64 = oracle.assign_rows(xs, rows, seg_off, C0, cent_off, decide="fp64", topk=8)
    ref = None
    for prec in PRECS:
        a, d = gpu_assign(ctx, c1["xs_d"], c1["seg_d"], C0, cent_off, prec)
        st = tac.tac_assign_stats(ctx)
        assert st["rows"] == xs.shape[0] and st["unassigned"] == 0
        ties = compare(rows, a, d, r32, r64)
        print(f"c1 prec {prec}: {rows.size} sampled rows, {ties} float64 ties, {st['fallback']} fallbacks")
        if ref is None:
            ref = a
        else:
            assert np.array_equal(a, ref)


def test_c1_update(ctx, c1):
    """A seeded random assignment of all 10M rows (each inside its token's
    centroids) averaged by tac_update against the oracle's float64 means: the
    tokens above 65,536 rows sum in float64 on the GPU, the others in
    compensated float32; counts exact."""
    xs, counts, kappa, cent_off, C0, w = c1["xs"], c1["counts"], c1["kappa"], c1["cent_off"], c1["C0"], c1["w"]
    rng = np.random.default_rng(61)
    seg = np.repeat(np.arange(w.vocab), counts)
    a_r = cent_off[seg] + (rng.random(xs.shape[0]) * kappa[seg]).astype(np.int64)
    del seg
    C_new, cnt_ref = oracle.update(xs, a_r, C0)
    Cn = torch.empty((w.k, 128), dtype=torch.float32, device="cuda")
    cnt = torch.empty(w.k, dtype=torch.int64, device="cuda")
    tac.tac_update(ctx, c1["xs_d"], c1["seg_d"], dev(a_r.astype(np.int32)), dev(C0), Cn, cnt)
    assert np.array_equal(host(cnt), cnt_ref)
    check_centroids(host(Cn), C_new)
