"""GPU edge cases through the C ABI: empty inputs, class boundaries of the
assignment kernel, epoch flushes, forced certificate fallbacks, exact ties on
dyadic inputs, the serving path's token grouping, and graph replay."""
import numpy as np
import pytest
import torch

import datagen
import oracle

from gpu_common import Case, check_assign, check_centroids, dev, host

pytestmark = pytest.mark.gpu

tac = pytest.importorskip("paper_2604_28142_amd")


@pytest.fixture(scope="module")
def ctx():
    c = tac.Context(0)
    yield c
    c.close()


def run_assign(ctx, xs, seg_off, C, cent_off, prec):
    N = xs.shape[0]
    a = torch.empty(max(N, 1), dtype=torch.int32, device="cuda")[:N]
    d = torch.empty(max(N, 1), dtype=torch.float32, device="cuda")[:N]
    J = torch.zeros(1, dtype=torch.float64, device="cuda")
    tac.tac_assign(ctx, dev(xs), dev(C), dev(cent_off), a, seg_off=dev(seg_off), precision=prec, dist=d, inertia=J)
    return host(a), host(d), float(host(J)[0])


def clustered(rng, n, k, spread=0.05):
    centres = rng.standard_normal((k, 128))
    centres /= np.linalg.norm(centres, axis=1, keepdims=True)
    x = centres[rng.integers(0, k, n)] + spread * rng.standard_normal((n, 128)) / np.sqrt(128)
    return (x / np.linalg.norm(x, axis=1, keepdims=True)).astype(np.float32)


def test_empty_inputs(ctx):
    x = torch.empty((0, 128), dtype=torch.float32, device="cuda")
    tok = torch.empty(0, dtype=torch.int32, device="cuda")
    perm = torch.empty(0, dtype=torch.int32, device="cuda")
    out = tac.tac_budget(ctx, x, tok, 5, 0, perm=perm)
    assert out["kappa"].sum() == 0 and np.all(out["seg_off"] == 0)
    with pytest.raises(tac.TacError):
        tac.tac_budget(ctx, x, tok, 5, 3, perm=perm)          # infeasible: no vectors
    a, d, J = run_assign(ctx, np.zeros((0, 128), np.float32), np.zeros(6, np.int64),
                         np.zeros((2, 128), np.float32), np.array([0, 1, 1, 2, 2, 2]), tac.TAC_BF16)
    assert a.shape == (0,) and J == 0.0


@pytest.mark.parametrize("kappa", [1, 2, 4, 5, 16, 17, 63, 64, 65, 300])
@pytest.mark.parametrize("prec", [0, 1, 2])
def test_class_boundaries_and_ragged_tiles(ctx, kappa, prec):
    rng = np.random.default_rng(kappa)
    sizes = [kappa, 3 * kappa + 7, 513, 1030]        # ragged against 16-row blocks and 512-row tiles
    xs = np.concatenate([clustered(rng, n, max(2, kappa // 2)) for n in sizes])
    seg_off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    picks = np.concatenate([rng.choice(n, kappa, replace=False) for n in sizes]).astype(np.int64)
    cent_off = np.arange(len(sizes) + 1, dtype=np.int64) * kappa
    C = np.concatenate([xs[seg_off[j] + picks[cent_off[j]:cent_off[j + 1]]] for j in range(len(sizes))])
    a, d, J = run_assign(ctx, xs, seg_off, C, cent_off, prec)
    ties, r64 = check_assign(xs, seg_off, C, cent_off, a, d)
    assert abs(J - r64["J"]) <= 1e-5 * max(r64["J"], 1e-30)


@pytest.mark.parametrize("n,route", [(9000, "persistent"), (6000, "split")])
def test_heavy_token_epoch_flush(ctx, n, route):
    """A token with 2,500 centroids spans three packed-index epochs (the last
    one ragged).  With 9,000 rows the 16-bit screens keep it on the persistent
    kernel; with 6,000 rows (at most 8,192) they cut it into the split route's
    1,024-centroid chunks.  FP32 runs the persistent kernel either way."""
    rng = np.random.default_rng(11)
    xs = clustered(rng, n, 400, spread=0.3)
    C = xs[rng.choice(n, 2500, replace=False)].copy()
    seg_off = np.array([0, n], np.int64)
    cent_off = np.array([0, 2500], np.int64)
    for prec in (0, 1, 2):
        a, d, J = run_assign(ctx, xs, seg_off, C, cent_off, prec)
        assert tac.tac_assign_stats(ctx)["rows"] == n
        check_assign(xs, seg_off, C, cent_off, a, d)


@pytest.mark.parametrize("scale", [1.0, 1.0e12, 1.0e-12])
def test_forced_certificate_fallback(ctx, scale):
    """Centroids nearly equidistant from every row defeat the screen's
    certificate; the fallback's rescoring still returns the exact argmin, also
    with every vector scaled far up or down (the fallback's own screen bound at
    large and small magnitudes)."""
    rng = np.random.default_rng(12)
    k = 700
    dirs = rng.standard_normal((k, 128))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    C = (scale * dirs * (1.0 + 1e-7 * rng.standard_normal((k, 1)))).astype(np.float32)
    xs = (scale * 1e-7 * rng.standard_normal((300, 128))).astype(np.float32)
    seg_off = np.array([0, 300], np.int64)
    cent_off = np.array([0, k], np.int64)
    for prec in (0, 1, 2):
        a, d, J = run_assign(ctx, xs, seg_off, C, cent_off, prec)
        assert tac.tac_assign_stats(ctx)["fallback"] > 0
        check_assign(xs, seg_off, C, cent_off, a, d, fp64=False)


def test_f16_operand_range(ctx):
    """The FP16 screen rounds x and c to FP16; rows and centroids beyond its
    range (or deep in its subnormals) leave no finite bound, so those rows are
    rescored exhaustively, and every row still gets the exact FP32 argmin."""
    rng = np.random.default_rng(16)
    sizes = [300, 260, 250]
    xs = np.concatenate([clustered(rng, n, 5) for n in sizes])
    xs[:20] *= 1.0e5                        # token 0: some rows past the FP16 range (|2x| > 65504)
    xs[300:560] *= 1.0e-6                   # token 1: tiny rows, FP16 subnormals
    seg_off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    kap = [40, 40, 40]
    cent_off = np.concatenate([[0], np.cumsum(kap)]).astype(np.int64)
    C = np.concatenate([xs[seg_off[j] + rng.choice(sizes[j], kap[j], replace=False)] for j in range(3)])
    C[-1] *= 1.0e5                          # one centroid past the range: the bound is infinite everywhere
    a, d, J = run_assign(ctx, xs, seg_off, C, cent_off, tac.TAC_F16)
    assert tac.tac_assign_stats(ctx)["fallback"] > 0
    check_assign(xs, seg_off, C, cent_off, a, d, fp64=False)
    a0, d0, J0 = run_assign(ctx, xs, seg_off, C, cent_off, tac.TAC_FP32)
    assert np.array_equal(a, a0) and np.array_equal(d, d0)


def test_update_long_runs(ctx):
    """Clusters far longer than one summation chunk, in a float64 token
    (more than 65,536 rows) and in a compensated-float32 token: means within
    1e-5 of the float64 oracle, exact counts, bitwise-equal repeated calls, and
    empty clusters keep their old centroid."""
    rng = np.random.default_rng(17)
    sizes = [70000, 3000, 40]
    xs = np.concatenate([clustered(rng, n, 3, spread=0.5) for n in sizes])
    seg_off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    kap = [3, 4, 2]
    cent_off = np.concatenate([[0], np.cumsum(kap)]).astype(np.int64)
    K = int(cent_off[-1])
    C_old = rng.standard_normal((K, 128)).astype(np.float32)
    a = np.empty(xs.shape[0], np.int64)
    a[:70000] = rng.choice([0, 1], 70000, p=[0.9, 0.1])        # centroid 2 stays empty
    a[70000:73000] = 3 + rng.choice([0, 1, 3], 3000)          # 1 of token 1 (centroid 5) stays empty
    a[73000:] = 7 + rng.integers(0, 2, 40)
    C1, cnt1 = oracle.update(xs, a, C_old)
    outs = []
    for _ in range(2):
        Cn = torch.empty((K, 128), dtype=torch.float32, device="cuda")
        cnt = torch.empty(K, dtype=torch.int64, device="cuda")
        tac.tac_update(ctx, dev(xs), dev(seg_off), dev(a.astype(np.int32)), dev(C_old), Cn, cnt)
        assert np.array_equal(host(cnt), cnt1)
        check_centroids(host(Cn), C1)
        outs.append(host(Cn))
    assert np.array_equal(outs[0], outs[1])
    empty = cnt1 == 0
    assert empty.sum() == 2 and np.array_equal(outs[0][empty], C_old[empty])


def _kahan32(vals):
    """Compensated float32 sum of the rows of `vals` in row order, returned as s - c."""
    s = np.zeros(vals.shape[1], np.float32)
    c = np.zeros(vals.shape[1], np.float32)
    for v in vals:
        y = v - c
        t = s + y
        c = (t - s) - y
        s = t
    return s - c


def _means_in_member_order(xs, a, K, wide_rows, chunk=256):
    """The update's arithmetic written out: members in ascending row order,
    runs above `chunk` members summed chunk by chunk and the chunk sums added in
    chunk order; float64 sums for the centroids in `wide_rows`, compensated
    float32 sums otherwise."""
    out = np.zeros((K, xs.shape[1]), np.float32)
    for k in range(K):
        m = xs[np.flatnonzero(a == k)]
        n = m.shape[0]
        if n == 0:
            continue
        parts = [m] if n <= chunk else [m[i:i + chunk] for i in range(0, n, chunk)]
        if k in wide_rows:
            sums = [np.cumsum(p.astype(np.float64), axis=0)[-1] for p in parts]
            tot = np.cumsum(np.stack(sums), axis=0)[-1]
            out[k] = (tot / n).astype(np.float32)
        else:
            sums = np.stack([_kahan32(p) for p in parts]).astype(np.float32)
            tot = sums[0] if len(parts) == 1 else _kahan32(sums)
            out[k] = tot / np.float32(n)
    return out


def test_update_run_length_boundaries(ctx):
    """Cluster sizes at every boundary of the update's loops (16-row load
    rounds, 64-index groups, 256-member chunks), members interleaved across
    each token, in a compensated-float32 token and a float64 one (more than
    65,536 rows): exact counts, means within 1e-5 of the float64 oracle, and
    bitwise equal to the update's summation order written out in numpy."""
    rng = np.random.default_rng(29)
    lens32 = [1, 2, 15, 16, 17, 31, 63, 64, 65, 127, 128, 129, 255, 256, 257, 300, 511, 512, 513, 1000, 0]
    lens64 = [65, 257, 66000, 0]
    xs, a, seg, k0 = [], [], [0], 0
    for lens in (lens32, lens64):
        lab = np.repeat(np.arange(len(lens)), lens)
        rng.shuffle(lab)
        xs.append(clustered(rng, lab.size, 4, spread=0.5))
        a.append(k0 + lab)
        seg.append(seg[-1] + lab.size)
        k0 += len(lens)
    xs = np.concatenate(xs)
    a = np.concatenate(a).astype(np.int64)
    seg_off = np.array(seg, np.int64)
    K = k0
    C_old = rng.standard_normal((K, 128)).astype(np.float32)
    C1, cnt1 = oracle.update(xs, a, C_old)
    Cn = torch.empty((K, 128), dtype=torch.float32, device="cuda")
    cnt = torch.empty(K, dtype=torch.int64, device="cuda")
    tac.tac_update(ctx, dev(xs), dev(seg_off), dev(a.astype(np.int32)), dev(C_old), Cn, cnt)
    got = host(Cn)
    assert np.array_equal(host(cnt), cnt1)
    check_centroids(got, C1)
    want = _means_in_member_order(xs, a, K, wide_rows=set(range(len(lens32), K)))
    empty = cnt1 == 0
    want[empty] = C_old[empty]
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))


def test_dyadic_exact_ties_bitwise(ctx):
    """Dyadic 1-D values in coordinate 0 make every float operation exact, so
    equal distances are exact ties; both paths break them to the lowest index
    exactly as the oracle does."""
    rng = np.random.default_rng(13)
    toks = []
    for j in range(12):
        kc = [1, 2, 3, 5, 6, 8, 12, 20, 5, 7, 33, 2][j]
        n = int(rng.integers(kc, 4 * kc + 10))
        vals = rng.integers(-64, 65, n) / 8.0
        cvals = rng.choice(np.arange(-64, 65, 2) / 8.0, kc, replace=False)   # midpoints on the grid
        toks.append((vals, cvals))
    xs = np.zeros((sum(len(v) for v, _ in toks), 128), np.float32)
    C = np.zeros((sum(len(c) for _, c in toks), 128), np.float32)
    xs[:, 0] = np.concatenate([v for v, _ in toks])
    C[:, 0] = np.concatenate([c for _, c in toks])
    seg_off = np.concatenate([[0], np.cumsum([len(v) for v, _ in toks])]).astype(np.int64)
    cent_off = np.concatenate([[0], np.cumsum([len(c) for _, c in toks])]).astype(np.int64)
    ref = oracle.assign(xs, seg_off, C, cent_off, decide="fp64")
    for prec in (0, 1, 2):
        a, d, J = run_assign(ctx, xs, seg_off, C, cent_off, prec)
        assert np.array_equal(a, ref["a"])
        assert np.array_equal(d.astype(np.float64), ref["D"])
        assert J == ref["J"]
    Cn = torch.empty((C.shape[0], 128), dtype=torch.float32, device="cuda")
    cnt = torch.empty(C.shape[0], dtype=torch.int64, device="cuda")
    tac.tac_update(ctx, dev(xs), dev(seg_off), dev(ref["a"].astype(np.int32)), dev(C), Cn, cnt)
    C1, cnt1 = oracle.update(xs, ref["a"], C)
    assert np.array_equal(host(cnt), cnt1)
    check_centroids(host(Cn), C1)


@pytest.mark.parametrize("n", [1, 700, 4096, 4097, 5000])
def test_serving_path_groups_unsorted_rows(ctx, n):
    """tac_assign with token ids (rows in any order) equals the sorted path;
    ids outside [0, T) and tokens without centroids give -1.  Batches of at
    most 4,096 rows are grouped in one work group, larger ones by the radix
    sort: both, and the boundary, give the oracle's grouping."""
    c = Case("small")
    rng = np.random.default_rng(14)
    idx = rng.permutation(c.x.shape[0])[:n]
    x, t = c.x[idx].copy(), c.tok[idx].copy()
    bad = min(7, n - 1)
    t[:bad] = c.T + 3                                  # invalid ids
    a = torch.empty(x.shape[0], dtype=torch.int32, device="cuda")
    d = torch.empty(x.shape[0], dtype=torch.float32, device="cuda")
    for prec in (0, 1, 2):
        tac.tac_assign(ctx, dev(x), dev(c.C0), dev(c.cent_off), a, tok=dev(t), precision=prec, dist=d)
        ga = host(a)
        assert np.all(ga[:bad] == -1)
        assert tac.tac_assign_stats(ctx)["unassigned"] >= bad
        keep = np.arange(bad, x.shape[0])
        perm, seg_off, _ = oracle.group_by_token(t[keep], c.T)
        ref = oracle.assign(x[keep][perm], seg_off, c.C0, c.cent_off, decide="fp32")
        exp = np.empty(keep.shape[0], np.int64)
        exp[perm] = ref["a"]
        assert np.array_equal(ga[keep], exp)


def test_graph_replay_equals_eager(ctx):
    from paper_2604_28142_amd import index as IX
    c = Case("small")
    d = c.device()
    ix = IX.Index(T=c.T, K=c.K, xs=d["xs"], perm=dev(c.perm.astype(np.int32)), seg_off=d["seg_off"],
                  cent_off=d["cent_off"], C=dev(c.C0))
    C0 = ix.C.clone()
    loop = IX.LloydLoop(ctx, ix, iters=3, precision=tac.TAC_BF16)
    loop.run()
    torch.cuda.synchronize()
    C_eager, a_eager, J_eager = ix.C.clone(), loop.assign.clone(), loop.inertia.clone()
    ix.C.copy_(C0)
    loop.capture()
    for rep in range(3):
        ix.C.copy_(C0)
        loop.replay()
        torch.cuda.synchronize()
        assert torch.equal(ix.C, C_eager), rep
        assert torch.equal(loop.assign, a_eager), rep
        assert torch.equal(loop.inertia, J_eager), rep
        # eager work between replays
        run_assign(ctx, c.xs, c.seg_off, c.C0, c.cent_off, tac.TAC_FP32)


def test_graph_survives_workspace_growth():
    """A Lloyd graph captured on a context stays valid after a later call on the
    same context (PQ training on a larger sample) grows the workspace: the
    replaced workspace is kept until the context is destroyed."""
    from paper_2604_28142_amd import index as IX
    ctx2 = tac.Context(0)
    try:
        c = Case("small")
        d = c.device()
        ix = IX.Index(T=c.T, K=c.K, xs=d["xs"], perm=dev(c.perm.astype(np.int32)), seg_off=d["seg_off"],
                      cent_off=d["cent_off"], C=dev(c.C0))
        C0 = ix.C.clone()
        loop = IX.LloydLoop(ctx2, ix, iters=3, precision=tac.TAC_BF16)
        loop.run()
        torch.cuda.synchronize()
        C_eager, a_eager = ix.C.clone(), loop.assign.clone()
        ix.C.copy_(C0)
        loop.capture()
        rng = np.random.default_rng(70)
        R = dev((0.1 * rng.standard_normal((300_000, 128))).astype(np.float32))
        init = R[:256].reshape(256, 32, 4).transpose(0, 1).contiguous()
        cb = torch.empty((32, 256, 4), dtype=torch.float32, device="cuda")
        tac.pq_train(ctx2, R, init, cb, iters=1)         # needs far more workspace than the graph's calls
        torch.cuda.synchronize()
        for rep in range(2):
            ix.C.copy_(C0)
            loop.replay()
            torch.cuda.synchronize()
            assert torch.equal(ix.C, C_eager), rep
            assert torch.equal(loop.assign, a_eager), rep
    finally:
        ctx2.close()


@pytest.mark.parametrize("tuning", [
    dict(direct_max_kappa=0, heavy_kappa=1, groups_per_cu=1, tile_blocks=0, waves_per_simd=0),
    dict(direct_max_kappa=16, heavy_kappa=64, groups_per_cu=0, tile_blocks=0, waves_per_simd=1),
    dict(direct_max_kappa=4, heavy_kappa=1024, groups_per_cu=0, tile_blocks=3, waves_per_simd=1),
    dict(direct_max_kappa=2, heavy_kappa=128, groups_per_cu=0, tile_blocks=4, waves_per_simd=0),
    dict(direct_max_kappa=4, heavy_kappa=256, groups_per_cu=1, tile_blocks=3, waves_per_simd=2)])
def test_tuning_keeps_results(ctx, tuning):
    """Launch tuning moves tokens between the direct and screened routes,
    reorders the work queue and changes the 16-bit screens' kernel (one or two
    work-groups per CU; 192-, 256- or 320-row items); the assignments stay
    those of the oracle."""
    rng = np.random.default_rng(15)
    kappas = [1, 3, 4, 5, 16, 17, 70]
    sizes = [40, 3 * 5 + 7, 200, 513, 90, 1030, 700]
    xs = np.concatenate([clustered(rng, n, 6) for n in sizes])
    seg_off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    cent_off = np.concatenate([[0], np.cumsum(kappas)]).astype(np.int64)
    C = np.concatenate([xs[seg_off[j] + rng.choice(sizes[j], kappas[j], replace=False)] for j in range(len(sizes))])
    before = ctx.get_tuning()
    try:
        assert ctx.set_tuning(**tuning) == tuning
        for prec in (0, 1, 2):
            a, d, J = run_assign(ctx, xs, seg_off, C, cent_off, prec)
            check_assign(xs, seg_off, C, cent_off, a, d)
    finally:
        ctx.set_tuning(**before)
    with pytest.raises(tac.TacError):
        ctx.set_tuning(direct_max_kappa=17)
    with pytest.raises(tac.TacError):
        ctx.set_tuning(tile_blocks=6)
    with pytest.raises(tac.TacError):
        ctx.set_tuning(waves_per_simd=3)
    with pytest.raises(tac.TacError):
        ctx.set_tuning(waves_per_simd=2, tile_blocks=5)
    assert ctx.get_tuning() == before


@pytest.mark.parametrize("wps,tile_blocks", [(1, 3), (1, 4), (1, 5)])
def test_tile_shapes_on_hot_tokens(ctx, wps, tile_blocks):
    """The one-work-group-per-CU tiles on tokens of 9,000 rows and 2,500 /
    4,097 centroids (several epochs and stages, ragged last tiles) and the
    split route (6,000 rows): every tile returns the oracle's FP32-decision
    assignments and the same distances as the default kernel (two work-groups
    per CU, 192-row items), bit for bit."""
    rng = np.random.default_rng(18)
    sizes, kappas = [9000, 9000, 6000, 700], [2500, 4097, 2500, 40]
    xs = np.concatenate([clustered(rng, n, 300, spread=0.3) for n in sizes])
    seg_off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    cent_off = np.concatenate([[0], np.cumsum(kappas)]).astype(np.int64)
    C = np.concatenate([xs[seg_off[j] + rng.choice(sizes[j], kappas[j], replace=False)] for j in range(len(sizes))])
    rows = np.sort(rng.choice(xs.shape[0], 3000, replace=False))
    before = ctx.get_tuning()
    try:
        for prec in (1, 2):
            ctx.set_tuning(tile_blocks=0, waves_per_simd=0)
            a0, d0, J0 = run_assign(ctx, xs, seg_off, C, cent_off, prec)
            ctx.set_tuning(tile_blocks=tile_blocks, waves_per_simd=wps)
            a, d, J = run_assign(ctx, xs, seg_off, C, cent_off, prec)
            assert np.array_equal(a, a0) and np.array_equal(d.view(np.uint32), d0.view(np.uint32)) and J == J0
            check_assign(xs, seg_off, C, cent_off, a[rows], d[rows], rows=rows)
    finally:
        ctx.set_tuning(**before)


def test_autotune_cache_roundtrip(ctx, tmp_path):
    from paper_2604_28142_amd import autotune
    c = Case("small")
    d = c.device()
    C = dev(c.C0)
    path = str(tmp_path / "tune.json")
    space = {"direct_max_kappa": [0, 4], "heavy_kappa": [256, 1024], "groups_per_cu": [0]}
    before = ctx.get_tuning()
    try:
        r1 = autotune.tune_assign(ctx, d["xs"], C, d["cent_off"], d["seg_off"], precision=tac.TAC_BF16, reps=1,
                                  cache_path=path, space=space)
        assert not r1["cached"] and len(r1["trials"]) >= 3
        assert ctx.get_tuning() == r1["tuning"]
        r2 = autotune.tune_assign(ctx, d["xs"], C, d["cent_off"], d["seg_off"], precision=tac.TAC_BF16,
                                  cache_path=path, space=space)
        assert r2["cached"] and r2["tuning"] == r1["tuning"]
        a, dd, _ = run_assign(ctx, c.xs, c.seg_off, c.C0, c.cent_off, tac.TAC_BF16)
        check_assign(c.xs, c.seg_off, c.C0, c.cent_off, a, dd, fp64=False)
    finally:
        ctx.set_tuning(**before)


@pytest.mark.parametrize("ksub", [16, 48, 20, 1, 256])
@pytest.mark.parametrize("normalize", [True, False])
def test_pq_encode_shapes_and_invalid_rows(ctx, ksub, normalize):
    """Both encode kernels (matrix-core screen for ksub % 16 == 0, scalar
    otherwise) on ragged row counts, with rows whose assignment is out of range."""
    rng = np.random.default_rng(100 + ksub)
    n, K = 1000 + ksub, 37
    x = clustered(rng, n, 9)
    C = x[rng.choice(n, K, replace=False)].copy()
    a = rng.integers(0, K, n).astype(np.int32)
    a[:5] = -1
    a[5:9] = K + 2
    cb = (0.25 * rng.standard_normal((32, ksub, 4))).astype(np.float32)
    codes = torch.empty((n, 32), dtype=torch.uint8, device="cuda")
    rho = torch.empty(n, dtype=torch.float32, device="cuda")
    tac.pq_encode(ctx, dev(x), dev(a), dev(C), dev(cb), codes, normalize=normalize, rnorm=rho)
    ok = (a >= 0) & (a < K)
    u32, rho32 = oracle.residuals(x[ok], C[a[ok]], normalize=normalize, mode="fp32")
    exp = oracle.pq_encode(u32, cb, decide="fp32")
    got = host(codes)
    assert np.array_equal(got[ok], exp)
    assert np.all(got[~ok] == 0) and np.all(host(rho)[~ok] == 0)
    assert np.array_equal(host(rho)[ok], rho32)


@pytest.mark.parametrize("n", [700, 32_768, 32_769])
def test_pq_encode_work_splits(ctx, n):
    """The encode's work split follows the input size (8 work-groups of 4
    subspaces per 512-row block up to 64 blocks, 2 of 16 beyond, on this
    device's 256 CUs); both splits, at their boundary, give the oracle's codes
    and norms."""
    rng = np.random.default_rng(120)
    K = 50
    x = clustered(rng, n, 9)
    C = x[rng.choice(n, K, replace=False)].copy()
    a = rng.integers(0, K, n).astype(np.int32)
    cb = (0.25 * rng.standard_normal((32, 256, 4))).astype(np.float32)
    codes = torch.empty((n, 32), dtype=torch.uint8, device="cuda")
    rho = torch.empty(n, dtype=torch.float32, device="cuda")
    tac.pq_encode(ctx, dev(x), dev(a), dev(C), dev(cb), codes, normalize=True, rnorm=rho)
    u32, rho32 = oracle.residuals(x, C[a], normalize=True, mode="fp32")
    assert np.array_equal(host(codes), oracle.pq_encode(u32, cb, decide="fp32"))
    assert np.array_equal(host(rho), rho32)


def test_pq_encode_ties_and_fallback(ctx):
    """Duplicate codes tie exactly (the lowest code wins); a codebook of nearly
    equal codes defeats the screen's certificate and is scanned exhaustively."""
    rng = np.random.default_rng(21)
    n, K, ksub = 700, 5, 64
    x = clustered(rng, n, 5)
    C = x[:K].copy()
    a = rng.integers(0, K, n).astype(np.int32)
    cb = (0.3 * rng.standard_normal((32, ksub, 4))).astype(np.float32)
    base = (0.3 * rng.standard_normal((4,))).astype(np.float32)
    cb[7] = base + (1e-7 * rng.standard_normal((ksub, 4))).astype(np.float32)   # near-ties in subspace 7
    cb[:, 40] = cb[:, 3]                                   # exact duplicates: code 3 must win over 40
    codes = torch.empty((n, 32), dtype=torch.uint8, device="cuda")
    tac.pq_encode(ctx, dev(x), dev(a), dev(C), dev(cb), codes)
    u32, _ = oracle.residuals(x, C[a], mode="fp32")
    exp = oracle.pq_encode(u32, cb, decide="fp32")
    got = host(codes)
    assert np.array_equal(got, exp)
    assert not np.any(got == 40)


@pytest.mark.parametrize("n", [700, 40_000])
def test_pq_encode_beyond_fp16_range(ctx, n):
    """Operands the split 16-bit screen cannot hold: a codebook coordinate
    beyond the FP16 range (every row of those subspaces is scanned
    exhaustively) and, without normalisation, residuals too large for FP16
    (the whole wave falls back); the codes are still the oracle's."""
    rng = np.random.default_rng(130)
    K = 7
    x = clustered(rng, n, 5)
    C = x[rng.choice(n, K, replace=False)].copy()
    a = rng.integers(0, K, n).astype(np.int32)
    cb = (0.25 * rng.standard_normal((32, 256, 4))).astype(np.float32)
    cb[9, 17] = [1.0e5, 0.0, 0.0, 0.0]   # never the nearest code, but outside FP16
    codes = torch.empty((n, 32), dtype=torch.uint8, device="cuda")
    tac.pq_encode(ctx, dev(x), dev(a), dev(C), dev(cb), codes, normalize=True)
    u32, _ = oracle.residuals(x, C[a], normalize=True, mode="fp32")
    assert np.array_equal(host(codes), oracle.pq_encode(u32, cb, decide="fp32"))
    xb = (x * np.float32(1.0e6)).astype(np.float32)
    Cb = (C * np.float32(1.0e6)).astype(np.float32)
    cb2 = (1.0e6 * cb).astype(np.float32)
    tac.pq_encode(ctx, dev(xb), dev(a), dev(Cb), dev(cb2), codes, normalize=False)
    u32b, _ = oracle.residuals(xb, Cb[a], normalize=False, mode="fp32")
    assert np.array_equal(host(codes), oracle.pq_encode(u32b, cb2, decide="fp32"))
