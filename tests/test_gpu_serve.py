"""GPU tests of the encode service: results equal the oracle's, are bitwise the
same alone and in a mixed batch, and unseen tokens fail only their document."""
import numpy as np
import pytest
import torch

import datagen
import oracle

from gpu_common import Case, dev

pytestmark = pytest.mark.gpu

tac = pytest.importorskip("paper_2604_28142_amd")
from paper_2604_28142_amd.serve import EncodeService, GpuExecutor, ResidentIndex, run_load  # noqa: E402


@pytest.fixture(scope="module")
def served():
    c = Case("small")
    a = oracle.assign(c.xs, c.seg_off, c.C0, c.cent_off, decide="fp32")["a"]
    u32, _ = oracle.residuals(c.xs, c.C0[a], mode="fp32")
    sample = datagen.pq_sample(u32.shape[0], 20_000, 0)
    cb = oracle.pq_train(u32[sample], 32, 256, 3, datagen.pq_init_rows(sample.shape[0], 256, 0), decide="fp32")
    index = ResidentIndex(T=c.T, K=c.K, C=dev(c.C0), cent_off=dev(c.cent_off), codebooks=dev(cb))
    lens, x, tok = datagen.serving_docs("small", 400, seed=3)
    edges = np.concatenate([[0], np.cumsum(lens)])
    docs = [(x[edges[i]:edges[i + 1]], tok[edges[i]:edges[i + 1]]) for i in range(len(lens))]
    ex = GpuExecutor(index, n_slots=3, max_rows=64 * 180)
    svc = EncodeService(ex, max_docs=64)
    yield c, cb, docs, svc
    svc.close()
    ex.close()


def _expected(c, cb, x, t):
    perm, seg_off, _ = oracle.group_by_token(t, c.T)
    r = oracle.assign(x[perm], seg_off, c.C0, c.cent_off, decide="fp32")
    a = np.empty_like(r["a"])
    a[perm] = r["a"]
    u, rho = oracle.residuals(x, c.C0[a], mode="fp32")
    return a, oracle.pq_encode(u, cb, decide="fp32"), rho


def test_service_matches_oracle_and_isolates_unseen(served):
    c, cb, docs, svc = served
    present = c.kappa > 0
    res, wall = run_load(svc, docs, None)
    n_fail = 0
    for (x, t), r in zip(docs, res):
        if not np.all(present[t]):
            assert isinstance(r, tac.TacError)
            n_fail += 1
            continue
        a, codes, rho = _expected(c, cb, x, t)
        assert np.array_equal(r.assign, a)
        assert np.array_equal(r.codes, codes)
        assert np.array_equal(r.rnorm, rho)
    assert svc.stats.docs >= len(docs)
    # a document with an id outside [0, T) fails on its own
    x, t = docs[0]
    bad = t.copy()
    bad[0] = c.T
    with pytest.raises(tac.TacError):
        svc.submit(x, bad).result()
    assert not isinstance(svc.submit(x, t).result(), Exception)


def test_alone_equals_in_the_mix(served):
    c, cb, docs, svc = served
    present = c.kappa > 0
    ok = [i for i, (x, t) in enumerate(docs) if np.all(present[t])][:200]
    mixed, _ = run_load(svc, [docs[i] for i in ok], None)
    for k, i in enumerate(ok):
        alone = svc.submit(*docs[i]).result()
        assert np.array_equal(alone.assign, mixed[k].assign)
        assert np.array_equal(alone.codes, mixed[k].codes)
        assert np.array_equal(alone.rnorm, mixed[k].rnorm)


def test_poisson_load_reports_latency(served):
    c, cb, docs, svc = served
    present = c.kappa > 0
    ok = [d for d in docs if np.all(present[d[1]])][:300]
    before = len(svc.stats.latencies)
    res, wall = run_load(svc, ok, datagen.poisson_arrivals(2000.0, len(ok), seed=1))
    lat = np.asarray(svc.stats.latencies[before:])
    assert lat.shape[0] == len(ok)
    assert np.all(lat > 0) and np.percentile(lat, 99) < wall


def test_graph_replay_equals_eager_and_budget_binds(served):
    """The replayed bucket graphs give bitwise the results of eager launches
    (several replays of each bucket, eager work between them), also under a
    device-memory budget that lets only about one large batch fly at a time."""
    c, cb, docs, svc = served
    present = c.kappa > 0
    ok = [d for d in docs if np.all(present[d[1]])][:240]
    index = svc.ex.index
    eager = GpuExecutor(index, n_slots=2, max_rows=64 * 180, graphs=False)
    s_eager = EncodeService(eager, max_docs=64)
    ref, _ = run_load(s_eager, ok, None)
    s_eager.close()
    eager.close()
    ex = GpuExecutor(index, n_slots=3, max_rows=64 * 180, graphs=True, buckets=[1024, 4096, 64 * 180])
    assert ex.batch_bytes(100) == ex.batch_bytes(1024) < ex.batch_bytes(1025)
    cap = ex.batch_bytes(64 * 180) + ex.batch_bytes(1024)
    s_graph = EncodeService(ex, max_docs=64, ledger_bytes=cap)
    try:
        for rep in range(2):
            res, _ = run_load(s_graph, ok, None)            # large batches (several buckets)
            one = [s_graph.submit(*ok[i]).result() for i in range(0, 40, 3)]  # small batches
            torch.cuda.synchronize()
            for r0, r in zip(ref, res):
                assert np.array_equal(r0.assign, r.assign) and np.array_equal(r0.codes, r.codes)
                assert np.array_equal(r0.rnorm.view(np.uint32), r.rnorm.view(np.uint32))
            for k, i in enumerate(range(0, 40, 3)):
                assert np.array_equal(ref[i].assign, one[k].assign) and np.array_equal(ref[i].codes, one[k].codes)
        assert s_graph.max_ledger_used <= cap
    finally:
        s_graph.close()
        ex.close()


def test_service_large_kappa_routes_match_oracle():
    """The service on an index with tokens of 2,048 to 9,000 centroids, as the
    10M- and 50M-row indexes have: batches that hold at most 8,192 rows of such
    a token take the split route, a batch with more of one takes the persistent
    route, and every document's assignments, codes and norms equal the oracle's."""
    rng = np.random.default_rng(77)
    kappa = np.array([9000, 4096, 2500, 2048, 700, 300, 64, 16, 4, 1], dtype=np.int64)
    T = kappa.shape[0]
    cent_off = np.concatenate([[0], np.cumsum(kappa)]).astype(np.int64)
    K = int(cent_off[-1])
    base = rng.standard_normal((T, 128)).astype(np.float32)
    C = np.concatenate([base[j] + 0.35 * rng.standard_normal((kappa[j], 128)).astype(np.float32) for j in range(T)])
    C /= np.linalg.norm(C, axis=1, keepdims=True)
    C = C.astype(np.float32)
    cb = (0.25 * rng.standard_normal((32, 256, 4))).astype(np.float32)
    index = ResidentIndex(T=T, K=K, C=dev(C), cent_off=dev(cent_off), codebooks=dev(cb))

    def doc(n, weights):
        t = rng.choice(T, n, p=weights).astype(np.int32)
        k = cent_off[t] + (rng.random(n) * kappa[t]).astype(np.int64)
        x = C[k] + 0.2 * rng.standard_normal((n, 128)).astype(np.float32)
        x /= np.linalg.norm(x, axis=1, keepdims=True)
        return x.astype(np.float32), t

    w_mix = np.array([0.3, 0.2, 0.15, 0.1, 0.1, 0.05, 0.04, 0.03, 0.02, 0.01])
    w_one = np.zeros(T)
    w_one[0] = 1.0
    docs = [doc(int(rng.integers(40, 200)), w_mix) for _ in range(48)]
    heavy = [doc(200, w_one) for _ in range(48)]     # 9,600 rows of the 9,000-centroid token in one batch
    ex = GpuExecutor(index, n_slots=2, max_rows=64 * 200)
    svc = EncodeService(ex, max_docs=64)
    try:
        for group in (docs, heavy):
            res, _ = run_load(svc, group, None)
            for (x, t), r in zip(group, res):
                perm, seg_off, _ = oracle.group_by_token(t, T)
                o = oracle.assign(x[perm], seg_off, C, cent_off, decide="fp32")
                a = np.empty_like(o["a"])
                a[perm] = o["a"]
                u, rho = oracle.residuals(x, C[a], mode="fp32")
                assert np.array_equal(r.assign, a)
                assert np.array_equal(r.codes, oracle.pq_encode(u, cb, decide="fp32"))
                assert np.array_equal(r.rnorm, rho)
    finally:
        svc.close()
        ex.close()
