"""CPU tests of the encode service's scheduler (admission, batching, ledger,
ordering, failure isolation) with a stand-in executor."""
import threading
import time

import numpy as np
import pytest

from paper_2604_28142_amd.serve import ROW_BYTES, EncodeService, run_load


class FakeExecutor:
    """Deterministic stand-in: assignment = token id (-1 for id 99), codes and
    norm derived from the row; optional delay and failure injection."""

    def __init__(self, n_slots=2, max_rows=1000, delay=0.002, fail_token=None):
        self.n_slots, self.max_rows, self.delay, self.fail_token = n_slots, max_rows, delay, fail_token
        self.out = {}
        self.lock = threading.Lock()
        self.inflight_rows = 0
        self.max_inflight_rows = 0
        self.batches = []

    def launch(self, slot, xs, toks):
        x = np.concatenate(xs)
        t = np.concatenate(toks)
        if self.fail_token is not None and np.any(t == self.fail_token):
            raise RuntimeError("injected kernel failure")
        with self.lock:
            self.inflight_rows += x.shape[0]
            self.max_inflight_rows = max(self.max_inflight_rows, self.inflight_rows)
            self.batches.append(len(xs))
        a = np.where(t == 99, -1, t).astype(np.int32)
        codes = (np.abs(x[:, :32]) * 1000).astype(np.uint8)
        rho = np.linalg.norm(x, axis=1).astype(np.float32)
        self.out[slot] = (a, codes, rho, time.perf_counter() + self.delay)
        return x.shape[0]

    def wait(self, slot, n):
        a, c, r, ready = self.out[slot]
        d = ready - time.perf_counter()
        if d > 0:
            time.sleep(d)
        with self.lock:
            self.inflight_rows -= n
        return a[:n], c[:n], r[:n]


def docs(n, seed=0, lo=3, hi=40):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        k = int(rng.integers(lo, hi + 1))
        out.append((rng.standard_normal((k, 128)).astype(np.float32), rng.integers(0, 50, k).astype(np.int32)))
    return out


def test_results_split_per_document_in_order():
    ex = FakeExecutor()
    svc = EncodeService(ex, max_docs=16)
    D = docs(200)
    res, _ = run_load(svc, D, None)
    svc.close()
    for (x, t), r in zip(D, res):
        assert np.array_equal(r.assign, t)
        assert np.array_equal(r.codes, (np.abs(x[:, :32]) * 1000).astype(np.uint8))
    assert svc.stats.docs == 200 and svc.stats.failed == 0
    assert max(ex.batches) <= 16
    # continuous batching: arrivals during earlier batches were grouped
    assert svc.stats.batches < 200


def test_ledger_bounds_memory_in_flight():
    ex = FakeExecutor(n_slots=3, max_rows=200, delay=0.003)
    cap = 250 * ROW_BYTES
    svc = EncodeService(ex, max_docs=64, ledger_bytes=cap)
    res, _ = run_load(svc, docs(150), None)
    svc.close()
    assert all(not isinstance(r, Exception) for r in res)
    assert ex.max_inflight_rows * ROW_BYTES <= cap


class BudgetedExecutor(FakeExecutor):
    """A stand-in that charges each batch its bytes like the GPU executor: a
    fixed workspace plus the rows of its bucket (powers of two from 64)."""

    FIXED, PER_ROW = 50_000, 600

    def __init__(self, **kw):
        super().__init__(**kw)
        self.inflight_bytes = 0
        self.max_inflight_bytes = 0
        self.bytes_of = {}

    def batch_bytes(self, rows):
        b = 64
        while b < rows:
            b *= 2
        return self.FIXED + min(b, self.max_rows) * self.PER_ROW

    def launch(self, slot, xs, toks):
        n = super().launch(slot, xs, toks)
        with self.lock:
            self.bytes_of[slot] = self.batch_bytes(n)
            self.inflight_bytes += self.bytes_of[slot]
            self.max_inflight_bytes = max(self.max_inflight_bytes, self.inflight_bytes)
        return n

    def wait(self, slot, n):
        out = super().wait(slot, n)
        with self.lock:
            self.inflight_bytes -= self.bytes_of[slot]
        return out


def test_memory_budget_binds_and_results_stay():
    """With a device-memory budget of one full batch and a bit, the three
    slots never hold more than the budget together: requests wait for memory
    (fewer batches in flight than slots) and every result is still the one a
    document gets alone."""
    D = docs(300, seed=7)
    free = BudgetedExecutor(n_slots=3, max_rows=400, delay=0.004)
    svc = EncodeService(free, max_docs=64)
    assert svc.ledger_cap == 3 * free.batch_bytes(400)
    ref, _ = run_load(svc, D, None)
    svc.close()
    ex = BudgetedExecutor(n_slots=3, max_rows=400, delay=0.004)
    cap = ex.batch_bytes(400) + ex.batch_bytes(100)
    svc = EncodeService(ex, max_docs=64, ledger_bytes=cap)
    res, _ = run_load(svc, D, None)
    svc.close()
    assert ex.max_inflight_bytes <= cap and svc.max_ledger_used <= cap
    assert ex.max_inflight_bytes > ex.batch_bytes(400)             # the budget was used, and it bound:
    assert free.max_inflight_bytes > cap                           # unbudgeted, more was in flight
    for r0, r in zip(ref, res):
        assert np.array_equal(r0.assign, r.assign) and np.array_equal(r0.codes, r.codes)
    tight = EncodeService(BudgetedExecutor(max_rows=400), ledger_bytes=60_000)
    try:
        with pytest.raises(ValueError):                            # a document alone beyond the budget
            tight.submit(np.zeros((200, 128), np.float32), np.zeros(200, np.int32))
    finally:
        tight.close()


def test_failed_batch_is_isolated_and_loop_continues():
    ex = FakeExecutor(fail_token=7)
    svc = EncodeService(ex, max_docs=1)          # one document per batch
    D = docs(30)
    D[5] = (D[5][0], np.full_like(D[5][1], 7))   # only this document carries the poisoned token
    for i, (x, t) in enumerate(D):
        if i != 5:
            D[i] = (x, np.where(t == 7, 8, t).astype(np.int32))
    res, _ = run_load(svc, D, None)
    svc.close()
    assert isinstance(res[5], RuntimeError)
    assert all(not isinstance(r, Exception) for i, r in enumerate(res) if i != 5)


def test_unseen_token_fails_only_its_document():
    from paper_2604_28142_amd._lib import TacError
    ex = FakeExecutor()
    svc = EncodeService(ex, max_docs=64)
    D = docs(40)
    D[3] = (D[3][0], np.where(np.arange(D[3][1].shape[0]) == 0, 99, D[3][1]).astype(np.int32))
    for i, (x, t) in enumerate(D):
        if i != 3:
            D[i] = (x, np.where(t == 99, 1, t).astype(np.int32))
    res, _ = run_load(svc, D, None)
    svc.close()
    assert isinstance(res[3], TacError)
    assert sum(isinstance(r, Exception) for r in res) == 1


def test_latency_accounts_for_slow_batches():
    ex = FakeExecutor(n_slots=1, delay=0.05)
    svc = EncodeService(ex, max_docs=4)
    res, wall = run_load(svc, docs(8), None)
    svc.close()
    assert len(svc.stats.latencies) == 8
    assert max(svc.stats.latencies) >= 0.05 * 2 - 1e-3     # at least two batches queued ahead
    assert svc.stats.percentile(99) <= wall + 1e-3


def test_rejects_malformed_documents():
    svc = EncodeService(FakeExecutor(), max_docs=4)
    with pytest.raises(ValueError):
        svc.submit(np.zeros((3, 64), np.float32), np.zeros(3, np.int32))
    with pytest.raises(ValueError):
        svc.submit(np.zeros((0, 128), np.float32), np.zeros(0, np.int32))
    svc.close()


def test_gc_tuning_lasts_while_any_service_runs():
    import gc
    before = gc.get_threshold()
    a = EncodeService(FakeExecutor())
    b = EncodeService(FakeExecutor())
    try:
        assert gc.get_threshold()[0] >= 50_000 and gc.get_freeze_count() > 0
        res, _ = run_load(a, docs(20, seed=5), None)
        assert all(not isinstance(r, Exception) for r in res)
    finally:
        a.close()
    assert gc.get_threshold()[0] >= 50_000          # b still serves
    b.close()
    assert gc.get_threshold() == before and gc.get_freeze_count() == 0
    c = EncodeService(FakeExecutor(), tune_gc=False)
    assert gc.get_threshold() == before
    c.close()
