"""Pins for the oracle's residual normalisation and product quantisation."""
import numpy as np

import datagen
import oracle


def _rows(n=3000, seed=0):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, 128)).astype(np.float32)
    c = (x + 0.2 * rng.standard_normal((n, 128))).astype(np.float32)
    c[:5] = x[:5]                        # zero residuals
    return x, c


def test_residual_norm_and_reconstruction():
    x, c = _rows()
    u, rho = oracle.residuals(x, c)
    nrm = np.linalg.norm(u, axis=1)
    assert np.all(rho[:5] == 0) and np.all(nrm[:5] == 0)
    assert np.allclose(nrm[5:], 1.0, atol=1e-14)
    assert np.allclose(c.astype(np.float64) + rho[:, None] * u, x, rtol=0, atol=1e-12)
    u32, rho32 = oracle.residuals(x, c, mode="fp32")
    assert u32.dtype == np.float32 and rho32.dtype == np.float32
    assert np.allclose(rho32, rho, rtol=2e-6)
    assert np.allclose(u32, u, atol=2e-6)


def test_encode_equals_brute_force():
    rng = np.random.default_rng(1)
    u = rng.standard_normal((64, 128)).astype(np.float32)
    cb = rng.standard_normal((32, 256, 4)).astype(np.float32)
    codes = oracle.pq_encode(u, cb)
    for i in range(0, 64, 7):
        for m in range(0, 32, 5):
            d = [sum((float(u[i, 4 * m + t]) - float(cb[m, b, t])) ** 2 for t in range(4)) for b in range(256)]
            assert codes[i, m] == int(np.argmin(d))
    c32 = oracle.pq_encode(u, cb, decide="fp32")
    codes, ti, tD = oracle.pq_encode(u, cb, topk=2)
    # fp32 decisions differ from fp64 ones only on sub-1e-5 gaps
    diff = c32 != codes
    assert np.all(tD[diff][:, 1] - tD[diff][:, 0] < 1e-5)


def test_training_on_few_rows_is_lossless():
    rng = np.random.default_rng(2)
    R = rng.standard_normal((200, 128)).astype(np.float32)
    R /= np.linalg.norm(R, axis=1, keepdims=True)
    init = np.arange(200).tolist() + [0] * 56      # codebook rows = the training rows
    cb = oracle.pq_train(R, 32, 256, 3, init)
    codes = oracle.pq_encode(R, cb)
    assert np.array_equal(oracle.pq_decode(codes, cb), R)


def test_scalar_quantiser_special_case():
    """With one coordinate per subspace PQ is nearest-value scalar quantisation."""
    rng = np.random.default_rng(3)
    u = rng.standard_normal((500, 8)).astype(np.float32)
    cb = np.sort(rng.standard_normal((8, 16, 1)).astype(np.float32), axis=1)
    codes = oracle.pq_encode(u, cb)
    for m in range(8):
        vals = cb[m, :, 0].astype(np.float64)
        mids = (vals[1:] + vals[:-1]) / 2
        expect = np.searchsorted(mids, u[:, m].astype(np.float64), side="left")
        assert np.array_equal(codes[:, m], expect)


def test_training_reduces_quantisation_error():
    x, tok = datagen.make("tiny")
    R = x[:2000] - x[:2000].mean(axis=0)
    R = (R / np.linalg.norm(R, axis=1, keepdims=True)).astype(np.float32)
    init = datagen.pq_init_rows(2000, 256, 0)
    err = []
    for it in (0, 1, 4):
        cb = oracle.pq_train(R, 32, 256, it, init)
        rec = oracle.pq_decode(oracle.pq_encode(R, cb), cb)
        err.append(float(((rec - R) ** 2).sum()))
    assert err[0] >= err[1] >= err[2]
