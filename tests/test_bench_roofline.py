"""The benchmark's per-token roofline (host arithmetic only): T_roof sums, over
the tokens, the larger of the matrix-core time of the screen flops and the HBM
time of the bytes, against the spec-sheet peaks and against the measured
ceilings; the fraction is T_roof over the measured kernel time."""
import numpy as np

import bench


def test_segment_roofline_hand_case():
    counts = np.array([1000, 50, 10, 0])
    kappa = np.array([100, 5, 2, 0])
    r = bench.segment_roofline(counts, kappa, 2.0, "bf16", 5000.0)
    d = 128
    # token 0: 2 d n kappa flops (screened); bytes 4 d n + 4 d kappa + 8 n
    f0, b0 = 2 * d * 1000 * 100, 4 * d * 1000 + 4 * d * 100 + 8 * 1000
    f1, b1 = 2 * d * 50 * 5, 4 * d * 50 + 4 * d * 5 + 8 * 50
    f2, b2 = 0.0, 4 * d * 10 + 4 * d * 2 + 8 * 10            # kappa <= 4: the direct route, no screen flops
    spec = sum(max(f / 2500e12, b / 8000e9) for f, b in ((f0, b0), (f1, b1), (f2, b2))) * 1e3
    meas = sum(max(f / 1950e12, b / 5000e9) for f, b in ((f0, b0), (f1, b1), (f2, b2))) * 1e3
    assert np.isclose(r["t_roof_ms"], spec, rtol=1e-12)
    assert np.isclose(r["frac"], spec / 2.0, rtol=1e-12)
    assert np.isclose(r["t_roof_measured_ceilings_ms"], meas, rtol=1e-12)
    assert np.isclose(r["frac_vs_measured_ceilings"], meas / 2.0, rtol=1e-12)


def test_segment_roofline_bounds():
    """A large-kappa token is bound by the matrix cores, a small one by HBM; the
    FP16 screen streams 2-byte centroid rows, the split BF16 screen 4-byte."""
    big = bench.segment_roofline(np.array([100_000]), np.array([20_000]), 1.0, "bf16", None)
    assert np.isclose(big["t_roof_ms"], 2 * 128 * 100_000 * 20_000 / 2500e12 * 1e3, rtol=1e-12)
    assert "frac_vs_measured_ceilings" not in big
    small_bf = bench.segment_roofline(np.array([100_000]), np.array([8]), 1.0, "bf16", None)["t_roof_ms"]
    small_f = bench.segment_roofline(np.array([100_000]), np.array([8]), 1.0, "f16", None)["t_roof_ms"]
    assert np.isclose(small_bf - small_f, 2 * 128 * 8 / 8000e9 * 1e3, rtol=1e-9)
