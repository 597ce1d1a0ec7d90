"""CPU checks of the C ABI: the library loads, exports every declared entry point,
and its host-side budget agrees with the oracle."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from oracle.budget import BudgetParams as OParams, Infeasible

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tac.h")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:tac_status|void|const char\*)\s+(\w+)\s*\(", src, flags=re.M)))


def test_library_exports_every_declared_symbol():
    tac = pytest.importorskip("paper_2604_28142_amd")
    lib = tac.load()
    names = declared()
    assert "tac_assign" in names and "pq_encode" in names and len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(tac._lib.EXPORTS) == names


def test_errors_without_device_are_reported_not_raised_from_c():
    tac = pytest.importorskip("paper_2604_28142_amd")
    with pytest.raises(tac.TacError):
        tac.tac_budget_from_stats(np.array([10]), np.array([0.5]), -1)


@pytest.mark.parametrize("seed", range(8))
@pytest.mark.parametrize("policy", [0, 1])
def test_host_budget_matches_oracle(seed, policy):
    tac = pytest.importorskip("paper_2604_28142_amd")
    rng = np.random.default_rng(seed)
    T = int(rng.integers(50, 3000))
    counts = np.floor(rng.pareto(1.0, T) * 200).astype(np.int64)
    counts[rng.random(T) < 0.05] = 0
    spread = rng.uniform(0.0, 0.6, T)
    spread[rng.random(T) < 0.02] = 0.0
    prm = dict(mu=int(rng.integers(2, 200)), eps=int(rng.integers(1, 8)), theta=float(rng.choice([0.0, 13.0, 39.0])))
    prm["tau"] = prm["mu"] + int(rng.integers(0, 300))
    for K in rng.integers(1, int(counts.sum()) + 1, 6):
        try:
            ref = oracle.budget(counts, spread, int(K), OParams(policy=policy, **prm))
        except Infeasible:
            with pytest.raises(tac.TacError) as e:
                tac.tac_budget_from_stats(counts, spread, int(K), tac.BudgetParams(theta_policy=policy, **prm))
            assert e.value.status == tac._lib.TAC_E_INFEASIBLE
            continue
        got, _ = tac.tac_budget_from_stats(counts, spread, int(K), tac.BudgetParams(theta_policy=policy, **prm))
        assert np.array_equal(got, ref)


def test_host_budget_golden():
    import json
    tac = pytest.importorskip("paper_2604_28142_amd")
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "budget_examples.json")))
    for c in g["cases"]:
        p = tac.BudgetParams(c.get("mu", 128), c.get("tau", 256), c.get("eps", 4), float(c.get("theta", 39)),
                             c["policy"])
        got, _ = tac.tac_budget_from_stats(c["counts"], c["spread"], c["K"], p)
        assert got.tolist() == c["kappa"]


def test_autotune_workload_key_tracks_structure():
    pytest.importorskip("paper_2604_28142_amd")
    from paper_2604_28142_amd import autotune
    seg = np.array([0, 10, 30, 31], np.int64)
    cen = np.array([0, 2, 7, 8], np.int64)
    k = autotune.workload_key(seg, cen, 1)
    assert k == autotune.workload_key(seg.copy(), cen.copy(), 1)
    assert k != autotune.workload_key(seg, cen, 0)
    assert k != autotune.workload_key(np.array([0, 11, 30, 31]), cen, 1)
    assert k != autotune.workload_key(seg, np.array([0, 3, 7, 8]), 1)
    # every knob of the default is searched: the tile knob sets the occupancy and tile shape together
    searched = {k for k in autotune.SPACE if k != "tile"} | {f for t in autotune.SPACE["tile"] for f in t}
    assert set(autotune.DEFAULT) == searched
    assert {"waves_per_simd": autotune.DEFAULT["waves_per_simd"],
            "tile_blocks": autotune.DEFAULT["tile_blocks"]} in autotune.SPACE["tile"]
    assert all(v in autotune.SPACE[n] for n, v in autotune.DEFAULT.items() if n in autotune.SPACE)
