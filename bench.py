"""Benchmark of the token-aware clustering build path on one MI355X.

One step = one pass of the whole hot path over the resident synthetic input:
group by token + budget, seeded initial centroids, 10 Lloyd iterations
(assign + update, replayed from one captured HIP graph), the final assignment,
PQ training on the normalised residuals of a seeded sample and the fused
residual + PQ encoding of every vector.

Metric (vectors assigned per second per Lloyd iteration) = N * iters / Lloyd
time, Lloyd time measured with HIP events around the graph replay inside each
step.  The headline is the 10M-row workload with the BF16 screen
(``--headline f16`` times the FP16 screen instead); the other precisions run
the same graph for comparison and must give identical final assignments.

After the headline the same run measures, unless switched off:
* global k-means on the same kernels (a row sample against all K centroids),
  beside the work ratio and the speed-up bounds of Sect. 2.1;
* the encode service against the resident index, at 0.3, 0.6 and 0.9 of its
  measured saturated rate;
* the 50M-row, 2,097,152-centroid workload (``c3`` block): one warm-up and one
  timed BF16 step, the FP16 and FP32 Lloyd legs, the per-token roofline, the
  final-assignment check, and the encode service against that index.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"bf16": 2500.0, "f16": 2500.0, "fp32": 157.3}   # dense MFMA TFLOP/s of an MI355X
PRODUCTS = {"bf16": 3, "f16": 1, "fp32": 1}              # matrix-core products per coordinate of x.c
HBM_PEAK = 8000.0                         # GB/s
# Matrix-core ceilings measured with a microbenchmark on an MI355X: the
# instruction each screen issues, at the kernel's occupancy (one wave per SIMD
# for the 16-bit screens, two for FP32), in TFLOP/s
MEASURED_MFMA = {"bf16": 1950.0, "f16": 1970.0, "fp32": 156.0}
STAGED_BYTES = {"bf16": 4, "f16": 2, "fp32": 4}          # bytes per centroid coordinate the screen streams

WORKLOAD_TEXT = {
    "c1": "10M token vectors x 128 fp32 (L2-normalised), Zipf(1.0) token ids over 30,522, 4 sub-centres per "
          "token (sigma 0.25), K=262,144 centroids, 10 Lloyd iterations, PQ M=32 x 256 trained on a 1M "
          "residual sample, all 10M encoded",
    "c3": "50M token vectors x 128 fp32, Zipf(1.0) over 30,522 ids, K=2,097,152 centroids, 10 Lloyd iterations, "
          "PQ M=32 x 256 on a 1M sample, all 50M encoded",
    "c0": "200k token vectors x 128 fp32, Zipf(1.1) over 2,000 ids, K=8,192, 10 Lloyd iterations",
}


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "assign_main_{prec}_{config}_traffic.md")
PMC_FILE = os.path.join(ROOT, "profiles", "assign_main_{prec}_{config}_mfma_busy.md")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2604_28142_amd", "csrc", f) for f in ("assign.hip", "tac_internal.h")]


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha1()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(config: str, prec: str):
    """HBM bytes per launch of the 16-bit assignment kernel from the committed counter
    summary, or None when there is none for this workload or it predates the kernel source."""
    try:
        text = open(TRAFFIC_FILE.format(prec=prec, config=config)).read()
    except OSError:
        return None
    vals = dict(ln.split(":", 1) for ln in text.splitlines() if ln.startswith(("traffic_bytes_per_launch:",
                                                                              "kernel_source_sha1:", "workload:")))
    if vals.get("kernel_source_sha1", "").strip() != kernel_source_hash():
        return None
    if vals.get("workload", "").strip() != config:
        return None
    return float(vals["traffic_bytes_per_launch"])


def measured_mfma_busy(config: str, prec: str):
    """Fraction of the matrix cores' cycles busy during the 16-bit assignment
    kernel, from the committed counter summary (SQ_VALU_MFMA_BUSY_CYCLES over
    SQ_BUSY_CYCLES times the SIMDs per counter), or None when there is none for
    this workload or it predates the kernel source."""
    try:
        text = open(PMC_FILE.format(prec=prec, config=config)).read()
    except OSError:
        return None
    vals = dict(ln.split(":", 1) for ln in text.splitlines() if ln.startswith(("mfma_busy_frac:",
                                                                              "kernel_source_sha1:", "workload:")))
    if vals.get("kernel_source_sha1", "").strip() != kernel_source_hash():
        return None
    if vals.get("workload", "").strip() != config:
        return None
    return float(vals["mfma_busy_frac"])


def host_info() -> dict:
    """Host cores visible to this process and the CPU model."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "logical_cpus": os.cpu_count(), "usable_cpus": usable}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(x, tok, w, sample_rows: int, one_core_rows: int = 0, seed: int = 0):
    """Time the oracle's float64 assignment of a uniform row sample (a row's
    assignment depends only on its token's centroids) on the host cores: with
    every BLAS thread, then (when one_core_rows > 0) a smaller sample on one.
    Returns (all-cores record, one-core record or None)."""
    import datagen
    import oracle
    from oracle.budget import BudgetParams
    from threadpoolctl import threadpool_info, threadpool_limits

    t0 = time.time()
    perm, seg_off, counts = oracle.group_by_token(tok, w.vocab)
    xs = x[perm]
    spread = oracle.spreads(xs, seg_off)
    kappa = oracle.budget(counts, spread, w.k, BudgetParams())
    cent_off = oracle.cent_offsets(kappa)
    picks = datagen.init_picks(counts, kappa, w.seed)
    C0 = oracle.init_centroids(xs, seg_off, cent_off, picks)
    log(f"cpu_baseline: oracle preparation {time.time() - t0:.1f}s")

    def timed(n, threads_label):
        rows = np.sort(np.random.default_rng([seed, 11]).choice(xs.shape[0], n, replace=False))
        t0 = time.perf_counter()
        oracle.assign_rows(xs, rows, seg_off, C0, cent_off, decide="fp64")
        dt = time.perf_counter() - t0
        threads = threads_label()
        return {"value": n / dt, "unit": "vectors/s", "cores": threads, "kind": "oracle",
                "sample": f"{n} uniformly sampled rows of the same workload assigned by the float64 oracle "
                          f"against their tokens' initial centroids ({dt:.1f}s on {threads} threads)",
                "host": host_info()}

    def blas_threads():
        return max([i["num_threads"] for i in threadpool_info()] or [1])

    full = timed(sample_rows, blas_threads)
    one = None
    if one_core_rows > 0:
        with threadpool_limits(limits=1):
            one = timed(one_core_rows, blas_threads)
    return full, one


def segment_roofline(counts, kappa, kernel_ms: float, prec: str, hbm_gbs: float | None):
    """Per-token roofline of one assignment launch: T_roof = sum over tokens of
    max(F_j / P, B_j / BW) with F_j = 2 d n_j kappa_j for the screened tokens
    (kappa_j > 4) and B_j = 4 d n_j (x) + b_c d kappa_j (the staged centroid
    copy) + 8 n_j (assignment and distance); the fraction is T_roof over the
    measured kernel time, against the spec-sheet peaks and against the measured
    ceilings (the kernel's own matrix instruction at its occupancy, and a
    device-to-device copy)."""
    d = 128
    n = counts.astype(np.float64)
    k = kappa.astype(np.float64)
    f = np.where(k > 4, 2.0 * d * n * k, 0.0)
    b = 4.0 * d * n + STAGED_BYTES[prec] * d * k + 8.0 * n
    t_spec = float(np.maximum(f / (PEAK[prec] * 1e12), b / (HBM_PEAK * 1e9)).sum()) * 1e3
    out = {"t_roof_ms": t_spec, "t_measured_ms": kernel_ms, "frac": t_spec / kernel_ms,
           "mfma_peak_tflops": PEAK[prec], "hbm_peak_gbs": HBM_PEAK}
    if hbm_gbs:
        t_meas = float(np.maximum(f / (MEASURED_MFMA[prec] * 1e12), b / (hbm_gbs * 1e9)).sum()) * 1e3
        out.update({"t_roof_measured_ceilings_ms": t_meas, "frac_vs_measured_ceilings": t_meas / kernel_ms,
                    "measured_mfma_tflops": MEASURED_MFMA[prec], "measured_copy_gbs": hbm_gbs})
    return out


def copy_bandwidth(torch, dev, nbytes: int = 1 << 31) -> float:
    """Device-to-device copy rate (read + write bytes per second, GB/s), best of three."""
    src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    best = float("inf")
    for _ in range(3):
        ev[0].record()
        dst.copy_(src)
        ev[1].record()
        ev[1].synchronize()
        best = min(best, ev[0].elapsed_time(ev[1]))
    del src, dst
    return 2.0 * nbytes / (best / 1e3) / 1e9


def speedup_bounds(counts, spread, kappa, K: int, tau: int = 256) -> dict:
    """Work ratio of one token-aware Lloyd iteration against global k-means
    (N K distances over sum_j n_j kappa_j) and the two lower bounds of Sect. 2.1's
    derivation: W / max w for the proportional allocation kappa_j = w_j / W * K,
    and K / max kappa_j for the allocation actually used."""
    n = counts.astype(np.float64)
    act = counts >= tau
    wj = np.sqrt(n[act]) * spread[act]
    return {"work_ratio": float(n.sum() * K / (n * kappa).sum()),
            "bound_sum_w_over_max_w": float(wj.sum() / wj.max()),
            "bound_K_over_max_kappa": float(K / kappa.max())}


def global_baseline(ctx, idx, w, tac_iter_ms: float, rows: int, seed: int = 0):
    """Plain (global) Lloyd on the same kernels: one segment holding a uniform
    sample of `rows` vectors and all K centroids of the build, one BF16
    assignment + update timed with HIP events (median of three, after one
    untimed); compared per vector with the token-aware iteration on the full
    input, beside the work ratio and the bounds of Sect. 2.1."""
    import torch
    import paper_2604_28142_amd as tac
    dev = idx.xs.device
    N = idx.xs.shape[0]
    sel = torch.from_numpy(np.sort(np.random.default_rng([seed, 12]).choice(N, rows, replace=False))).to(dev)
    xg = idx.xs.index_select(0, sel).contiguous()
    seg = torch.tensor([0, rows], dtype=torch.int64, device=dev)
    coff = torch.tensor([0, idx.K], dtype=torch.int64, device=dev)
    a = torch.empty(rows, dtype=torch.int32, device=dev)
    Cn = torch.empty_like(idx.C)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    stream = ctx.stream
    tac.tac_assign(ctx, xg, idx.C, coff, a, seg_off=seg, precision=tac.TAC_BF16)   # sizes the workspace
    tac.tac_update(ctx, xg, seg, a, idx.C, Cn)
    times = []
    for _ in range(3):
        ev[0].record(stream)
        tac.tac_assign(ctx, xg, idx.C, coff, a, seg_off=seg, precision=tac.TAC_BF16)
        tac.tac_update(ctx, xg, seg, a, idx.C, Cn)
        ev[1].record(stream)
        ev[1].synchronize()
        times.append(ev[0].elapsed_time(ev[1]))
    ms = float(np.median(times))
    del xg, Cn, a
    per_vec_global = ms / rows
    per_vec_tac = tac_iter_ms / N
    h = idx.host
    out = {"rows": rows, "centroids": idx.K, "ms_per_iter": ms,
           "vectors_per_s": rows / (ms / 1e3), "tac_speedup_per_vector": per_vec_global / per_vec_tac,
           **speedup_bounds(h["counts"], h["spread"], h["kappa"], idx.K),
           "note": "one segment: a uniform row sample against all K centroids of the build, same BF16 kernels; "
                   "work_ratio = N K / sum n_j kappa_j of the budget used (theta policy fill-then-relax)"}
    return out


SERVE_FRACTIONS = (0.3, 0.6, 0.9)   # Poisson arrival rates as fractions of the measured saturated rate


def serve_bench(idx, w, requests: int, seed: int = 0, label: str | None = None):
    """Encode service against the resident index: saturated throughput (all
    requests submitted at once), then Poisson arrivals at 0.3, 0.6 and 0.9 of
    it (first 5% of each run's requests discarded)."""
    import datagen
    from paper_2604_28142_amd.serve import EncodeService, GpuExecutor, ResidentIndex, run_load

    index = ResidentIndex(T=idx.T, K=idx.K, C=idx.C, cent_off=idx.cent_off, codebooks=idx.codebooks)
    ex = GpuExecutor(index, n_slots=3, max_rows=512 * 180)
    svc = EncodeService(ex, max_docs=512)
    lens, x, tok = datagen.serving_docs(w, requests, seed=seed + 20)
    edges = np.concatenate([[0], np.cumsum(lens)])
    docs = [(x[edges[i]:edges[i + 1]], tok[edges[i]:edges[i + 1]]) for i in range(len(lens))]
    run_load(svc, docs[:2000], None)                      # warm-up (workspaces, kernels)
    nsat = min(len(docs), 10_000)
    _, wall = run_load(svc, docs[:nsat], None)
    r_sat = nsat / wall
    log(f"serve {label or w.name}: saturated {r_sat:.0f} docs/s")
    out = {"index": label or f"{w.name}: K={w.k} centroids, PQ 32x256", "requests_per_rate": requests,
           "docs_mean_vectors": float(lens.mean()), "saturated_docs_per_s": r_sat,
           "graph_buckets_rows": ex.buckets if ex.graphs else None, "ledger_bytes": svc.ledger_cap, "rates": []}
    for i, frac in enumerate(SERVE_FRACTIONS):
        rate = frac * r_sat
        arr = datagen.poisson_arrivals(rate, len(docs), seed=seed + 3 * (i + 1))
        b0 = svc.stats.batches
        res, wall = run_load(svc, docs, arr)
        skip = len(docs) // 20
        lat = np.array([r.latency for r in res[skip:]])
        vec = float(lens[skip:].sum())
        out["rates"].append({"fraction_of_saturation": frac, "docs_per_s": rate,
                             "p50_ms": 1e3 * float(np.percentile(lat, 50)),
                             "p99_ms": 1e3 * float(np.percentile(lat, 99)),
                             "batches": svc.stats.batches - b0,
                             "vectors_per_s": vec / (wall * (len(docs) - skip) / len(docs))})
        log(f"serve {label or w.name}: {frac:.1f} x R_sat = {rate:.0f}/s p50 {out['rates'][-1]['p50_ms']:.2f} ms "
            f"p99 {out['rates'][-1]['p99_ms']:.2f} ms")
    svc.close()
    ex.close()
    return out


def index_structures(ctx, idx, w, N):
    """Inverted lists and document layout (Sect. 2.2) from the step's final
    assignment and codes; the build's vectors form documents of 30-180
    consecutive input rows (seeded).  Timed with HIP events on the context's
    stream; the inputs are mapped back to input order beforehand."""
    import datagen
    import torch
    import paper_2604_28142_amd as tac
    doc_off_h = datagen.build_doc_offsets(N, w.seed)
    D = doc_off_h.size - 1
    dev = idx.xs.device
    perm = idx.perm.long()
    doc_in = torch.from_numpy(np.repeat(np.arange(D, dtype=np.int32), np.diff(doc_off_h))).to(dev)
    doc_sorted = doc_in[perm].contiguous()
    assign_in = torch.empty_like(idx.assign)
    assign_in[perm] = idx.assign
    codes_in = torch.empty_like(idx.codes)
    codes_in[perm] = idx.codes
    K = idx.C.shape[0]
    M = idx.codes.shape[1]
    list_off = torch.empty(K + 1, dtype=torch.int64, device=dev)
    list_docs = torch.empty(N, dtype=torch.int32, device=dev)
    layout = torch.empty(N * (4 + M), dtype=torch.uint8, device=dev)
    doc_off = torch.from_numpy(doc_off_h).to(dev)
    stream = ctx.stream
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    tac.tac_ivf_build(ctx, idx.assign, doc_sorted, K, D, list_off, list_docs)    # sizes the workspace
    ms_ivf, ms_lay = [], []
    for _ in range(3):
        ev[0].record(stream)
        tac.tac_ivf_build(ctx, idx.assign, doc_sorted, K, D, list_off, list_docs)
        ev[1].record(stream)
        tac.tac_doc_layout(ctx, assign_in, codes_in, doc_off, layout)
        ev[2].record(stream)
        ev[2].synchronize()
        ms_ivf.append(ev[0].elapsed_time(ev[1]))
        ms_lay.append(ev[1].elapsed_time(ev[2]))
    entries = int(list_off[-1].item())
    lay_bytes = 2.0 * N * (4 + M)
    info = {"documents": D, "list_entries": entries, "ivf_build_ms": float(np.median(ms_ivf)),
            "doc_layout_ms": float(np.median(ms_lay)),
            "doc_layout_GBps": lay_bytes / (float(np.median(ms_lay)) / 1e3) / 1e9}
    rnorm_in = torch.empty_like(idx.rnorm)
    rnorm_in[perm] = idx.rnorm
    return info, (layout, doc_off, rnorm_in, list_off, list_docs)


def query_path(ctx, idx, w, index, nqueries=64, nq=32, kc=40, ncand=1000, graph_leg=True):
    """Both phases of retrieval (Sect. 2.2) for synthetic queries against the
    built index: the gather phase (kappa_c = `kc` centroids per query token,
    kappa_d = `ncand` candidates per query) and the refine phase (MaxSim over
    the PQ-coded candidates).  Timed with HIP events on the context's stream
    (median of 5 calls each; the gather call is synchronous).  Algorithmic work
    of refine per scored document token: 552 bytes from HBM (its centroid row,
    36 layout bytes, its norm) and 2 * 128 * nq flops; of the gather's
    similarities, 2 * 128 flops per (query token, centroid)."""
    import datagen
    import torch
    import paper_2604_28142_amd as tac
    layout, doc_off, rnorm_in, list_off, list_docs = index
    dev = idx.xs.device
    D = doc_off.shape[0] - 1
    Q = torch.from_numpy(datagen.queries(w, nqueries, nq, seed=w.seed)).to(dev)
    cand = torch.empty((nqueries, ncand), dtype=torch.int32, device=dev)
    gscore = torch.empty((nqueries, ncand), dtype=torch.float32, device=dev)
    gargs = (ctx, Q, idx.C, list_off, list_docs, D, kc, cand, gscore)
    tac.tac_gather(*gargs)                         # sizes the workspace
    gms = []
    for _ in range(5):
        t0 = time.perf_counter()
        tac.tac_gather(*gargs)
        gms.append((time.perf_counter() - t0) * 1e3)
    tg = float(np.median(gms))
    cand_h = cand.cpu().numpy()
    filled = int((cand_h >= 0).sum())
    scores = torch.empty(cand.shape, dtype=torch.float32, device=dev)
    args = (ctx, Q, idx.C, idx.codebooks, layout, doc_off, rnorm_in, cand, scores)
    tac.tac_maxsim(*args)
    stream = ctx.stream
    ms = []
    for _ in range(5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        tac.tac_maxsim(*args)
        e1.record(stream)
        e1.synchronize()
        ms.append(e0.elapsed_time(e1))
    t = float(np.median(ms))
    off_h = doc_off.cpu().numpy()
    ok = cand_h >= 0
    tokens = int((off_h[cand_h[ok] + 1] - off_h[cand_h[ok]]).sum())
    K = idx.C.shape[0]
    graph = graph_gather(ctx, idx, Q, list_off, list_docs, D, kc, ncand, cand_h) if graph_leg else None
    return {"queries": nqueries, "query_tokens": nq, "kappa_c": kc, "kappa_d": ncand, "graph_gather": graph,
            "gather": {"ms": tg, "queries_per_s": nqueries / (tg / 1e3), "candidates_filled": filled,
                       "similarity_TFLOPs": nqueries * nq * K * 2.0 * 128 / (tg / 1e3) / 1e12,
                       "note": "exact top-kappa_c centroids (the paper's HNSW approximates them); wall time of "
                               "the synchronous call"},
            "refine": {"ms": t, "queries_per_s": nqueries / (t / 1e3), "docs_per_s": filled / (t / 1e3),
                       "doc_tokens_scored": tokens, "GBps_algorithmic": tokens * 552 / (t / 1e3) / 1e9,
                       "TFLOPs_algorithmic": tokens * 2.0 * 128 * nq / (t / 1e3) / 1e12,
                       "scores_finite_where_filled": bool(torch.isfinite(scores[cand >= 0]).all().item())}}


ROUTER_STRIDE = 16


def graph_gather(ctx, idx, Q, list_off, list_docs, D, kc, kd, exact_cand):
    """The gather with its centroid step on the neighbour graph instead of the
    exact scan (the paper's HNSW setting: 32 neighbours, ef = 1.5 kappa_c):
    graph build time, search time of every query token, recall of the exact
    top-kappa_c, and the overlap of the kappa_d candidates with the exact
    gather's.  Routers: the first centroid of every token with centroids and
    every 16th centroid (a token's centroids sit in a few far-apart groups, so
    one entry per token would start most searches in the wrong group)."""
    import torch
    import paper_2604_28142_amd as tac
    dev = idx.xs.device
    K = idx.C.shape[0]
    B, nq = Q.shape[0], Q.shape[1]
    ef = min(64, (3 * kc + 1) // 2)
    coff = idx.host["cent_off"]
    ent = np.union1d(coff[:-1][np.diff(coff) > 0], np.arange(0, K, ROUTER_STRIDE))
    entry = torch.from_numpy(ent.astype(np.int32)).to(dev)
    nbr = torch.empty((K, 64), dtype=torch.int32, device=dev)
    stream = ctx.stream

    def timed(fn, reps):
        out = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn()
            e1.record(stream)
            e1.synchronize()
            out.append(e0.elapsed_time(e1))
        return float(np.median(out))

    torch.cuda.synchronize()
    build_ms = timed(lambda: tac.tac_graph_build(ctx, idx.C, nbr), 1)   # one build (seconds at 2M centroids)
    Qr = Q.reshape(B * nq, -1)
    gid = torch.empty((B * nq, kc), dtype=torch.int32, device=dev)
    gsim = torch.empty((B * nq, kc), dtype=torch.float32, device=dev)
    eid = torch.empty_like(gid)
    esim = torch.empty_like(gsim)
    search = lambda: tac.tac_graph_search(ctx, Qr, idx.C, nbr, entry, ef, kc, gid, gsim)
    search()
    search_ms = timed(search, 5)
    exact = lambda: tac.tac_centroid_topk(ctx, Qr, idx.C, kc, eid, esim)
    exact()
    exact_ms = timed(exact, 3)
    g, e = gid.cpu().numpy(), eid.cpu().numpy()
    recall = float(np.mean([len(set(g[r]) & set(e[r])) / kc for r in range(g.shape[0])]))
    cand = torch.empty((B, kd), dtype=torch.int32, device=dev)
    score = torch.empty((B, kd), dtype=torch.float32, device=dev)
    lists = lambda: tac.tac_gather_lists(ctx, gid.view(B, nq, kc), gsim.view(B, nq, kc), list_off, list_docs, K, D,
                                         kd, cand, score)
    lists()
    t0 = time.perf_counter()
    lists()
    lists_ms = (time.perf_counter() - t0) * 1e3
    c = cand.cpu().numpy()
    overlap = float(np.mean([len(set(c[b][c[b] >= 0]) & set(exact_cand[b][exact_cand[b] >= 0]))
                             / max(1, int((exact_cand[b] >= 0).sum())) for b in range(B)]))
    return {"degree": 32, "reverse_edges": 32, "ef": ef, "routers": int(entry.shape[0]),
            "routers_rule": f"first centroid of every token, and every {ROUTER_STRIDE}th centroid", "build_ms": build_ms,
            "search_ms": search_ms, "exact_topk_ms": exact_ms, "query_tokens": B * nq,
            "recall_at_kappa_c": recall, "lists_gather_ms": lists_ms,
            "gather_ms_total": search_ms + lists_ms, "candidate_overlap_with_exact": overlap}


def prepare(ctx, w, x, tok):
    """Group + budget (one eager pass, which also sizes the workspace), the
    seeded initial centroids and the PQ sample of a workload resident in HBM."""
    import datagen
    from paper_2604_28142_amd import index as IX
    N = x.shape[0]
    idx = IX.group_and_budget(ctx, x, tok, w.vocab, w.k)
    counts, kappa = idx.host["counts"], idx.host["kappa"]
    picks = datagen.init_picks(counts, kappa, w.seed)
    sample = datagen.pq_sample(N, w.pq_sample, w.seed)
    init_rows = datagen.pq_init_rows(sample.shape[0], w.pq_ksub, w.seed)
    IX.init_centroids(ctx, idx, picks)
    C0 = idx.C.clone()
    screen = kappa > 4
    F = 2.0 * 128 * float((counts[screen] * kappa[screen]).sum())   # algorithmic contraction flops per assign
    log(f"{w.name} budget: K={int(kappa.sum())}, max kappa={int(kappa.max())}, screen flops/assign={F:.3e}")
    return dict(idx=idx, counts=counts, kappa=kappa, picks=picks, sample=sample, init_rows=init_rows, C0=C0, F=F)


def make_step(ctx, w, x, tok, P, stream):
    """One pass of the whole path on a prepared workload, the Lloyd iterations
    replayed from `lp`'s graph; returns (step ms, Lloyd ms, final-assign kernel
    ms, encode kernel ms) -- the kernel times when kernel timing is on."""
    import torch
    import paper_2604_28142_amd as tac
    from paper_2604_28142_amd import index as IX
    idx = P["idx"]
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]

    def step(lp):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = tac.tac_budget(ctx, x, tok, w.vocab, w.k, perm=idx.perm, xs=idx.xs, seg_off=idx.seg_off,
                             cent_off=idx.cent_off)
        assert np.array_equal(out["kappa"], P["kappa"])
        IX.init_centroids(ctx, idx, P["picks"])
        ev[0].record(stream)
        lp.replay()
        ev[1].record(stream)
        IX.final_assign(ctx, idx, precision=lp.precision)
        IX.train_pq(ctx, idx, P["sample"], P["init_rows"], M=w.pq_m, ksub=w.pq_ksub, iters=10)
        IX.encode_all(ctx, idx)
        torch.cuda.synchronize()
        timing = ctx.timing_enabled
        return ((time.perf_counter() - t0) * 1e3, ev[0].elapsed_time(ev[1]),
                ctx.kernel_ms(tac._lib.TAC_SLOT_ASSIGN) if timing else float("nan"),
                ctx.kernel_ms(tac._lib.TAC_SLOT_ENCODE) if timing else float("nan"))
    return step


PRECS = ("bf16", "f16", "fp32")


def prec_id(tac, name: str) -> int:
    return {"bf16": tac.TAC_BF16, "f16": tac.TAC_F16, "fp32": tac.TAC_FP32}[name]


def run_headline(args, dev):
    """The headline workload: K timed steps of the headline precision, the
    comparison legs, kernel times and rooflines, index structures, the query
    path, global k-means, the encode service and the CPU oracle baseline.
    Returns the JSON line (without the c3 block); frees its device state."""
    import torch

    import datagen
    import paper_2604_28142_amd as tac
    from paper_2604_28142_amd import autotune
    from paper_2604_28142_amd import index as IX

    w = dataclasses.replace(datagen.WORKLOADS[args.config], seed=args.seed)
    t0 = time.time()
    x_h, tok_h = datagen.make(w)
    N = x_h.shape[0]
    log(f"data: {N} x 128 generated in {time.time() - t0:.1f}s")
    x = torch.from_numpy(x_h).to(dev)
    tok = torch.from_numpy(tok_h).to(dev)
    ctx = tac.Context(0)
    stream = torch.cuda.current_stream(dev)
    if args.calibration_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    P = prepare(ctx, w, x, tok)
    idx, counts, kappa, C0, F = P["idx"], P["counts"], P["kappa"], P["C0"], P["F"]

    hl = args.headline
    legs = [hl] + [nm for nm in PRECS if nm != hl and not getattr(args, f"no_{nm}", False)]
    loops, tuned, tuning = {}, {}, {}
    for name in legs:
        prec = prec_id(tac, name)
        if not args.no_autotune:
            # launch tuning for this precision, measured on the initial centroids (cached per workload);
            # it is baked into the captured graph
            r = autotune.tune_assign(ctx, idx.xs, idx.C, idx.cent_off, idx.seg_off, precision=prec,
                                     host_seg_off=idx.host["seg_off"], host_cent_off=idx.host["cent_off"])
            tuned[name] = {"tuning": r["tuning"], "assign_ms": r["ms"], "default_assign_ms": r["default_ms"],
                           "cached": r["cached"]}
            log(f"autotune {name}: {r['tuning']} {r['ms']:.2f} ms (default {r['default_ms']:.2f} ms)")
        tuning[name] = ctx.get_tuning()
        lp = IX.LloydLoop(ctx, idx, iters=args.iters, precision=prec)
        idx.C.copy_(C0)
        lp.run()                       # eager: sizes the workspace, sets kernel attributes
        torch.cuda.synchronize()
        lp.capture()
        loops[name] = lp
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]

    def lloyd_ms(lp):
        idx.C.copy_(C0)
        ev[0].record(stream)
        lp.replay()
        ev[1].record(stream)
        ev[1].synchronize()
        return ev[0].elapsed_time(ev[1])

    step = make_step(ctx, w, x, tok, P, stream)
    head = loops[hl]
    ctx.set_tuning(**tuning[hl])
    # kernel events: each step's final assignment (one launch of the persistent 16-bit assignment
    # kernel) and its encode kernel are timed on the context's stream inside the timed region
    ctx.enable_timing(True)
    for _ in range(args.warmup):
        step(head)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    res = [step(head) for _ in range(args.steps)]
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t_start) * 1e3
    ctx.enable_timing(False)
    step_ms = [r[0] for r in res]
    lloyd = [r[1] for r in res]
    assign_kernel_ms = float(np.mean([r[2] for r in res]))
    encode_kernel_ms = float(np.mean([r[3] for r in res]))
    final_head = idx.assign.clone()
    lloyd_med = float(np.median(lloyd))
    value = N * args.iters / (lloyd_med / 1e3)
    log(f"{hl}: steps {['%.1f' % s for s in step_ms]} ms, Lloyd {['%.2f' % l for l in lloyd]} ms")

    # comparison legs: the same captured Lloyd graph and final assignment in the other precisions
    extra = {}
    leg_ms = {hl: lloyd_med}
    same_all = True
    for name in legs[1:]:
        ctx.set_tuning(**tuning[name])
        ms = float(np.median([lloyd_ms(loops[name]) for _ in range(2)]))
        leg_ms[name] = ms
        IX.final_assign(ctx, idx, precision=prec_id(tac, name))
        same = bool(torch.equal(idx.assign, final_head))
        same_all = same_all and same
        extra[name] = {"lloyd_ms_per_iter": ms / args.iters, "value": N * args.iters / (ms / 1e3),
                       "final_argmin_identical_to_" + hl: same}
        log(f"{name}: Lloyd {ms:.1f} ms; identical final assignments: {same}")
    ctx.set_tuning(**tuning[hl])
    if "fp32" in leg_ms:
        for name in ("bf16", "f16"):
            if name in leg_ms:
                extra[f"{name}_over_fp32"] = leg_ms["fp32"] / leg_ms[name]
    extra["final_argmin_identical"] = same_all

    # dominant kernel: the persistent assignment kernel, timed with HIP events on its stream
    ctx.enable_timing(True)
    idx.C.copy_(C0)
    kms, stats = {}, {}
    for name in legs:
        ctx.set_tuning(**tuning[name])
        vals = []
        for _ in range(3):
            tac.tac_assign(ctx, idx.xs, idx.C, idx.cent_off, idx.assign, seg_off=idx.seg_off,
                           precision=prec_id(tac, name))
            vals.append(ctx.kernel_ms(tac._lib.TAC_SLOT_ASSIGN))
        kms[name] = float(np.mean(vals))
        stats[name] = tac.tac_assign_stats(ctx)
    ctx.set_tuning(**tuning[hl])
    tac.tac_update(ctx, idx.xs, idx.seg_off, idx.assign, idx.C, loops[hl].other)
    upd_ms = ctx.kernel_ms(tac._lib.TAC_SLOT_UPDATE)
    IX.encode_all(ctx, idx)
    enc_ms = ctx.kernel_ms(tac._lib.TAC_SLOT_ENCODE)
    ctx.enable_timing(False)
    achieved = F / (assign_kernel_ms / 1e3) / 1e12
    extra["kernels_ms"] = {f"assign_{hl}_timed_region": assign_kernel_ms, "pq_encode_timed_region": encode_kernel_ms,
                           **{f"assign_{nm}": kms[nm] for nm in legs}, "update_means": upd_ms, "pq_encode": enc_ms}
    extra["assign_counters"] = stats
    if tuned:
        extra["autotune"] = tuned
    extra["lloyd_ms_per_iter"] = lloyd_med / args.iters
    extra["screen_flops_per_assign"] = F
    extra["mfma_executed_tflops"] = {nm: PRODUCTS[nm] * F / (kms[nm] / 1e3) / 1e12 for nm in legs}
    if "fp32" in kms:
        extra["fp32_roofline_frac"] = F / (kms["fp32"] / 1e3) / 1e12 / PEAK["fp32"]
    copy_gbs = copy_bandwidth(torch, dev)
    extra["segment_roofline"] = {nm: segment_roofline(counts, kappa, kms[nm], nm, copy_gbs) for nm in legs}
    log(f"per-token roofline: {extra['segment_roofline']}")

    extra["index_structures"], index = index_structures(ctx, idx, w, N)
    log(f"inverted lists + document layout: {extra['index_structures']}")
    extra["query_path"] = query_path(ctx, idx, w, index)
    log(f"query path (gather + refine): {extra['query_path']}")
    del index

    # the final centroids and codebooks of the headline precision for the index-based legs
    idx.C.copy_(C0)
    head.replay()
    IX.final_assign(ctx, idx, precision=head.precision)
    if args.global_baseline:
        extra["global_kmeans"] = global_baseline(ctx, idx, w, lloyd_med / args.iters, args.global_baseline)
        log(f"global k-means: {extra['global_kmeans']}")
    loops.clear()
    del head
    if not args.no_serve:
        extra["encode_service"] = serve_bench(idx, w, args.serve_requests)
    ctx.close()
    del idx, P, x, tok, final_head
    torch.cuda.synchronize()
    torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu_baseline:
        n_cpu = min(args.cpu_sample, N)
        cpu, cpu1 = cpu_baseline(x_h, tok_h, w, n_cpu, min(args.cpu_one_core_sample, N))
        cpu["value"] = float(cpu["value"])
        if cpu1:
            extra["cpu_baseline_one_core"] = cpu1

    return {
        "metric": "vectors assigned/sec per Lloyd iter, bf16 vs fp32 at equal argmin; encode p99",
        "value": value,
        "unit": "vectors/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": float(np.mean(step_ms)),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": hl,
        "data": "synthetic",
        "config": {"workload": f"{args.config}: {WORKLOAD_TEXT[args.config]}", "vectors": N, "tokens": w.vocab,
                   "centroids": w.k, "lloyd_iters": args.iters, "budget": "mu=128 tau=256 eps=4 theta=39",
                   "seed": args.seed, "timed_region_ms": wall},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK[hl], "unit": "TFLOP/s",
                     "frac": achieved / PEAK[hl],
                     "traffic": measured_traffic(args.config, hl) if args.seed == 0 else None,
                     "mfma_busy": measured_mfma_busy(args.config, hl) if args.seed == 0 else None,
                     "kernel": f"assign_main<{hl}> (persistent screen + per-lane top-3 + certificate)"},
        "cpu_baseline": cpu,
        **extra,
    }


def run_c3(args, dev):
    """The 50M-row, 2,097,152-centroid workload: one warm-up and one timed step
    with the BF16 screen (Lloyd replayed from its graph), the FP16 and FP32
    Lloyd legs run eagerly (launch overhead is negligible at about 0.5-1.8 s
    per iteration) with their final assignments compared, per-token rooflines
    of each precision's final-assignment kernel, and the encode service against
    the built index."""
    import torch

    import datagen
    import paper_2604_28142_amd as tac
    from paper_2604_28142_amd import autotune
    from paper_2604_28142_amd import index as IX

    w = dataclasses.replace(datagen.WORKLOADS["c3"], seed=args.seed)
    t0 = time.time()
    x_h, tok_h = datagen.make(w)
    N = x_h.shape[0]
    x = torch.from_numpy(x_h).to(dev)
    tok = torch.from_numpy(tok_h).to(dev)
    del x_h, tok_h
    log(f"c3 data: {N} x 128 generated and copied in {time.time() - t0:.1f}s")
    ctx = tac.Context(0)
    stream = torch.cuda.current_stream(dev)
    P = prepare(ctx, w, x, tok)
    idx, counts, kappa, C0, F = P["idx"], P["counts"], P["kappa"], P["C0"], P["F"]
    out = {"workload": f"c3: {WORKLOAD_TEXT['c3']}", "vectors": N, "centroids": w.k, "lloyd_iters": args.iters,
           "max_kappa": int(kappa.max()), "screen_flops_per_assign": F,
           **speedup_bounds(counts, idx.host["spread"], kappa, w.k)}
    legs = ["bf16"] + [nm for nm in ("f16", "fp32") if not getattr(args, f"no_{nm}", False)]
    tuning = {}
    for name in legs:
        if name != "fp32" and not args.no_autotune:
            r = autotune.tune_assign(ctx, idx.xs, idx.C, idx.cent_off, idx.seg_off, precision=prec_id(tac, name),
                                     space={"tile": autotune.SPACE["tile"]},
                                     host_seg_off=idx.host["seg_off"], host_cent_off=idx.host["cent_off"])
            out[f"autotune_{name}"] = {"tuning": r["tuning"], "assign_ms": r["ms"], "default_assign_ms": r["default_ms"],
                                       "cached": r["cached"], "trials": r.get("trials")}
            log(f"c3 autotune {name}: {r['tuning']} {r['ms']:.1f} ms (default {r['default_ms']:.1f} ms)")
        else:
            ctx.set_tuning(**autotune.DEFAULT)
        tuning[name] = ctx.get_tuning()

    ctx.set_tuning(**tuning["bf16"])
    lp = IX.LloydLoop(ctx, idx, iters=args.iters, precision=tac.TAC_BF16)
    idx.C.copy_(C0)
    lp.run()
    torch.cuda.synchronize()
    lp.capture()
    step = make_step(ctx, w, x, tok, P, stream)
    ctx.enable_timing(True)
    warm = step(lp)
    timed = step(lp)
    ctx.enable_timing(False)
    final_bf16 = idx.assign.clone()
    C_bf16 = idx.C.clone()
    lloyd = {"bf16": timed[1]}
    kms = {"bf16": timed[2]}
    out["bf16"] = {"step_ms": timed[0], "warmup_step_ms": warm[0], "lloyd_ms": timed[1],
                   "lloyd_ms_per_iter": timed[1] / args.iters, "value": N * args.iters / (timed[1] / 1e3),
                   "assign_kernel_ms": timed[2], "pq_encode_kernel_ms": timed[3]}
    log(f"c3 bf16: step {timed[0]:.0f} ms, Lloyd {timed[1]:.0f} ms, assign kernel {timed[2]:.1f} ms")
    del lp
    same_all = True
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    for name in legs[1:]:
        ctx.set_tuning(**tuning[name])
        lpx = IX.LloydLoop(ctx, idx, iters=args.iters, precision=prec_id(tac, name))
        idx.C.copy_(C0)
        ev[0].record(stream)
        lpx.run()
        ev[1].record(stream)
        ev[1].synchronize()
        lloyd[name] = ev[0].elapsed_time(ev[1])
        del lpx
        ctx.enable_timing(True)
        IX.final_assign(ctx, idx, precision=prec_id(tac, name))
        kms[name] = ctx.kernel_ms(tac._lib.TAC_SLOT_ASSIGN)
        ctx.enable_timing(False)
        same = bool(torch.equal(idx.assign, final_bf16))
        same_all = same_all and same
        out[name] = {"lloyd_ms": lloyd[name], "lloyd_ms_per_iter": lloyd[name] / args.iters,
                     "value": N * args.iters / (lloyd[name] / 1e3), "assign_kernel_ms": kms[name],
                     "final_argmin_identical_to_bf16": same, "assign_counters": tac.tac_assign_stats(ctx)}
        log(f"c3 {name}: Lloyd {lloyd[name]:.0f} ms, assign kernel {kms[name]:.1f} ms, identical: {same}")
    out["final_argmin_identical"] = same_all
    if "fp32" in lloyd:
        for name in ("bf16", "f16"):
            if name in lloyd:
                out[f"{name}_over_fp32"] = lloyd["fp32"] / lloyd[name]
    out["roofline"] = {nm: {"achieved_tflops": F / (kms[nm] / 1e3) / 1e12, "peak": PEAK[nm],
                            "frac": F / (kms[nm] / 1e3) / 1e12 / PEAK[nm]} for nm in kms}
    copy_gbs = copy_bandwidth(torch, dev)
    out["segment_roofline"] = {nm: segment_roofline(counts, kappa, kms[nm], nm, copy_gbs) for nm in kms}
    log(f"c3 rooflines: {out['roofline']}")

    # the built index (BF16 centroids and codebooks) for the query path and the encode service
    idx.C.copy_(C_bf16)
    idx.assign = final_bf16
    del C_bf16
    if not args.no_query:
        t0 = time.time()
        out["index_structures"], index = index_structures(ctx, idx, w, N)
        out["query_path"] = query_path(ctx, idx, w, index)
        out["query_path"]["wall_s"] = time.time() - t0
        log(f"c3 query path: {out['query_path']}")
        del index
    if not args.no_serve:
        out["encode_service"] = serve_bench(idx, w, args.c3_serve_requests,
                                            label=f"c3: K={w.k} centroids (max kappa {int(kappa.max())}), PQ 32x256")
    ctx.close()
    del idx, P, x, tok
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c1", choices=["c0", "c1", "c3"])
    ap.add_argument("--iters", type=int, default=10)
    ap.add_argument("--seed", type=int, default=0, help="data seed of the workload (0: the headline data)")
    ap.add_argument("--cpu-sample", type=int, default=300_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-one-core-sample", type=int, default=20_000,
                    help="rows of the single-thread oracle timing (0: skip it)")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-f16", action="store_true", help="skip the FP16-screen comparison leg")
    ap.add_argument("--no-bf16", action="store_true", help="skip the BF16-screen comparison leg")
    ap.add_argument("--headline", default="bf16", choices=["bf16", "f16"],
                    help="16-bit screen timed in the steps (the other runs as a comparison leg)")
    ap.add_argument("--serve-requests", type=int, default=20_000)
    ap.add_argument("--c3-serve-requests", type=int, default=8_000)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-c3", action="store_true", help="skip the 50M-row, 2,097,152-centroid block")
    ap.add_argument("--no-query", action="store_true", help="skip the 50M-row block's query path (graph build included)")
    ap.add_argument("--global-baseline", type=int, default=200_000, metavar="ROWS",
                    help="rows of the global k-means leg (one segment, all K centroids); 0 skips it")
    ap.add_argument("--calibration-copy", action="store_true",
                    help="first run one plain 1 GiB device copy (reference dispatch for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the multi-GPU design is "
              f"described but not built", file=sys.stderr)
        sys.exit(2)

    import torch
    dev = torch.device("cuda:0")
    line = run_headline(args, dev)
    if args.config != "c3" and not args.no_c3:
        t0 = time.time()
        line["c3"] = run_c3(args, dev)
        line["c3"]["block_wall_s"] = time.time() - t0
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
