"""Benchmark of the batched FBPQ search on one MI355X.

Workload (default): 10M SIFT-like points (256-component Gaussian mixture,
uint8 values), multi-index with T=4096 centroids per half (16.7M cells), PQ
M=16 x 256 words on displacements, one batch of 10,000 queries with L=10,000
candidates and k=100. A step is one full search of the batch (first layer,
traversal, layout, scan with fused top-k), queries and results resident in HBM.

Prints one JSON line: queries/s, step latency percentiles, per-kernel device
time from HIP events, the scan kernel's achieved bandwidth against the HBM
roofline (HIP events around that one kernel inside the timed steps), and the
FP64 CPU oracle timed on a bounded sample of the same batch.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
FP32_MFMA_TFLOPS = 157.3

WORKLOADS = {
    "batched": dict(N=10_000_000, T=4096, M=16, nq=10_000, L=10_000, k=100),
    "plain": dict(N=100_000, T=64, M=8, nq=100, L=10_000, k=10),
    # served: Zipf(1.1) cell sizes over T^2 cells, Poisson arrivals
    "served": dict(N=1_000_000_000, T=16384, M=8, L=(10_000, 30_000, 100_000), k=10,
                   offered=(1000, 2000, 5000, 10000, 20000, 40000, 80000)),
    # local codebooks (HBPQ): per-query L log-uniform in [L_lo, L_hi]
    "local": dict(N=100_000_000, T=4096, M=16, nq=10_000, L_lo=10_000, L_hi=100_000, k=10),
    # GIST-like width: D = 384 at the same 8-byte codes, FBPQ against the O(D) scan at each L
    "gist": dict(N=50_000_000, D=384, T=1024, M=8, nq=10_000, L=(10_000, 30_000, 100_000), k=10),
}


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def roofline_models(ix, nq: int, L: int, k: int, ncand: int) -> dict:
    """Algorithmic work per launch of the kernels a roofline is reported for.

    score:     M code bytes per candidate (the scan's HBM stream)
    select:    the 4-byte distance of every candidate, plus k (id, distance) results per query
    prefix:    the 4-byte approximate key of every (query, half, centroid), plus P (key, index) outputs
    half_keys: 2 (D/2) FLOP per (query, half, centroid) on the FP32 matrix cores
    """
    P = 128
    csrc = os.path.join(ROOT, "paper_1404_1831_amd", "csrc")
    gbs = dict(bound="hbm", peak=HBM_PEAK_GBPS, unit="GB/s", scale=1e9)
    return {
        "score": dict(gbs, kernel="k_score_query", amount=ncand * ix.M, what="code bytes",
                      source=os.path.join(csrc, "k_items.hip")),
        "select": dict(gbs, kernel="k_select_dist", amount=ncand * 4 + nq * k * 12, what="distance and result bytes",
                       source=os.path.join(csrc, "k_items.hip")),
        "prefix": dict(gbs, kernel="k_prefix_wave", amount=nq * 2 * ix.T * 4 + nq * 2 * P * 12,
                       what="approximate-key and prefix bytes", source=os.path.join(csrc, "k_rank.hip")),
        "half_keys": dict(bound="mfma", peak=FP32_MFMA_TFLOPS, unit="TFLOP/s", scale=1e12, kernel="k_half_approx",
                          amount=nq * 2 * ix.T * (ix.D // 2) * 2, what="FP32 matrix-core FLOP",
                          source=os.path.join(csrc, "k_rank.hip")),
    }


def traffic_from_profile(kernel: str, source: str):
    """HBM bytes per launch from the committed counter summary of this kernel,
    if the kernel's source file is unchanged since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    with open(source, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    if rec.get("source_sha256") != sha:
        return None
    return rec.get("hbm_bytes_per_launch")


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="batched", choices=sorted(WORKLOADS))
    ap.add_argument("--nq", type=int, default=None)
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target duration of the CPU oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--served-n", type=int, default=0, help="served workload: points (default 1e9)")
    ap.add_argument("--served-seconds", type=float, default=2.0, help="served workload: seconds per offered load")
    ap.add_argument("--served-lanes", type=int, default=2)
    ap.add_argument("--served-batch", type=int, default=512)
    ap.add_argument("--plain-queries", type=int, default=200,
                    help="queries searched one launch sequence at a time, for the per-query comparison")
    ap.add_argument("--adc-steps", type=int, default=3,
                    help="batches searched with the O(D) Multi-D-ADC rerank, for the comparison (0: skip)")
    ap.add_argument("--profile-steps", type=int, default=3,
                    help="untimed steps with every kernel timed, for the per-kernel breakdown")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="also run a plain elementwise copy of this many MiB (read once, written once), "
                         "the reference dispatch for scaling HBM traffic counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this search runs on one GPU; --gpus above 1 is not supported"}))
        return 2

    import torch

    import synth
    from paper_1404_1831_amd.build import LIB
    if not os.path.exists(LIB):
        from paper_1404_1831_amd.build import build
        build()
    from paper_1404_1831_amd import fbpq

    w = dict(WORKLOADS[args.workload])
    if args.workload == "served":
        return run_served(args, w)
    if args.workload == "local":
        return run_local(args, w)
    if args.workload == "gist":
        return run_gist(args, w)
    if args.nq:
        w["nq"] = args.nq
    dev = torch.device("cuda:0")
    t0 = time.time()
    means = synth.gmm_means(0)
    base = synth.sample_points(w["N"], means, 1, dev)
    ix = synth.build_index(base, w["T"], w["M"], keep_base=False)
    del base
    Q = synth.make_queries(w["nq"], means, 2, dev)
    torch.cuda.synchronize()
    log(f"index built in {time.time() - t0:.1f}s: N={ix.N} T={ix.T} M={ix.M} "
        f"nonempty cells={int((np.diff(ix.offsets) > 0).sum())}")

    h = fbpq.fbpq_index_create(ix, 0)
    fbpq.fbpq_build_tables(h)
    nq, L, k = w["nq"], w["L"], w["k"]
    d_q = torch.from_numpy(Q).to(dev).contiguous()
    d_ids = torch.empty(nq, k, dtype=torch.int64, device=dev)
    d_d = torch.empty(nq, k, dtype=torch.float32, device=dev)
    Ls = np.full(nq, L, np.int64)
    ks = np.full(nq, k, np.int32)
    stream = torch.cuda.current_stream(dev)

    for i in range(args.warmup):
        fbpq.fbpq_search_device(h, d_q, Ls, ks, k, d_ids, d_d, stream)
        log(f"warmup {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()

    # per-kernel breakdown (untimed): HIP events around every launch
    fbpq.fbpq_set_option(h, "profile", 1)
    fbpq.fbpq_set_option(h, "profile_mask", -1)
    for s in range(len(fbpq.STAGES)):
        fbpq.fbpq_profile_read(h, s, reset=True)
    for _ in range(args.profile_steps):
        fbpq.fbpq_search_device(h, d_q, Ls, ks, k, d_ids, d_d, stream)
    torch.cuda.synchronize()
    prof = {}
    for s, name in enumerate(fbpq.STAGES):
        ms, n = fbpq.fbpq_profile_read(h, s, reset=True)
        prof[name] = {"ms_per_launch": ms / n if n else None, "launches": n}
    log("kernels: " + ", ".join(f"{n}={v['ms_per_launch']:.4f}" for n, v in prof.items() if v["ms_per_launch"]))

    # the dominant kernel among those with a roofline model
    ncand = nq * min(L, ix.N)
    models = roofline_models(ix, nq, L, k, ncand)
    dom = max(models, key=lambda s: prof[s]["ms_per_launch"] or 0.0)
    fbpq.fbpq_set_option(h, "profile_mask", 1 << fbpq.STAGES.index(dom))

    step_ms = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        a = time.perf_counter()
        fbpq.fbpq_search_device(h, d_q, Ls, ks, k, d_ids, d_d, stream)
        torch.cuda.synchronize()
        step_ms.append((time.perf_counter() - a) * 1e3)
    torch.cuda.synchronize()
    total_s = time.perf_counter() - t_start
    log(f"timed {args.steps} steps in {total_s:.3f}s")
    dom_ms, dom_n = fbpq.fbpq_profile_read(h, fbpq.STAGES.index(dom), reset=True)
    fbpq.fbpq_set_option(h, "profile", 0)
    dom_ms = dom_ms / dom_n if dom_n else None

    # the same batch with the first round replayed from a captured HIP graph
    fbpq.fbpq_set_option(h, "graph", 1)
    for _ in range(2):  # the first call captures
        fbpq.fbpq_search_device(h, d_q, Ls, ks, k, d_ids, d_d, stream)
    torch.cuda.synchronize()
    a = time.perf_counter()
    for _ in range(args.steps):
        fbpq.fbpq_search_device(h, d_q, Ls, ks, k, d_ids, d_d, stream)
        torch.cuda.synchronize()
    graph_ms = (time.perf_counter() - a) * 1e3 / args.steps
    fbpq.fbpq_set_option(h, "graph", 0)
    log(f"graph replays: {graph_ms:.3f} ms per batch")

    # plain per-query launches at equal L and k, on the first queries of the batch
    npl = min(nq, args.plain_queries)
    Ls1, ks1 = np.full(1, L, np.int64), np.full(1, k, np.int32)
    for i in range(min(npl, 5)):
        fbpq.fbpq_search_device(h, d_q[i:i + 1], Ls1, ks1, k, d_ids[i:i + 1], d_d[i:i + 1], stream)
    torch.cuda.synchronize()
    a = time.perf_counter()
    for i in range(npl):
        fbpq.fbpq_search_device(h, d_q[i:i + 1], Ls1, ks1, k, d_ids[i:i + 1], d_d[i:i + 1], stream)
    torch.cuda.synchronize()
    plain_s = time.perf_counter() - a
    log(f"plain per-query launches: {npl} queries in {plain_s:.3f}s")

    ms_per_step = total_s * 1e3 / args.steps
    qps = nq / (ms_per_step / 1e3)
    model = models[dom]
    achieved = model["amount"] / (dom_ms * 1e-3) / model["scale"] if dom_ms else None
    roof = {"bound": model["bound"], "achieved": achieved, "peak": model["peak"], "unit": model["unit"],
            "frac": achieved / model["peak"] if achieved else None,
            "traffic": traffic_from_profile(model["kernel"], model["source"]),
            "kernel": model["kernel"], "algorithmic_per_launch": model["amount"], "what": model["what"],
            "ms_per_launch": dom_ms, "launches": dom_n}
    score_ms = prof["score"]["ms_per_launch"]
    scan_GBps = ncand * ix.M / (score_ms * 1e-3) / 1e9 if score_ms else None

    res_ids = d_ids.cpu().numpy()
    res_d = d_d.cpu().numpy()
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        threads = oracle.host_threads()
        n0 = min(nq, 2 * threads)
        a = time.perf_counter()
        o_ids, o_d, _, _ = oracle.search(ix, Q[:n0], L, k, nthreads=threads)
        t_first = time.perf_counter() - a
        n1 = int(min(nq, max(n0, n0 * args.cpu_seconds / max(t_first, 1e-3))))
        if n1 > n0:
            a = time.perf_counter()
            o_ids, o_d, _, _ = oracle.search(ix, Q[:n1], L, k, nthreads=threads)
            t_cpu = time.perf_counter() - a
        else:
            n1, t_cpu = n0, t_first
        overlap = float(np.mean([len(set(res_ids[r]) & set(o_ids[r])) / k for r in range(n1)]))
        rel = np.abs(res_d[:n1].astype(np.float64) - o_d) / np.maximum(o_d, 1.0)
        cpu = {"value": n1 / t_cpu, "unit": "queries/s", "cores": threads, "kind": "oracle",
               "sample": f"first {n1} of the {nq} queries, same index, L={L}, k={k}",
               "topk_overlap_with_gpu": overlap, "max_rel_dist_diff": float(rel.max())}
        log(f"cpu oracle: {n1} queries in {t_cpu:.1f}s on {threads} threads")

    # the Multi-D-ADC baseline on the GPU: the same search with every candidate
    # scored by explicit O(D) reconstruction instead of the FBPQ tables
    adc = None
    if args.adc_steps > 0:
        fbpq.fbpq_set_option(h, "adc_od", 1)
        for _ in range(2):
            fbpq.fbpq_search_device(h, d_q, Ls, ks, k, d_ids, d_d, stream)
        torch.cuda.synchronize()
        a = time.perf_counter()
        for _ in range(args.adc_steps):
            fbpq.fbpq_search_device(h, d_q, Ls, ks, k, d_ids, d_d, stream)
        torch.cuda.synchronize()
        adc_ms = (time.perf_counter() - a) * 1e3 / args.adc_steps
        fbpq.fbpq_set_option(h, "adc_od", 0)
        adc = {"ms_per_step": adc_ms, "value": nq / (adc_ms / 1e3), "fbpq_speedup": adc_ms / ms_per_step}
        log(f"Multi-D-ADC O(D) baseline: {adc_ms:.3f} ms per batch (FBPQ {ms_per_step:.3f} ms)")

    # OPQ: the same index declared to live in a rotated space, searched with the
    # batch expressed in the original space (Rot^T q), so the rotation kernel
    # maps it back: the cost of the query rotation inside a full search
    opq = None
    if args.adc_steps > 0:
        import dataclasses
        Rot = synth.random_rotation(ix.D, seed=23)
        rix = dataclasses.replace(ix, Rot=Rot)
        hr = fbpq.fbpq_index_create(rix, 0)
        fbpq.fbpq_build_tables(hr)
        d_qo = (d_q.double() @ torch.from_numpy(Rot).to(dev).double()).float().contiguous()
        for _ in range(2):
            fbpq.fbpq_search_device(hr, d_qo, Ls, ks, k, d_ids, d_d, stream)
        torch.cuda.synchronize()
        fbpq.fbpq_set_option(hr, "profile", 1)
        fbpq.fbpq_set_option(hr, "profile_mask", 1 << fbpq.STAGES.index("rotate"))
        a = time.perf_counter()
        for _ in range(args.adc_steps):
            fbpq.fbpq_search_device(hr, d_qo, Ls, ks, k, d_ids, d_d, stream)
        torch.cuda.synchronize()
        opq_ms = (time.perf_counter() - a) * 1e3 / args.adc_steps
        rot_ms, rot_n = fbpq.fbpq_profile_read(hr, fbpq.STAGES.index("rotate"), reset=True)
        fbpq.fbpq_free_index(hr)
        opq = {"ms_per_step": opq_ms, "value": nq / (opq_ms / 1e3),
               "rotate_ms_per_launch": rot_ms / rot_n if rot_n else None}
        log(f"OPQ rotation: {opq_ms:.3f} ms per batch, rotation kernel "
            f"{(rot_ms / rot_n if rot_n else float('nan')):.4f} ms")

    if args.calibrate_copy_mib > 0:
        nel = args.calibrate_copy_mib * (1 << 20) // 4
        x = torch.ones(nel, dtype=torch.float32, device=dev)
        y = torch.empty_like(x)
        for _ in range(3):
            torch.neg(x, out=y)
        torch.cuda.synchronize()
        log(f"copy calibration: 3 x {args.calibrate_copy_mib} MiB read + written")
        del x, y

    fbpq.fbpq_free_index(h)
    out = {
        "metric": "queries/s at fixed L, Recall@10 = oracle, 1 GPU; p50/p99 latency; scan GB/s",
        "value": qps,
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "p50_ms": float(np.percentile(step_ms, 50)),
        "p99_ms": float(np.percentile(step_ms, 99)),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload} FBPQ: N={ix.N}, T={ix.T} per half, M={ix.M}, "
                               f"nq={nq} per batch, L={L}, k={k}",
                   "N": ix.N, "T": ix.T, "M": ix.M, "nq": nq, "L": L, "k": k},
        "kernels": prof,
        "graph_replay": {"ms_per_step": graph_ms, "value": nq / (graph_ms / 1e3)},
        "multi_d_adc_baseline": adc,
        "opq_rotation": opq,
        "plain_per_query": ({"queries": npl, "value": npl / plain_s, "unit": "queries/s",
                             "ms_per_query": plain_s * 1e3 / npl} if npl > 0 else None),
        "scan_GBps": scan_GBps,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))
    return 0


def run_local(args, w) -> int:
    """Local codebooks (HBPQ, Section 3.2): a batch with per-query L, timed
    with the local codebooks and, on the same index and queries, with the
    global ones (FBPQ)."""
    import torch

    import synth
    from paper_1404_1831_amd.build import LIB
    if not os.path.exists(LIB):
        from paper_1404_1831_amd.build import build
        build()
    from paper_1404_1831_amd import fbpq

    if args.nq:
        w["nq"] = args.nq
    dev = torch.device("cuda:0")
    t0 = time.time()
    means = synth.gmm_means(0)
    base = synth.sample_points(w["N"], means, 1, dev)
    gix = synth.build_index(base, w["T"], w["M"], keep_base=False)
    del base
    torch.cuda.empty_cache()
    ix = synth.with_local_codebooks(gix)
    nq, k = w["nq"], w["k"]
    Q = synth.make_queries(nq, means, 2, dev)
    Ls, _ = synth.draw_L_k(nq, 3, w["L_lo"], w["L_hi"])
    Ls = np.ascontiguousarray(Ls, np.int64)
    ks = np.full(nq, k, np.int32)
    log(f"index built in {time.time() - t0:.1f}s: N={ix.N} T={ix.T} M={ix.M}, local codebooks "
        f"{2 * ix.QL.nbytes / 2**20:.0f} MiB; mean L {Ls.mean():.0f}")
    d_q = torch.from_numpy(Q).to(dev).contiguous()
    d_ids = torch.empty(nq, k, dtype=torch.int64, device=dev)
    d_d = torch.empty(nq, k, dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream(dev)
    ncand = int(np.minimum(Ls, ix.N).sum())

    def timed(h, label):
        for i in range(args.warmup):
            fbpq.fbpq_search_device(h, d_q, Ls, ks, k, d_ids, d_d, stream)
        torch.cuda.synchronize()
        fbpq.fbpq_set_option(h, "profile", 1)
        fbpq.fbpq_set_option(h, "profile_mask", -1)
        for s_ in range(len(fbpq.STAGES)):
            fbpq.fbpq_profile_read(h, s_, reset=True)
        for _ in range(args.profile_steps):
            fbpq.fbpq_search_device(h, d_q, Ls, ks, k, d_ids, d_d, stream)
        torch.cuda.synchronize()
        prof = {}
        for s_, name in enumerate(fbpq.STAGES):
            ms, n = fbpq.fbpq_profile_read(h, s_, reset=True)
            prof[name] = {"ms_per_launch": ms / n if n else None, "launches": n}
        log(f"{label} kernels: " + ", ".join(f"{n}={v['ms_per_launch']:.4f}" for n, v in prof.items()
                                              if v["ms_per_launch"]))
        fbpq.fbpq_set_option(h, "profile_mask", 1 << fbpq.STAGES.index("scan_wide"))
        torch.cuda.synchronize()
        a = time.perf_counter()
        for _ in range(args.steps):
            fbpq.fbpq_search_device(h, d_q, Ls, ks, k, d_ids, d_d, stream)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - a) * 1e3 / args.steps
        sw_ms, sw_n = fbpq.fbpq_profile_read(h, fbpq.STAGES.index("scan_wide"), reset=True)
        fbpq.fbpq_set_option(h, "profile", 0)
        log(f"{label}: {ms:.3f} ms per batch")
        return ms, prof, (sw_ms / sw_n if sw_n else None), sw_n

    h = fbpq.fbpq_index_create(ix, 0)
    fbpq.fbpq_build_tables(h)
    fbpq.fbpq_set_option(h, "stats", 1)
    ms, prof, sw_ms, sw_n = timed(h, "local")
    stats = fbpq.fbpq_stats_read(h)
    log(f"local path counters: {stats}")
    res_ids, res_d = d_ids.cpu().numpy(), d_d.cpu().numpy()
    fbpq.fbpq_free_index(h)
    hg = fbpq.fbpq_index_create(gix, 0)
    fbpq.fbpq_build_tables(hg)
    g_ms, g_prof, _, _ = timed(hg, "global")
    fbpq.fbpq_free_index(hg)

    # the scan with local codebooks: M code bytes per candidate over its time
    achieved = ncand * ix.M / (sw_ms * 1e-3) / 1e9 if sw_ms else None
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBPS if achieved else None, "traffic": None,
            "kernel": "k_scan_wide", "algorithmic_per_launch": ncand * ix.M, "what": "code bytes",
            "ms_per_launch": sw_ms, "launches": sw_n}
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        threads = oracle.host_threads()
        n0 = min(nq, threads)
        a = time.perf_counter()
        o_ids, o_d, _, _ = oracle.search(ix, Q[:n0], Ls[:n0], k, nthreads=threads)
        t_first = time.perf_counter() - a
        n1 = int(min(nq, max(n0, n0 * args.cpu_seconds / max(t_first, 1e-3))))
        if n1 > n0:
            a = time.perf_counter()
            o_ids, o_d, _, _ = oracle.search(ix, Q[:n1], Ls[:n1], k, nthreads=threads)
            t_cpu = time.perf_counter() - a
        else:
            n1, t_cpu = n0, t_first
        overlap = float(np.mean([len(set(res_ids[r]) & set(o_ids[r])) / k for r in range(n1)]))
        rel = np.abs(res_d[:n1].astype(np.float64) - o_d) / np.maximum(o_d, 1.0)
        cpu = {"value": n1 / t_cpu, "unit": "queries/s", "cores": threads, "kind": "oracle",
               "sample": f"first {n1} of the {nq} queries, same index and local codebooks, their own L, k={k}",
               "topk_overlap_with_gpu": overlap, "max_rel_dist_diff": float(rel.max())}
        log(f"cpu oracle: {n1} queries in {t_cpu:.1f}s on {threads} threads")
    out = {
        "metric": "queries/s at fixed L, Recall@10 = oracle, 1 GPU; p50/p99 latency; scan GB/s",
        "value": nq / (ms / 1e3), "unit": "queries/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"local codebooks (HBPQ): N={ix.N}, T={ix.T} per half, M={ix.M}, nq={nq} per batch, "
                               f"L log-uniform in [{w['L_lo']}, {w['L_hi']}], k={k}",
                   "N": ix.N, "T": ix.T, "M": ix.M, "nq": nq, "k": k, "mean_L": float(Ls.mean())},
        "kernels": prof,
        "path_counters": stats,
        "global_codebooks_same_L": {"ms_per_step": g_ms, "value": nq / (g_ms / 1e3), "kernels": g_prof},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))
    return 0


def run_gist(args, w) -> int:
    """The GIST-like width (D = 384, T = 1024, M = 8 bytes of code): FBPQ and the
    Multi-D-ADC O(D) scan on the same index and batch at each L. The FBPQ scan
    costs M lookups per candidate whatever D is, the O(D) scan D/2 multiply-adds
    per half, so the ratio grows with D at fixed M (Section 3.1, Table 2)."""
    import torch

    import synth
    from paper_1404_1831_amd.build import LIB
    if not os.path.exists(LIB):
        from paper_1404_1831_amd.build import build
        build()
    from paper_1404_1831_amd import fbpq

    if args.nq:
        w["nq"] = args.nq
    dev = torch.device("cuda:0")
    t0 = time.time()
    means = synth.gmm_means(0, D=w["D"])
    base = synth.sample_points(w["N"], means, 1, dev)
    ix = synth.build_index(base, w["T"], w["M"], keep_base=False)
    del base
    torch.cuda.empty_cache()
    nq, k = w["nq"], w["k"]
    Q = synth.make_queries(nq, means, 2, dev)
    log(f"index built in {time.time() - t0:.1f}s: N={ix.N} D={ix.D} T={ix.T} M={ix.M} "
        f"nonempty cells={int((np.diff(ix.offsets) > 0).sum())}")
    d_q = torch.from_numpy(Q).to(dev).contiguous()
    d_ids = torch.empty(nq, k, dtype=torch.int64, device=dev)
    d_d = torch.empty(nq, k, dtype=torch.float32, device=dev)
    ks = np.full(nq, k, np.int32)
    stream = torch.cuda.current_stream(dev)
    h = fbpq.fbpq_index_create(ix, 0)
    fbpq.fbpq_build_tables(h)

    def timed(Ls, od):
        fbpq.fbpq_set_option(h, "adc_od", od)
        for _ in range(args.warmup):
            fbpq.fbpq_search_device(h, d_q, Ls, ks, k, d_ids, d_d, stream)
        torch.cuda.synchronize()
        fbpq.fbpq_set_option(h, "profile", 1)
        fbpq.fbpq_set_option(h, "profile_mask", -1)
        for s_ in range(len(fbpq.STAGES)):
            fbpq.fbpq_profile_read(h, s_, reset=True)
        a = time.perf_counter()
        for _ in range(args.steps):
            fbpq.fbpq_search_device(h, d_q, Ls, ks, k, d_ids, d_d, stream)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - a) * 1e3 / args.steps
        prof = {}
        for s_, name in enumerate(fbpq.STAGES):
            t, n = fbpq.fbpq_profile_read(h, s_, reset=True)
            prof[name] = {"ms_per_launch": t / n if n else None, "launches": n}
        fbpq.fbpq_set_option(h, "profile", 0)
        return ms, prof

    legs = []
    first = None
    for L in w["L"]:
        Ls = np.full(nq, L, np.int64)
        f_ms, f_prof = timed(Ls, 0)
        if first is None:
            first = (L, f_ms, f_prof, d_ids.cpu().numpy(), d_d.cpu().numpy())
        o_ms, o_prof = timed(Ls, 1) if args.adc_steps > 0 else (None, None)
        legs.append({"L": L, "fbpq_ms_per_batch": f_ms, "fbpq_queries_per_s": nq / (f_ms / 1e3),
                     "od_ms_per_batch": o_ms, "fbpq_speedup": (o_ms / f_ms) if o_ms else None,
                     "fbpq_kernels": f_prof, "od_kernels": o_prof})
        log(f"L={L}: FBPQ {f_ms:.3f} ms per batch, O(D) " + (f"{o_ms:.3f} ms, {o_ms / f_ms:.1f}x" if o_ms else "skipped"))
    fbpq.fbpq_free_index(h)

    L0, ms0, prof0, res_ids, res_d = first
    # the dominant scan kernel of the FBPQ search at the first L: M code bytes per candidate
    scans = {"score": "k_score_query", "scan_wide": "k_scan_wide", "scan2": "k_scan2"}
    dom = max(scans, key=lambda s_: (prof0[s_]["ms_per_launch"] or 0.0) * (prof0[s_]["launches"] or 0))
    ncand = nq * min(L0, ix.N)
    d_ms = prof0[dom]["ms_per_launch"]
    achieved = ncand * ix.M / (d_ms * 1e-3) / 1e9 if d_ms else None
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBPS if achieved else None, "traffic": None,
            "kernel": scans[dom], "algorithmic_per_launch": ncand * ix.M, "what": "code bytes",
            "ms_per_launch": d_ms, "launches": prof0[dom]["launches"]}
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        threads = oracle.host_threads()
        Ls0 = np.full(nq, L0, np.int64)
        n0 = min(nq, threads)
        a = time.perf_counter()
        o_ids, o_d, _, _ = oracle.search(ix, Q[:n0], Ls0[:n0], k, nthreads=threads)
        t_first = time.perf_counter() - a
        n1 = int(min(nq, max(n0, n0 * args.cpu_seconds / max(t_first, 1e-3))))
        if n1 > n0:
            a = time.perf_counter()
            o_ids, o_d, _, _ = oracle.search(ix, Q[:n1], Ls0[:n1], k, nthreads=threads)
            t_cpu = time.perf_counter() - a
        else:
            n1, t_cpu = n0, t_first
        overlap = float(np.mean([len(set(res_ids[r]) & set(o_ids[r])) / k for r in range(n1)]))
        rel = np.abs(res_d[:n1].astype(np.float64) - o_d) / np.maximum(o_d, 1.0)
        cpu = {"value": n1 / t_cpu, "unit": "queries/s", "cores": threads, "kind": "oracle",
               "sample": f"first {n1} of the {nq} queries, same index, L={L0}, k={k}",
               "topk_overlap_with_gpu": overlap, "max_rel_dist_diff": float(rel.max())}
        log(f"cpu oracle: {n1} queries in {t_cpu:.1f}s on {threads} threads")
    out = {
        "metric": "queries/s at fixed L, Recall@10 = oracle, 1 GPU; p50/p99 latency; scan GB/s",
        "value": nq / (ms0 / 1e3), "unit": "queries/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms0, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"GIST-like FBPQ: N={ix.N}, D={ix.D}, T={ix.T} per half, M={ix.M}, "
                               f"nq={nq} per batch, L={L0} (and {', '.join(str(x) for x in w['L'][1:])} "
                               f"in legs), k={k}",
                   "N": ix.N, "D": ix.D, "T": ix.T, "M": ix.M, "nq": nq, "k": k},
        "legs": legs,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))
    return 0


def run_served(args, w) -> int:
    """Continuous batching under Poisson arrivals: per offered load, the achieved
    rate and the latency from submit to result on the host (p50, p99)."""
    import threading

    import torch

    import synth
    from paper_1404_1831_amd.build import LIB
    if not os.path.exists(LIB):
        from paper_1404_1831_amd.build import build
        build()
    from paper_1404_1831_amd import fbpq

    N = args.served_n or w["N"]
    dev = torch.device("cuda:0")
    t0 = time.time()
    ix = synth.zipf_index(N, w["T"], w["M"], device=dev)
    torch.cuda.empty_cache()
    cnt = np.diff(ix.offsets)
    log(f"zipf index built in {time.time() - t0:.1f}s: N={ix.N} T={ix.T} M={ix.M} "
        f"largest cell={int(cnt.max())} nonempty={float((cnt > 0).mean()):.3f}")
    h = fbpq.fbpq_index_create(ix, 0)
    fbpq.fbpq_build_tables(h)
    means = synth.gmm_means(0)
    k, Ls = w["k"], np.asarray(w["L"], np.int64)
    rng = np.random.default_rng(4)
    # one direct batch first: the same search the lanes run
    Qc = synth.make_queries(64, means, 3)
    a = time.perf_counter()
    try:
        fbpq.fbpq_search_uneven(h, Qc, np.full(64, int(Ls.max()), np.int64), np.full(64, k, np.int32), k)
        msg = "all served"
    except fbpq.FbpqError as e:
        if e.code != fbpq.FBPQ_E_CAPACITY:
            raise
        msg = str(e)
    log(f"direct batch of 64 at L={int(Ls.max())}: {(time.perf_counter() - a) * 1e3:.1f} ms ({msg})")
    rows = []
    for rate in w["offered"]:
        nreq = int(rate * args.served_seconds)
        Q = synth.make_queries(nreq, means, 2)
        L = Ls[rng.integers(0, len(Ls), nreq)]
        gaps = rng.exponential(1.0 / rate, nreq)
        s = fbpq.fbpq_server_create(h, args.served_batch, args.served_lanes, k)
        lat, done_t, nfail = [], [], 0

        def submit():
            t = time.perf_counter()
            for i in range(nreq):
                t += gaps[i]
                dt = t - time.perf_counter()
                if dt > 0:
                    time.sleep(dt)
                fbpq.fbpq_server_submit(s, Q[i], int(L[i]), k, i)

        th = threading.Thread(target=submit)
        a = time.perf_counter()
        th.start()
        got = 0
        while got < nreq:
            tags, ids, d, times, st = fbpq.fbpq_server_poll(s, 4096, k, wait_s=0.05)
            got += len(tags)
            ok = st == 0
            nfail += int((~ok).sum())
            lat.extend((times[ok, 2] - times[ok, 0]).tolist())
            if len(tags):
                done_t.append(time.perf_counter())
            if time.perf_counter() - a > args.served_seconds * 20 + 60:
                break
        th.join()
        elapsed = (done_t[-1] if done_t else time.perf_counter()) - a
        _, batches, batched = fbpq.fbpq_server_counts(s)
        err = fbpq.fbpq_server_first_error(s)
        fbpq.fbpq_server_destroy(s)
        if nfail:
            log(f"offered {rate}/s: {nfail} requests failed: {err}")
        lat_ms = np.asarray(lat) * 1e3
        row = {"offered_qps": rate, "requests": nreq, "completed": got - nfail, "failed": nfail,
               "achieved_qps": (got - nfail) / elapsed,
               "p50_ms": float(np.percentile(lat_ms, 50)), "p99_ms": float(np.percentile(lat_ms, 99)),
               "mean_batch": batched / max(1, batches)}
        rows.append(row)
        log(f"offered {rate}/s: achieved {row['achieved_qps']:.0f}/s p50 {row['p50_ms']:.2f} ms "
            f"p99 {row['p99_ms']:.2f} ms mean batch {row['mean_batch']:.1f}")
    fbpq.fbpq_free_index(h)
    best = max(rows, key=lambda r: r["achieved_qps"])
    out = {
        "metric": "served queries: achieved rate and p50/p99 latency vs offered load, 1 GPU",
        "value": best["achieved_qps"], "unit": "queries/s", "n_gpus": 1, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"served FBPQ: N={ix.N} with Zipf(1.1) cell sizes, T={ix.T} per half, "
                               f"M={ix.M}, L in {Ls.tolist()}, k={k}, {args.served_lanes} lanes, "
                               f"batches of at most {args.served_batch}"},
        "served": rows,
    }
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
