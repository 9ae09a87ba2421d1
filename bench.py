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
FP16_MFMA_TFLOPS = 2500.0  # dense

WORKLOADS = {
    "batched": dict(N=10_000_000, T=4096, M=16, nq=10_000, L=10_000, k=100),
    "plain": dict(N=100_000, T=64, M=8, nq=100, L=10_000, k=10),
    # uneven batch: per-query L log-uniform in [L_lo, L_hi], k drawn from ks
    "uneven": dict(N=100_000_000, T=16384, M=8, nq=20_000, L_lo=1_000, L_hi=100_000, ks=(1, 10, 100)),
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


def host_facts() -> dict:
    """The host the CPU baseline runs on: core counts and CPU model."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        aff = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        aff = None
    return {"nproc": os.cpu_count(), "affinity_cores": aff, "cpu_model": model}


def roofline_models(ix, nq: int, k_max: int, ncand: int, cand: dict, split_keys: bool = True) -> dict:
    """Algorithmic work per launch of the kernels a roofline is reported for.

    score, scan_wide, scan2: M code bytes per candidate the kernel scores (the
               scan's HBM stream; candidates per kernel from the path counters)
    select:    the 4-byte distance of every candidate, plus k (id, distance) results per query
    prefix:    the 4-byte approximate key of every (query, half, centroid), plus P (key, index) outputs
    half_keys: 2 (D/2) FLOP per (query, half, centroid): on the FP32 matrix
               cores, or three times that on the FP16 ones in the split form
               (D/2 = 64 and split_keys)
    """
    P = 128
    csrc = os.path.join(ROOT, "paper_1404_1831_amd", "csrc")
    gbs = dict(bound="hbm", peak=HBM_PEAK_GBPS, unit="GB/s", scale=1e9)
    return {
        "score": dict(gbs, kernel="k_score_query", amount=cand.get("score", ncand) * ix.M, what="code bytes",
                      source=os.path.join(csrc, "k_items.hip")),
        "scan_wide": dict(gbs, kernel="k_scan_wide", amount=cand.get("scan_wide", 0) * ix.M, what="code bytes",
                          source=os.path.join(csrc, "k_scan.hip")),
        "scan2": dict(gbs, kernel="k_scan2", amount=cand.get("scan2", 0) * ix.M, what="code bytes",
                      source=os.path.join(csrc, "k_scan.hip")),
        "select": dict(gbs, kernel="k_select_dist", amount=ncand * 4 + nq * k_max * 12,
                       what="distance and result bytes", source=os.path.join(csrc, "k_items.hip")),
        "prefix": dict(gbs, kernel="k_prefix_wave", amount=nq * 2 * ix.T * 4 + nq * 2 * P * 12,
                       what="approximate-key and prefix bytes", source=os.path.join(csrc, "k_rank.hip")),
        "half_keys": (dict(bound="mfma", peak=FP16_MFMA_TFLOPS, unit="TFLOP/s", scale=1e12, kernel="k_half_approx",
                           amount=3 * nq * 2 * ix.T * (ix.D // 2) * 2,
                           what="FP16 matrix-core FLOP (three products of the split form)",
                           source=os.path.join(csrc, "k_rank.hip"))
                      if split_keys and ix.D // 2 == 64 else
                      dict(bound="mfma", peak=FP32_MFMA_TFLOPS, unit="TFLOP/s", scale=1e12, kernel="k_half_approx",
                           amount=nq * 2 * ix.T * (ix.D // 2) * 2, what="FP32 matrix-core FLOP",
                           source=os.path.join(csrc, "k_rank.hip"))),
    }


def scan_roof(model: dict, ms: float, peaks: dict):
    """The scan roof of a code-scanning kernel as the survey defines it: the
    larger of its code bytes at the HBM peak and its table lookups (one 4-byte
    LDS read per code byte, the tables folded) at the measured LDS gather rate,
    and the fraction roof / measured time."""
    if not ms or model.get("what") != "code bytes" or not peaks.get("lds_gather_lookups_per_s"):
        return None
    hbm_ms = model["amount"] / (HBM_PEAK_GBPS * 1e9) * 1e3
    lds_ms = model["amount"] / peaks["lds_gather_lookups_per_s"] * 1e3
    roof = max(hbm_ms, lds_ms)
    return {"kernel": model["kernel"], "hbm_ms": hbm_ms, "lds_ms": lds_ms, "roof_ms": roof, "measured_ms": ms,
            "frac": roof / ms, "lds_rate_lookups_per_s": peaks["lds_gather_lookups_per_s"],
            "definition": "max(code bytes / 8 TB/s, lookups / measured LDS gather rate) / kernel time"}


def traffic_from_profile(kernel: str, source: str, workload: str):
    """HBM bytes per launch from the committed counter summary of this kernel
    on this workload, if the kernel's source file is unchanged since the
    counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    with open(source, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    if rec.get("source_sha256") != sha or rec.get("workload") != workload:
        return None
    return rec.get("hbm_bytes_per_launch")


def exact_nn(base, Q, chunk: int = 1 << 20):
    """Index of the nearest base point of every query (FP64 squared distance,
    ties to the lower index): FP32 distances on the GPU shortlist 32 points
    per query, FP64 decides among them."""
    import torch
    dev = base.device
    q = torch.from_numpy(np.ascontiguousarray(Q, np.float32)).to(dev)
    qn = (q * q).sum(1, keepdim=True)
    best_d = torch.full((q.shape[0], 32), float("inf"), device=dev)
    best_i = torch.zeros((q.shape[0], 32), dtype=torch.int64, device=dev)
    for s in range(0, base.shape[0], chunk):
        x = base[s:s + chunk].to(torch.float32)
        d = qn - 2.0 * (q @ x.T) + (x * x).sum(1)[None, :]
        v, i = torch.topk(d, min(32, d.shape[1]), dim=1, largest=False)
        cd = torch.cat([best_d, v], 1)
        ci = torch.cat([best_i, i + s], 1)
        o = torch.argsort(cd, dim=1)[:, :32]
        best_d, best_i = torch.gather(cd, 1, o), torch.gather(ci, 1, o)
    cand = best_i.cpu().numpy()
    pts = base[best_i.reshape(-1)].cpu().numpy().astype(np.float64).reshape(cand.shape[0], cand.shape[1], -1)
    d64 = ((pts - np.asarray(Q, np.float64)[:, None, :]) ** 2).sum(2)
    order = np.lexsort((cand, d64), axis=1)[:, 0]
    return cand[np.arange(cand.shape[0]), order]


def recall_at(ids: np.ndarray, nn: np.ndarray, R: int) -> float:
    """Recall@R of the paper: the fraction of queries whose nearest neighbour
    is among the first R results."""
    return float(np.mean([nn[r] in ids[r, :R] for r in range(len(nn))]))


def cpu_baseline(ix, Q, Ls, ks, k_max, res_ids, res_d, seconds: float, what: str, nn=None) -> dict:
    """The FP64 oracle timed on the host: all its threads on a sample sized to
    about `seconds`, then one thread on a few queries (per-query time)."""
    import oracle
    threads = oracle.host_threads()
    nq = Q.shape[0]
    n0 = min(nq, 2 * threads)
    a = time.perf_counter()
    oracle.search(ix, Q[:n0], Ls[:n0], ks[:n0], kmax=k_max, nthreads=threads)
    t_first = time.perf_counter() - a
    n1 = int(min(nq, max(n0, n0 * seconds / max(t_first, 1e-3))))
    a = time.perf_counter()
    o_ids, o_d, _, _ = oracle.search(ix, Q[:n1], Ls[:n1], ks[:n1], kmax=k_max, nthreads=threads)
    t_cpu = time.perf_counter() - a
    n_st = max(1, min(nq, int(n1 / threads / 4)))
    a = time.perf_counter()
    oracle.search(ix, Q[:n_st], Ls[:n_st], ks[:n_st], kmax=k_max, nthreads=1)
    t_st = time.perf_counter() - a
    ov = [len(set(res_ids[r, :ks[r]]) & set(o_ids[r, :ks[r]])) / ks[r] for r in range(n1)]
    kk = np.arange(k_max)[None, :] < ks[:n1, None]
    rel = np.abs(res_d[:n1].astype(np.float64) - o_d)[kk] / np.maximum(o_d[kk], 1.0)
    out = {"value": n1 / t_cpu, "unit": "queries/s", "cores": threads, "kind": "oracle",
           "sample": f"first {n1} of the {nq} queries, {what}",
           "single_thread_ms_per_query": t_st * 1e3 / n_st, "single_thread_queries": n_st,
           "topk_overlap_with_gpu": float(np.mean(ov)), "max_rel_dist_diff": float(rel.max())}
    out.update(host_facts())
    if nn is not None:
        m = min(n1, len(nn))
        sel = ks[:m] >= 10
        if sel.any():
            out["recall_at_10_oracle"] = recall_at(o_ids[:m][sel], nn[:m][sel], 10)
            out["recall_at_10_gpu_same_queries"] = recall_at(res_ids[:m][sel], nn[:m][sel], 10)
    log(f"cpu oracle: {n1} queries in {t_cpu:.1f}s on {threads} threads; one thread {out['single_thread_ms_per_query']:.2f} ms/query")
    return out


def hbm_copy_peak(dev, mib: int = 2048, reps: int = 5) -> float:
    """Bytes read plus written per second by a device-to-device tensor copy."""
    import torch
    x = torch.ones(mib << 18, dtype=torch.float32, device=dev)
    y = torch.empty_like(x)
    y.copy_(x)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        y.copy_(x)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del x, y
    return 2 * (mib << 20) / (ms * 1e-3) / 1e9


def served_ladder(fbpq, h, Q, Ls, k: int, rates, seconds: float, lanes: int, batch: int, check=None) -> list:
    """Poisson arrivals at each offered rate through a server on handle h. Per
    rate: achieved rate, p50 / p99 of submit-to-result latency over all
    requests (a failed request counts at its completion time) and over the
    successful ones, failures. check(tags, ids, dists) sees the results."""
    import threading
    rng = np.random.default_rng(4)
    rows = []
    for rate in rates:
        nreq = max(1, int(rate * seconds))
        qi = rng.integers(0, Q.shape[0], nreq)
        L = Ls[rng.integers(0, len(Ls), nreq)]
        gaps = rng.exponential(1.0 / rate, nreq)
        s = fbpq.fbpq_server_create2(h, batch, lanes, k)
        refused = []

        def submit():
            t = time.perf_counter()
            for i in range(nreq):
                t += gaps[i]
                dt = t - time.perf_counter()
                if dt > 0:
                    time.sleep(dt)
                if fbpq.fbpq_server_submit(s, Q[qi[i]], int(L[i]), k, i) != fbpq.FBPQ_OK:
                    refused.append(i)

        th = threading.Thread(target=submit)
        a = time.perf_counter()
        th.start()
        lat_all, lat_ok, nfail, got, done_t = [], [], 0, 0, a
        tags_all, ids_all, d_all = [], [], []
        while True:
            tags, ids, d, times, st = fbpq.fbpq_server_poll(s, 4096, k, wait_s=0.05)
            got += len(tags)
            if len(tags):
                done_t = time.perf_counter()
                lat = (times[:, 2] - times[:, 0]) * 1e3
                lat_all.extend(lat.tolist())
                lat_ok.extend(lat[st == 0].tolist())
                nfail += int((st != 0).sum())
                if check is not None:
                    tags_all.append(tags.copy())
                    ids_all.append(ids.copy())
                    d_all.append(d.copy())
            if not th.is_alive() and got + len(refused) >= nreq:
                break
            if time.perf_counter() - a > seconds * 20 + 60:
                break
        th.join()
        stats = fbpq.fbpq_server_stats(s)
        err = fbpq.fbpq_server_first_error(s)
        fbpq.fbpq_server_destroy(s)
        if nfail:
            log(f"offered {rate}/s: {nfail} requests failed: {err}")
        row = {"offered_qps": rate, "requests": nreq, "completed": got - nfail, "failed": nfail,
               "refused": len(refused), "achieved_qps": (got - nfail) / max(done_t - a, 1e-9),
               "p50_ms": float(np.percentile(lat_all, 50)) if lat_all else None,
               "p99_ms": float(np.percentile(lat_all, 99)) if lat_all else None,
               "p99_ms_successful": float(np.percentile(lat_ok, 99)) if lat_ok else None,
               "mean_batch": stats["batched"] / max(1, stats["batches"]),
               "peak_reserved_bytes": stats["peak_reserved"]}
        if check is not None and tags_all:
            row["oracle_check"] = check(np.concatenate(tags_all), np.concatenate(ids_all), np.concatenate(d_all),
                                        qi, L)
        rows.append(row)
        log(f"offered {rate}/s: achieved {row['achieved_qps']:.0f}/s p50 {row['p50_ms']:.2f} ms "
            f"p99 {row['p99_ms']:.2f} ms mean batch {row['mean_batch']:.1f} failed {nfail}")
    return rows


def oracle_checker(ix, Q, k: int, n_check: int):
    """check() for served_ladder: the oracle on n_check requests sampled from
    those that completed; a request matches when its distances agree with the
    oracle's within 1e-4 relative and its ids are the oracle's but where
    distances tie within that tolerance at the k-th place."""
    import oracle

    def check(tags, ids, d, qi, L):
        rng = np.random.default_rng(11)
        ok_rows = np.nonzero(ids[:, 0] != -2)[0]
        pick = rng.choice(ok_rows, size=min(n_check, len(ok_rows)), replace=False) if len(ok_rows) else []
        if len(pick) == 0:
            return {"checked": 0, "matched": 0}
        t = tags[pick]
        o_ids, o_d, _, _ = oracle.search(ix, Q[qi[t]], L[t], k, nthreads=oracle.host_threads())
        matched, worst = 0, []
        for r, p in enumerate(pick):
            q = Q[qi[t[r]]].astype(np.float64)
            # |d32 - d64| <= 1e-4 d64 + 1e-6 (|q|^2 + |x|^2), with |x| <= |q| + sqrt(d64)
            tol = 1e-4 * o_d[r] + 1e-6 * (q @ q + (np.sqrt(q @ q) + np.sqrt(np.maximum(o_d[r], 0))) ** 2)
            g_d = d[p].astype(np.float64)
            good = bool(np.all(np.abs(g_d - o_d[r]) <= tol))
            firm = o_d[r] < o_d[r][k - 1] - 2 * tol[k - 1]  # not tied with the k-th within tolerance
            good = good and set(o_ids[r][firm].tolist()) <= set(ids[p].tolist())
            matched += int(good)
            if not good:
                worst.append({"tag": int(t[r]), "L": int(L[t[r]]),
                              "max_abs_diff": float(np.max(np.abs(g_d - o_d[r]))),
                              "ids_missing": sorted(set(o_ids[r][firm].tolist()) - set(ids[p].tolist()))[:5]})
        return {"checked": int(len(pick)), "matched": matched, "mismatches": worst[:5]}
    return check


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="batched", choices=sorted(WORKLOADS))
    ap.add_argument("--nq", type=int, default=None)
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target duration of the CPU oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--recall-queries", type=int, default=1000,
                    help="queries whose exact nearest neighbour is found by brute force, for Recall@10")
    ap.add_argument("--served-n", type=int, default=0, help="served workload: points (default 1e9)")
    ap.add_argument("--served-seconds", type=float, default=2.0, help="served workload: seconds per offered load")
    ap.add_argument("--served-lanes", type=int, default=4)
    ap.add_argument("--served-batch", type=int, default=512)
    ap.add_argument("--served-check", type=int, default=200,
                    help="served requests checked against the oracle per offered load")
    ap.add_argument("--served-rates", default="2000,10000",
                    help="batched workload: offered loads of the short served leg on the same index ('' to skip)")
    ap.add_argument("--plain-queries", type=int, default=200,
                    help="queries searched one launch sequence at a time, for the per-query comparison")
    ap.add_argument("--adc-steps", type=int, default=3,
                    help="batches searched with the O(D) Multi-D-ADC rerank, for the comparison (0: skip)")
    ap.add_argument("--profile-steps", type=int, default=3,
                    help="untimed steps with every kernel timed, for the per-kernel breakdown")
    ap.add_argument("--tune-cache", default=os.path.join(ROOT, "paper_1404_1831_amd", "tune_cache.jsonl"),
                    help="autotuner cache (JSON lines); '' to keep the library defaults")
    ap.add_argument("--option", action="append", default=[],
                    help="library option key=value set on the search handle (repeatable)")
    ap.add_argument("--no-uneven", action="store_true",
                    help="batched workload: skip the uneven-batch leg (N=1e8, T=16384, per-query L and k)")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="also run a plain elementwise copy of this many MiB (read once, written once), "
                         "the reference dispatch for scaling HBM traffic counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this search runs on one GPU; --gpus above 1 is not supported"}))
        return 2

    from paper_1404_1831_amd.build import LIB
    if not os.path.exists(LIB):
        from paper_1404_1831_amd.build import build
        build()

    w = dict(WORKLOADS[args.workload])
    if args.workload == "served":
        return run_served(args, w)
    if args.workload == "local":
        return run_local(args, w)
    if args.workload == "gist":
        return run_gist(args, w)
    out = run_batch(args, w)
    if args.workload == "batched" and not args.no_uneven:
        # the uneven-batch configuration in the same run, with its own
        # roofline, oracle sample and recall (no served, O(D) or plain legs)
        import copy
        import gc
        gc.collect()
        a2 = copy.copy(args)
        a2.workload, a2.nq, a2.plain_queries, a2.adc_steps, a2.served_rates = "uneven", None, 0, 0, ""
        a2.recall_queries = min(args.recall_queries, 500)
        a2.cpu_seconds = min(args.cpu_seconds, 8.0)
        a2.calibrate_copy_mib = 0
        u = run_batch(a2, dict(WORKLOADS["uneven"]))
        out["uneven_workload"] = {key: u[key] for key in (
            "value", "unit", "ms_per_step", "p50_ms", "p99_ms", "step_ms", "config", "kernels", "path_counters",
            "recall", "autotune", "graph_replay", "scan_roof", "roofline", "cpu_baseline")}
    print(json.dumps(out))
    return 0


def run_batch(args, w) -> dict:
    """One batch searched as a whole (batched, uneven and plain workloads);
    returns the result line."""
    import torch

    import synth
    from paper_1404_1831_amd import fbpq

    if args.nq:
        w["nq"] = args.nq
    dev = torch.device("cuda:0")
    t0 = time.time()
    means = synth.gmm_means(0)
    base = synth.sample_points(w["N"], means, 1, dev)
    ix = synth.build_index(base, w["T"], w["M"], keep_base=False)
    nq = w["nq"]
    Q = synth.make_queries(nq, means, 2, dev)
    if "L" in w:
        Ls = np.full(nq, w["L"], np.int64)
        ks = np.full(nq, w["k"], np.int32)
        k = w["k"]
        lk_desc = f"L={w['L']}, k={k}"
    else:
        Ls, ks = synth.draw_L_k(nq, 3, w["L_lo"], w["L_hi"], w["ks"])
        Ls = np.ascontiguousarray(Ls, np.int64)
        ks = np.ascontiguousarray(ks, np.int32)
        k = int(max(w["ks"]))
        lk_desc = (f"L log-uniform in [{w['L_lo']}, {w['L_hi']}] (mean {Ls.mean():.0f}), "
                   f"k drawn from {list(w['ks'])}")
    torch.cuda.synchronize()
    log(f"index built in {time.time() - t0:.1f}s: N={ix.N} T={ix.T} M={ix.M} "
        f"nonempty cells={int((np.diff(ix.offsets) > 0).sum())}; {lk_desc}")

    h = fbpq.fbpq_index_create(ix, 0)
    fbpq.fbpq_build_tables(h)
    for kv in args.option:
        key, val = kv.split("=")
        fbpq.fbpq_set_option(h, key, int(val))
    d_q = torch.from_numpy(Q).to(dev).contiguous()
    d_ids = torch.empty(nq, k, dtype=torch.int64, device=dev)
    d_d = torch.empty(nq, k, dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream(dev)

    def search():
        fbpq.fbpq_search_device(h, d_q, Ls, ks, k, d_ids, d_d, stream)

    tune = None
    if args.tune_cache:
        # the autotuner's setting for this geometry, batch and device (tuned
        # once and kept in the cache file)
        a = time.perf_counter()
        tune = fbpq.fbpq_autotune_cached(h, d_q, Ls, ks, k, d_ids, d_d, stream, args.tune_cache, reps=3)
        log(f"autotuner ({'cached' if tune['from_cache'] else 'tuned'} in {time.perf_counter() - a:.1f}s): {tune}")
    for kv in args.option:  # explicit options override the tuned ones
        key, val = kv.split("=")
        fbpq.fbpq_set_option(h, key, int(val))

    # path counters (untimed steps of their own: their atomics would slow the kernels)
    fbpq.fbpq_set_option(h, "stats", 1)
    for _ in range(args.profile_steps):
        search()
    torch.cuda.synchronize()
    stats = fbpq.fbpq_stats_read(h)
    fbpq.fbpq_set_option(h, "stats", 0)
    # per-kernel breakdown (untimed): HIP events around every launch
    fbpq.fbpq_set_option(h, "profile", 1)
    fbpq.fbpq_set_option(h, "profile_mask", -1)
    for s in range(len(fbpq.STAGES)):
        fbpq.fbpq_profile_read(h, s, reset=True)
    for _ in range(args.profile_steps):
        search()
    torch.cuda.synchronize()
    prof = {}
    for s, name in enumerate(fbpq.STAGES):
        ms, n = fbpq.fbpq_profile_read(h, s, reset=True)
        prof[name] = {"ms_per_launch": ms / n if n else None, "launches": n}
    log("kernels: " + ", ".join(f"{n}={v['ms_per_launch']:.4f}" for n, v in prof.items() if v["ms_per_launch"]))
    log(f"path counters over {args.profile_steps} steps: {stats}")

    # the dominant kernel among those with a roofline model (total time per step)
    ncand = int(np.minimum(Ls, ix.N).sum())
    per = max(1, args.profile_steps)
    cand = {"score": stats.get("cand_cell_scan", ncand * per) // per,
            "scan_wide": stats.get("cand_wide", 0) // per, "scan2": stats.get("cand_two_pass", 0) // per}
    split = not any(kv.replace(" ", "") == "split_keys=0" for kv in args.option)
    models = roofline_models(ix, nq, k, ncand, cand, split)

    def total(s):
        p = prof[s]
        return (p["ms_per_launch"] or 0.0) * (p["launches"] or 0)

    dom = max(models, key=total)
    fbpq.fbpq_set_option(h, "profile_mask", 1 << fbpq.STAGES.index(dom))

    # no interpreter garbage collection from here to the end of the timed
    # steps: a collection pause between two launches idles the stream
    import gc
    gc.collect()
    gc.disable()
    # the warmup steps right before the timed ones, in their configuration
    # (the clocks fall while the host reads the counters and profiles)
    for i in range(args.warmup):
        search()
        torch.cuda.synchronize()
    log(f"{args.warmup} warmup steps done")
    fbpq.fbpq_profile_read(h, fbpq.STAGES.index(dom), reset=True)

    step_ms = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        a = time.perf_counter()
        search()
        torch.cuda.synchronize()
        step_ms.append((time.perf_counter() - a) * 1e3)
    torch.cuda.synchronize()
    total_s = time.perf_counter() - t_start
    gc.enable()
    log(f"timed {args.steps} steps in {total_s:.3f}s: " + ", ".join(f"{x:.3f}" for x in step_ms) + " ms")
    dom_ms, dom_n = fbpq.fbpq_profile_read(h, fbpq.STAGES.index(dom), reset=True)
    fbpq.fbpq_set_option(h, "profile", 0)
    dom_ms = dom_ms / dom_n if dom_n else None
    res_ids = d_ids.cpu().numpy()
    res_d = d_d.cpu().numpy()

    # the same batch with the first round replayed from a captured HIP graph
    fbpq.fbpq_set_option(h, "graph", 1)
    for _ in range(2):  # the first call captures
        search()
    torch.cuda.synchronize()
    a = time.perf_counter()
    for _ in range(args.steps):
        search()
        torch.cuda.synchronize()
    graph_ms = (time.perf_counter() - a) * 1e3 / args.steps
    fbpq.fbpq_set_option(h, "graph", 0)
    log(f"graph replays: {graph_ms:.3f} ms per batch")

    # the per-query cell scan (one launch stage per query) in place of the
    # persistent work-queue scan, all else equal
    stage_ms = None
    if tune and tune["persist"]:
        fbpq.fbpq_set_option(h, "persist", 0)
        search()
        torch.cuda.synchronize()
        a = time.perf_counter()
        for _ in range(args.steps):
            search()
            torch.cuda.synchronize()
        stage_ms = (time.perf_counter() - a) * 1e3 / args.steps
        fbpq.fbpq_set_option(h, "persist", 1)
        log(f"per-query cell scan instead of the persistent scan: {stage_ms:.3f} ms per batch")

    # plain per-query launches at equal L and k, on the first queries of the batch
    npl = min(nq, args.plain_queries)
    for i in range(min(npl, 5)):
        fbpq.fbpq_search_device(h, d_q[i:i + 1], Ls[i:i + 1], ks[i:i + 1], k, d_ids[i:i + 1], d_d[i:i + 1], stream)
    torch.cuda.synchronize()
    a = time.perf_counter()
    for i in range(npl):
        fbpq.fbpq_search_device(h, d_q[i:i + 1], Ls[i:i + 1], ks[i:i + 1], k, d_ids[i:i + 1], d_d[i:i + 1], stream)
    torch.cuda.synchronize()
    plain_s = time.perf_counter() - a
    log(f"plain per-query launches: {npl} queries in {plain_s:.3f}s")

    # exact nearest neighbours of the first queries (brute force on the GPU),
    # for Recall@10: after the timed legs, so that neither this work nor the
    # release of its buffers and of the base points comes just before them
    nr = min(nq, args.recall_queries)
    a = time.perf_counter()
    nn = exact_nn(base, Q[:nr]) if nr > 0 else None
    log(f"exact nearest neighbours of {nr} queries in {time.perf_counter() - a:.1f}s")
    del base
    torch.cuda.empty_cache()

    ms_per_step = total_s * 1e3 / args.steps
    qps = nq / (ms_per_step / 1e3)
    model = models[dom]
    achieved = model["amount"] / (dom_ms * 1e-3) / model["scale"] if dom_ms else None
    roof = {"bound": model["bound"], "achieved": achieved, "peak": model["peak"], "unit": model["unit"],
            "frac": achieved / model["peak"] if achieved else None,
            "traffic": traffic_from_profile(model["kernel"], model["source"], args.workload),
            "kernel": model["kernel"], "algorithmic_per_launch": model["amount"], "what": model["what"],
            "ms_per_launch": dom_ms, "launches": dom_n}
    scan_ms = sum(total(s) for s in ("score", "scan_wide", "scan2", "select")) / per
    scan_GBps = ncand * ix.M / (scan_ms * 1e-3) / 1e9 if scan_ms else None

    sel10 = ks[:nr] >= 10
    recall = {"queries": int(sel10.sum()), "recall_at_10": recall_at(res_ids[:nr][sel10], nn[sel10], 10)
              if nr and sel10.any() else None,
              "recall_at_1": recall_at(res_ids[:nr], nn, 1) if nr else None,
              "definition": "fraction of queries whose exact nearest neighbour (FP64, brute force over the "
                            "base points) is among the first R results; queries with k >= 10"}

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(ix, Q, Ls, ks, k, res_ids, res_d, args.cpu_seconds,
                           f"same index, their own L and k ({lk_desc})", nn)

    served = None
    if args.workload == "batched" and args.served_rates:
        rates = [int(x) for x in args.served_rates.split(",") if x]
        served = served_ladder(fbpq, h, Q, Ls[:1], k, rates, 1.0, args.served_lanes, args.served_batch)

    # the Multi-D-ADC baseline on the GPU: the same search with every candidate
    # scored by explicit O(D) reconstruction instead of the FBPQ tables
    adc = None
    if args.adc_steps > 0 and args.workload == "batched":
        fbpq.fbpq_set_option(h, "adc_od", 1)
        for _ in range(2):
            search()
        torch.cuda.synchronize()
        a = time.perf_counter()
        for _ in range(args.adc_steps):
            search()
        torch.cuda.synchronize()
        adc_ms = (time.perf_counter() - a) * 1e3 / args.adc_steps
        fbpq.fbpq_set_option(h, "adc_od", 0)
        adc = {"ms_per_step": adc_ms, "value": nq / (adc_ms / 1e3), "fbpq_speedup": adc_ms / ms_per_step}
        log(f"Multi-D-ADC O(D) baseline: {adc_ms:.3f} ms per batch (FBPQ {ms_per_step:.3f} ms)")

    # OPQ: the same index declared to live in a rotated space, searched with the
    # batch expressed in the original space (Rot^T q), so the rotation kernel
    # maps it back: the cost of the query rotation inside a full search
    opq = None
    if args.adc_steps > 0 and args.workload == "batched":
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

    peaks = {"hbm_copy_GBps": hbm_copy_peak(dev)}
    if hasattr(fbpq, "fbpq_probe_lds_gather"):
        peaks["lds_gather_lookups_per_s"] = fbpq.fbpq_probe_lds_gather(0)
    log(f"measured peaks: {peaks}")
    sroof = scan_roof(model, dom_ms, peaks)
    if sroof:
        log(f"scan roof: {sroof}")

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
        "step_ms": step_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload} FBPQ: N={ix.N}, T={ix.T} per half, M={ix.M}, "
                               f"nq={nq} per batch, {lk_desc}",
                   "N": ix.N, "T": ix.T, "M": ix.M, "nq": nq, "k_max": k, "mean_L": float(Ls.mean()),
                   "options": args.option},
        "kernels": prof,
        "path_counters": stats,
        "recall": recall,
        "autotune": tune,
        "per_query_scan_launch": ({"ms_per_step": stage_ms, "value": nq / (stage_ms / 1e3)} if stage_ms else None),
        "graph_replay": {"ms_per_step": graph_ms, "value": nq / (graph_ms / 1e3)},
        "multi_d_adc_baseline": adc,
        "opq_rotation": opq,
        "plain_per_query": ({"queries": npl, "value": npl / plain_s, "unit": "queries/s",
                             "ms_per_query": plain_s * 1e3 / npl} if npl > 0 else None),
        "served_same_index": served,
        "scan_GBps": scan_GBps,
        "measured_peaks": peaks,
        "scan_roof": sroof,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    return out


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
    rate and the latency from submit to result on the host (p50, p99), with
    sampled requests checked against the oracle."""
    import torch

    import synth
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
    # one direct batch first: the same search the lanes run
    Qc = synth.make_queries(64, means, 3)
    a = time.perf_counter()
    rc = fbpq.fbpq_search_uneven_rc(h, Qc, np.full(64, int(Ls.max()), np.int64), np.full(64, k, np.int32), k)[0]
    log(f"direct batch of 64 at L={int(Ls.max())}: {(time.perf_counter() - a) * 1e3:.1f} ms (code {rc})")
    nmax = int(max(w["offered"]) * args.served_seconds)
    Q = synth.make_queries(nmax, means, 2)
    check = oracle_checker(ix, Q, k, args.served_check) if args.served_check > 0 else None
    rows = served_ladder(fbpq, h, Q, Ls, k, w["offered"], args.served_seconds, args.served_lanes,
                         args.served_batch, check)
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
