#!/usr/bin/env python
"""Benchmark of the Hilbert-forest hot path on one MI355X.

Default workload ("search-23Mx384"): 23,000,000 x 384 fp16 points of a seeded
8,192-component Gaussian mixture on the sphere, 10,000 queries from the same
mixture, a forest of 1,280 trees with leaves of at most 100 points, 512-bit SRP
sketches, k1 = 70, k2 = 1000, h = 0, k = 30 by inner product with an FP32
rerank (the shape of the paper's Task 1; the budget is the cheapest found at
recall@30 >= 0.7 on this data).  One step = one hf_search call over the whole query batch
(descent of every tree, Hamming filter, expansion, rerank); the forest is
built once before timing, as the paper reports index construction apart
from search.  The JSON line reports QPS, recall@30 against an exact GPU brute
force, the roofline of the dominant kernel (HIP events on the library's
stream over the timed region), the exact brute force it is measured against
(timed once, with the FP16-MFMA ceiling of a brute force) and the CPU oracle
timed on a bounded sample.

--peaks runs the standalone ceiling probes (copy, random gathers of 64-, 128-
and 768-byte records, fp16 MFMA) and prints their results as one JSON line.

"graph-3Mx384" times hf_knn_graph (Algorithm 2) on the 3M x 384 mixture.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# The paper's trade-off tables (Section 3.2 Table 1: n, k1, k2, h, recall@30,
# seconds for 10,000 queries; Section 4.2 Table 2: seconds, recall@15, n, k1,
# k2), re-run on the synthetic stand-ins with the same parameters.  The
# graph's k1 (candidates around a position) is read as the window +-k1/2; the
# sketch stage keeps at most 256 (the last row asks 300).
TABLE1 = [(160, 1420, 370, 2, 0.729, 54.9), (160, 1420, 360, 2, 0.728, 18.0), (160, 1300, 350, 2, 0.719, 17.9),
          (160, 1300, 340, 2, 0.718, 16.1), (160, 1200, 330, 2, 0.710, 14.9), (160, 1200, 320, 2, 0.709, 17.3),
          (160, 1100, 310, 2, 0.700, 13.6), (160, 1100, 300, 2, 0.699, 15.7), (120, 4000, 1000, 2, 0.791, 29.4),
          (120, 3200, 1000, 2, 0.772, 25.8), (120, 2800, 1000, 2, 0.760, 23.6), (120, 2400, 1000, 2, 0.745, 23.8),
          (120, 2000, 1000, 2, 0.726, 19.4), (120, 1800, 1000, 2, 0.715, 18.3), (120, 1600, 1000, 2, 0.703, 19.6),
          (120, 1600, 800, 2, 0.700, 15.6)]
TABLE2 = [(74.0, 0.805, 80, 96, 60), (109.0, 0.855, 112, 106, 75), (164.0, 0.905, 160, 130, 100),
          (330.0, 0.955, 280, 168, 150), (856.0, 0.985, 720, 170, 300)]
MFMA_F16_PEAK_TFLOPS = 2500.0
PROFILES = os.path.join(ROOT, "profiles")


def kernel_source_hash(path):
    """Hash of a kernel's source file(s): counters recorded for another version are not reused."""
    import hashlib

    h = hashlib.sha256()
    for p in [path] if isinstance(path, str) else path:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(name, src, config):
    """HBM bytes per launch of a kernel, and the launch size they were taken
    on, from its committed rocprofv3 counter summary (FETCH_SIZE and
    WRITE_SIZE scaled by a plain-copy calibration); None when the summary is
    missing, was taken on another configuration, or the kernel source changed."""
    path = os.path.join(PROFILES, name)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_sha256_16") != kernel_source_hash(src) or rec.get("config") != config:
        return None
    return rec["hbm_bytes_per_launch"], rec["units_per_launch"]


def log(*a):
    print("[bench %.1fs]" % (time.time() - T0), *a, file=sys.stderr, flush=True)


T0 = time.time()


def _rescore_topk(rows_fp64, cand, k):
    """Top-k of candidate ids by (FP64 score desc, id asc); rows_fp64(cand) gives the scores."""
    import torch

    sc = rows_fp64(cand)
    # sort by id first, then stably by score: ties keep the smaller id first
    o = torch.argsort(cand, dim=1)
    cand, sc = torch.gather(cand, 1, o), torch.gather(sc, 1, o)
    o = torch.argsort(-sc, dim=1, stable=True)
    return torch.gather(cand, 1, o)[:, :k]


def ground_truth_ip(x, q, k, xchunk=1 << 20, qchunk=2500, extra=64):
    """Exact top-k by inner product: an FP32 screen on the GPU keeps the best
    k + 64 of all N rows, which are rescored in FP64 and re-sorted (score desc,
    id asc).  For recall only."""
    import torch

    nq, kk = q.shape[0], k + extra
    best_s = torch.full((nq, kk), -float("inf"), device=x.device)
    best_i = torch.zeros((nq, kk), dtype=torch.int64, device=x.device)
    qf = q.float()
    for xs in range(0, x.shape[0], xchunk):
        xf = x[xs:xs + xchunk].float()
        for qs in range(0, nq, qchunk):
            S = qf[qs:qs + qchunk] @ xf.T
            s, i = torch.topk(S, min(kk, S.shape[1]), dim=1)
            cs = torch.cat([best_s[qs:qs + qchunk], s], 1)
            ci = torch.cat([best_i[qs:qs + qchunk], i + xs], 1)
            s2, j = torch.topk(cs, kk, dim=1)
            best_s[qs:qs + qchunk] = s2
            best_i[qs:qs + qchunk] = torch.gather(ci, 1, j)
            del S
        del xf
    out = torch.empty((nq, k), dtype=torch.int64, device=x.device)
    qd = q.double()
    for qs in range(0, nq, qchunk):
        qq = qd[qs:qs + qchunk]
        out[qs:qs + qchunk] = _rescore_topk(
            lambda c: (x[c].double() * qq[:, None, :]).sum(-1), best_i[qs:qs + qchunk], k)
    return out


def ground_truth_graph(x, rows, k, xchunk=1 << 20, extra=64):
    """Exact k-NN graph rows by cosine, self excluded: FP32 screen of the best
    k + 64, FP64 rescore and re-sort (cosine desc, id asc)."""
    import torch

    xn = x.float()
    xn = xn / torch.linalg.vector_norm(xn, dim=1, keepdim=True)
    q = xn[rows]
    kk = k + extra
    best_s = torch.full((rows.numel(), kk), -float("inf"), device=x.device)
    best_i = torch.zeros((rows.numel(), kk), dtype=torch.int64, device=x.device)
    for xs in range(0, x.shape[0], xchunk):
        S = q @ xn[xs:xs + xchunk].T
        self_hit = (rows >= xs) & (rows < xs + S.shape[1])
        S[self_hit.nonzero().flatten(), (rows[self_hit] - xs)] = -float("inf")
        s, i = torch.topk(S, min(kk, S.shape[1]), dim=1)
        cs = torch.cat([best_s, s], 1)
        ci = torch.cat([best_i, i + xs], 1)
        s2, j = torch.topk(cs, kk, dim=1)
        best_s, best_i = s2, torch.gather(ci, 1, j)
    xd = x.double()
    nd = torch.linalg.vector_norm(xd, dim=1)
    out = torch.empty((rows.numel(), k), dtype=torch.int64, device=x.device)
    for s0 in range(0, rows.numel(), 2500):
        r = rows[s0:s0 + 2500]
        out[s0:s0 + 2500] = _rescore_topk(
            lambda c: (xd[c] * xd[r][:, None, :]).sum(-1) / (nd[r, None] * nd[c]), best_i[s0:s0 + 2500], k)
    return out


def audit(hf, torch, x, q, ids, scores):
    """Error of GPU scores against the FP64 audit kernel, over valid ids."""
    exact = hf.audit_scores(x, q, ids.int().contiguous())
    ok = ids >= 0
    err = (scores.double() - exact).abs()[ok]
    return {"max_abs": err.max().item(), "mean_abs": err.mean().item(), "pairs": int(ok.sum().item())}


def recall(found, truth):
    import torch

    k = truth.shape[1]
    hit = (found[:, :k].unsqueeze(2).long() == truth.unsqueeze(1)).any(2).sum().item()
    return hit / float(truth.numel())


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo), for the CPU-baseline record."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _set_affinity_all_threads(cpus):
    """CPU affinity of every thread of this process (OpenMP's pool included)."""
    for tid in os.listdir("/proc/self/task"):
        try:
            os.sched_setaffinity(int(tid), cpus)
        except OSError:
            pass


def cpu_runs(fn):
    """fn(threads) timed twice in this process: on every core the process may
    use (OpenMP at its default thread count), then on 8 of them with 8 OpenMP
    threads (the paper's 8-core limit).  Returns [(record, cores), ...]."""
    import oracle

    allowed = sorted(os.sched_getaffinity(0))
    threads_all = oracle.set_num_threads(1)
    oracle.set_num_threads(threads_all)
    out = [(fn(threads_all), {"threads": threads_all, "cpus": len(allowed), "pinned": False})]
    eight = set(allowed[:8])
    try:
        _set_affinity_all_threads(eight)
        oracle.set_num_threads(len(eight))
        out.append((fn(len(eight)), {"threads": len(eight), "cpus": len(eight), "pinned": True}))
    finally:
        oracle.set_num_threads(threads_all)
        _set_affinity_all_threads(set(allowed))
    return out


def cpu_baseline_search(args, gpu_entries_per_s):
    """The oracle (untuned) on a bounded sample of the search workload, with as
    many window entries per query as the GPU run (16 trees x n k1 / 16 each):
    the Hamming filter's work per query is matched, the data set is smaller."""
    import numpy as np

    import datagen
    import oracle

    n_s, t_s, nq_s = 100_000, 16, 1_000
    k1_s = min(n_s, args.trees * args.k1 // t_s)
    w = datagen.WORKLOADS["search-23Mx384"]
    comps = max(1, round(w["n_comp"] * n_s / w["n"]))
    x, q = datagen.mixture(n_s, w["d"], comps, w["sigma"], w["seed"], dtype=np.float16,
                           query_seed=w["query_seed"], nq=nq_s)
    F = oracle.build_forest(x, T=t_s, M=args.leaf, seed=5, sketch_seed=6)

    def run(threads):
        t = time.perf_counter()
        oracle.search(F, q, k1_s, args.k2, args.h, args.k)
        return time.perf_counter() - t

    recs = []
    for dt, c in cpu_runs(run):
        ent = nq_s * t_s * k1_s / dt
        recs.append({"value": nq_s / dt, "unit": "queries/s", "cores": c["threads"], "pinned_8": c["pinned"],
                     "kind": "oracle", "cpu_model": cpu_model(), "window_entries_per_s": ent,
                     "gpu_over_cpu_per_entry": gpu_entries_per_s / ent,
                     "sample": "oracle search (Alg. 1 stages after the build) of %d queries on a %d x %d sample "
                               "of the same mixture recipe (%d components), %d trees x k1=%d window entries per "
                               "query (the GPU run: %d x %d), k2=%d h=%d k=%d; %.2f s on %d threads%s"
                               % (nq_s, n_s, w["d"], comps, t_s, k1_s, args.trees, args.k1, args.k2, args.h,
                                  args.k, dt, c["threads"], " pinned to 8 cores" if c["pinned"] else "")})
        log("cpu baseline search: %.2f s on %d threads (%.3g window entries/s)" % (dt, c["threads"], ent))
    res = dict(recs[0])
    res["pinned_8_cores"] = recs[1] if len(recs) > 1 else None
    return res


def cpu_baseline_graph(args, n_full):
    """The oracle graph on a 100K sample (16 orders, 1,000 rows), scaled to the
    full workload's orders, points and rows."""
    import numpy as np

    import datagen
    import oracle

    n_s, rows_s, o_s = 100_000, 1_000, min(16, args.orders)
    w = datagen.WORKLOADS["graph-3Mx384"]
    comps = max(1, round(w["n_comp"] * n_s / w["n"]))
    x = datagen.mixture(n_s, w["d"], comps, w["sigma"], w["seed"], dtype=np.float16)

    def run(threads):
        t = time.perf_counter()
        orders, _ = oracle.graph_orders(x, o_s, 3)
        t_sort = time.perf_counter() - t
        t = time.perf_counter()
        oracle.graph_rows(x, orders, args.window, args.k, np.arange(rows_s))
        return t_sort, time.perf_counter() - t

    recs = []
    for (t_sort, t_rows), c in cpu_runs(run):
        # sorts scale with orders x points (n log n taken as linear: favours the
        # CPU), candidate lists with orders x rows
        f_o = args.orders / o_s
        est = t_sort * f_o * (n_full / n_s) + t_rows * f_o * (n_full / rows_s)
        recs.append({"value": est, "unit": "s", "cores": c["threads"], "pinned_8": c["pinned"], "kind": "oracle",
                     "cpu_model": cpu_model(),
                     "sample": "oracle graph on a %d x %d sample of the same recipe: %d orders sorted in %.2f s, "
                               "candidate lists (w=%d, k=%d) of %d rows in %.2f s, on %d threads%s; value = sort "
                               "time x (%d/%d orders) x (%d/%d points) + row time x (%d/%d orders) x (%d/%d rows)"
                               % (n_s, w["d"], o_s, t_sort, args.window, args.k, rows_s, t_rows, c["threads"],
                                  " pinned to 8 cores" if c["pinned"] else "", args.orders, o_s, n_full, n_s,
                                  args.orders, o_s, n_full, rows_s)})
        log("cpu baseline graph: estimated %.0f s on %d threads" % (est, c["threads"]))
    res = dict(recs[0])
    res["pinned_8_cores"] = recs[1] if len(recs) > 1 else None
    return res


def bench_search(args, hf, torch, ws):
    import datagen

    N = args.n or ws["n"]
    nq = args.nq or ws["nq"]
    d = ws["d"]
    log("drawing %d x %d data and %d queries on the device" % (N, d, nq))
    x = datagen.mixture_device(N, d, ws["n_comp"], ws["sigma"], ws["seed"], ws["unit"])
    q = datagen.mixture_device(nq, d, ws["n_comp"], ws["sigma"], ws["seed"], ws["unit"],
                               draw_seed=ws["query_seed"])
    torch.cuda.synchronize()
    log("building forest: %d trees, leaves <= %d" % (args.trees, args.leaf))
    hf.timing_enable(True)
    t = time.perf_counter()
    forest = hf.Forest(x, n_trees=args.trees, leaf_max=args.leaf, seed=5, sketch_seed=6)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t
    build_stages = hf.timing_read()
    log("forest built in %.2f s: %s" % (build_s, {k: round(v[0], 1) for k, v in build_stages.items()}))
    log("ground truth (exact GPU brute force)")
    torch.cuda.synchronize()
    t = time.perf_counter()
    gt = ground_truth_ip(x, q, args.k)
    torch.cuda.synchronize()
    gt_s = time.perf_counter() - t
    # exact search scores every (query, point) pair: 2 N d flops per query
    bf_flop = 2.0 * N * d * nq
    brute = {"qps": nq / gt_s, "recall": 1.0,
             "method": "FP32 GEMM (torch) and top-(k+64) over 1M-row chunks of all N rows, the k+64 rescored "
                       "in FP64 and re-sorted",
             "fp16_mfma_ceiling_qps": nq / (bf_flop / (MFMA_F16_PEAK_TFLOPS * 1e12))}
    log("brute force: %.0f QPS (an fp16 MFMA brute force could reach at most %.0f QPS)"
        % (brute["qps"], brute["fp16_mfma_ceiling_qps"]))
    sweep = []
    if args.sweep:
        for cfg in args.sweep.split(";"):
            v = [int(u) for u in cfg.split(",")]
            k1, k2, h, tr = v[0], v[1], v[2], (v[3] if len(v) > 3 else 0)
            forest.search(q, args.k, k1, k2, h, trees=tr)
            torch.cuda.synchronize()
            t = time.perf_counter()
            ids, _ = forest.search(q, args.k, k1, k2, h, trees=tr)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t
            r = recall(ids, gt)
            sweep.append({"k1": k1, "k2": k2, "h": h, "trees": tr or args.trees, "recall": r, "qps": nq / dt})
            log("sweep k1=%d k2=%d h=%d trees=%d: recall %.4f, %.0f QPS" % (k1, k2, h, tr or args.trees, r, nq / dt))
            hf.timing_read()
    for _ in range(args.warmup):
        forest.search(q, args.k, args.k1, args.k2, args.h)
    torch.cuda.synchronize()
    hf.timing_read()
    log("timing %d steps" % args.steps)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(args.steps):
        ids, sc = forest.search(q, args.k, args.k1, args.k2, args.h)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    stages = hf.timing_read()
    hf.timing_enable(False)
    rec = recall(ids, gt)
    qps = nq * args.steps / dt
    alt = None
    if args.alt:
        a1, a2, ah = (int(v) for v in args.alt.split(","))
        forest.search(q, args.k, a1, a2, ah)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.steps):
            aids, _ = forest.search(q, args.k, a1, a2, ah)
        torch.cuda.synchronize()
        adt = time.perf_counter() - t
        alt = {"k1": a1, "k2": a2, "h": ah, "recall": recall(aids, gt), "qps": nq * args.steps / adt,
               "ms_per_step": adt * 1e3 / args.steps}
        log("alternative budget k1=%d k2=%d h=%d: recall %.4f, %.0f QPS" % (a1, a2, ah, alt["recall"], alt["qps"]))
    exact = None
    if args.exact:
        # the same budget with windows centred on each query's exact rank
        # along every tree's curve instead of its leaf's midpoint
        forest.search(q, args.k, args.k1, args.k2, args.h, position="exact")
        torch.cuda.synchronize()
        hf.timing_enable(True)
        hf.timing_read()
        t = time.perf_counter()
        for _ in range(args.steps):
            eids, _ = forest.search(q, args.k, args.k1, args.k2, args.h, position="exact")
        torch.cuda.synchronize()
        edt = time.perf_counter() - t
        est = hf.timing_read()
        hf.timing_enable(False)
        exact = {"position": "exact rank", "recall": recall(eids, gt), "qps": nq * args.steps / edt,
                 "ms_per_step": edt * 1e3 / args.steps,
                 "stages_ms_per_step": {k_: v_[0] / args.steps for k_, v_ in est.items()}}
        log("exact positions: recall %.4f, %.0f QPS (descent %.2f ms)" % (
            exact["recall"], exact["qps"], exact["stages_ms_per_step"].get("descend", 0.0)))
    c3 = None
    if args.c3:
        # the same data, queries and k at 160 trees (the forest's first 160:
        # tree t does not depend on the trees after it)
        c1_, c2_, ch_, ct_ = (int(v) for v in args.c3.split(","))
        forest.search(q, args.k, c1_, c2_, ch_, trees=ct_)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.steps):
            cids, _ = forest.search(q, args.k, c1_, c2_, ch_, trees=ct_)
        torch.cuda.synchronize()
        cdt = time.perf_counter() - t
        c3 = {"trees": ct_, "k1": c1_, "k2": c2_, "h": ch_, "recall": recall(cids, gt),
              "qps": nq * args.steps / cdt, "ms_per_step": cdt * 1e3 / args.steps}
        log("%d trees k1=%d k2=%d h=%d: recall %.4f, %.0f QPS" % (ct_, c1_, c2_, ch_, c3["recall"], c3["qps"]))
    table1 = None
    if args.tables:
        table1 = []
        for (tn, t1, t2, th, prec_, psec) in TABLE1:
            forest.search(q, args.k, t1, t2, th, trees=tn)
            torch.cuda.synchronize()
            t = time.perf_counter()
            tids, _ = forest.search(q, args.k, t1, t2, th, trees=tn)
            torch.cuda.synchronize()
            tdt = time.perf_counter() - t
            table1.append({"n": tn, "k1": t1, "k2": t2, "h": th, "recall": recall(tids, gt), "qps": nq / tdt,
                           "paper_recall": prec_, "paper_s_per_10k_queries": psec})
        log("Table 1 rows on the stand-in: %s" % [(r_["n"], r_["k1"], round(r_["recall"], 3), round(r_["qps"]))
                                                   for r_ in table1])
    log("recall@%d %.4f, %.0f QPS, stages %s" % (args.k, rec, qps,
                                                  {k: round(v[0] / args.steps, 2) for k, v in stages.items()}))
    # roofline of the dominant kernel: the Hamming filter streams n*k1 window
    # entries per query, each a 4-byte position read, a 64-byte sketch read and
    # a 2-byte distance write (duplicates included, as the paper counts them)
    T = args.trees
    ln = min(args.k1, N)
    ham_ms, ham_n = stages["hamming"]
    per_launch_q = nq * args.steps / ham_n
    bytes_launch = per_launch_q * (T * ln * 70 + T * 4 + 64 + 513 * 4)
    achieved = bytes_launch / (ham_ms / ham_n * 1e-3) / 1e9
    src = [os.path.join(ROOT, "paper_2508_21682_amd", "csrc", "hf_bfilter.hip")]
    cfg = {"n": N, "queries": nq, "trees": T, "leaf_max": args.leaf, "k1": args.k1, "k2": args.k2, "h": args.h}
    rec_t = measured_traffic("filter_search-23Mx384_counters.json", src, cfg)
    # bytes per query scale with the launch's queries
    traffic = rec_t[0] * per_launch_q / rec_t[1] if rec_t else None
    # the filter stage: the bucketed filter's kernels (threshold, count, scan,
    # plan, scatter, score, select); the entry-by-entry filter of the queries
    # it flags is timed with the selection stage
    roof = {"bound": "hbm", "kernel": "hamming filter stage (k_tau k_bcount k_brow_scan k_bplan k_bscatter k_bscore "
            "k_bselect)", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "bytes_per_launch": bytes_launch, "ms_per_launch": ham_ms / ham_n}
    res = {"metric": "QPS @recall@30>=0.7 (23Mx384)", "value": qps, "unit": "queries/s",
           "ms_per_step": dt * 1e3 / args.steps, "recall": rec, "higher_is_better": True,
           "config": {"workload": args.workload, "n": N, "d": d, "queries": nq, "trees": T,
                      "leaf_max": args.leaf, "k": args.k, "k1": args.k1, "k2": args.k2, "h": args.h,
                      "sketch_bits": 512, "rerank": "fp32"},
           "build_s": build_s, "roofline": roof, "brute_force": brute, "alt_budget": alt, "config3": c3,
           "exact_position": exact, "table1": table1,
           "window_entries_per_s": nq * args.steps * T * ln / dt,
           "stages_ms_per_step": {k: v[0] / args.steps for k, v in stages.items()}}
    if sweep:
        res["sweep"] = sweep
    res["audit_fp32"] = audit(hf, torch, x, q, ids, sc)
    if args.forms:
        res["forms"] = {}
        for prec in args.forms.split(","):
            forest.add_precision(prec)
            if prec == "c4":
                # the paper's layout: coordinate-sign sketches for the filter
                forest.set_sketch("sign")
            for _ in range(args.warmup):
                forest.search(q, args.k, args.k1, args.k2, args.h, precision=prec)
            hf.timing_enable(True)
            hf.timing_read()
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(args.steps):
                pid, psc = forest.search(q, args.k, args.k1, args.k2, args.h, precision=prec)
            torch.cuda.synchronize()
            pdt = time.perf_counter() - t
            pst = hf.timing_read()
            hf.timing_enable(False)
            form = {"qps": nq * args.steps / pdt, "recall": recall(pid, gt), "ms_per_step": pdt * 1e3 / args.steps,
                    "stages_ms_per_step": {k_: v[0] / args.steps for k_, v in pst.items()}}
            if alt:
                # the budget with the +-h expansion, where E is about 3x C2
                forest.search(q, args.k, alt["k1"], alt["k2"], alt["h"], precision=prec)
                torch.cuda.synchronize()
                t = time.perf_counter()
                for _ in range(args.steps):
                    aid, _ = forest.search(q, args.k, alt["k1"], alt["k2"], alt["h"], precision=prec)
                torch.cuda.synchronize()
                adt2 = time.perf_counter() - t
                form["alt_budget"] = {"recall": recall(aid, gt), "qps": nq * args.steps / adt2,
                                      "qps_fp32": alt["qps"]}
            if prec == "c4":
                # scores are inner products with the decoded 4-bit rows; their
                # distance to the exact FP64 scores is the codes' error
                form.update({"sketch": "coordinate signs (%d bits)" % x.shape[1],
                             "row_bytes": x.shape[1] // 2 + 4, "row_bytes_fp16": 2 * x.shape[1],
                             "audit_final_vs_exact": audit(hf, torch, x, q, pid, psc)})
                forest.set_sketch("srp")
                log("form c4: recall %.4f, %.0f QPS, rerank %.2f ms, score error vs exact max %.3g" % (
                    form["recall"], form["qps"], form["stages_ms_per_step"].get("rerank", 0.0),
                    form["audit_final_vs_exact"]["max_abs"]))
            else:
                sub = q[:1000]
                r = forest.search_lowprec_debug(sub, args.k, args.k1, args.k2, args.h, prec)
                p2i = forest.pos2id().long()
                sp = r["surv_pos"].long()
                ok = sp >= 0
                sid = torch.where(ok, p2i[sp.clamp(min=0)], torch.full_like(sp, -1)).int()
                lp_err = audit(hf, torch, x, sub, sid, r["surv_score"])
                form.update({"survivors": 4 * args.k, "audit_final_fp32": audit(hf, torch, x, q, pid, psc),
                             "audit_lowprec_scores": lp_err})
                log("form %s: recall %.4f, %.0f QPS, low-precision score error max %.3g" % (
                    prec, form["recall"], form["qps"], lp_err["max_abs"]))
            res["forms"][prec] = form
    lhash = None
    if args.learned:
        res.setdefault("forms", {})["learned"], lhash = bench_learned(args, hf, torch, ws, forest, x, q, gt, nq)
    forest.free()
    return res, lhash


def bench_learned(args, hf, torch, ws, forest, x, q, gt, nq):
    """Learned sketches: the MLP hash trained by libhf on pairs the forest
    itself generates -- for every training query its 30 best results at a
    larger budget (positives) and, per positive, one of its C2 candidates
    (close in SRP Hamming distance) that is not among them (hard negative) --
    then used as the forest's sketches at the same (k1, k2, h); SRP is
    restored afterwards.  Returns (record, the trained hash)."""
    import datagen
    import numpy as np

    ntr, kn = args.learned_queries, args.learned_nn
    qt = datagen.mixture_device(ntr, ws["d"], ws["n_comp"], ws["sigma"], ws["seed"], ws["unit"], draw_seed=2513)
    g1, g2, gh = (int(v) for v in args.learned_budget.split(","))
    log("learned hash: forest pairs of %d training queries (k1=%d k2=%d h=%d)" % (ntr, g1, g2, gh))
    torch.cuda.synchronize()
    t = time.perf_counter()
    nn_l, c2_l = [], []
    for s0 in range(0, ntr, 10000):
        r = forest.search_debug(qt[s0:s0 + 10000], kn, g1, g2, gh)
        nn_l.append(r["ids"].long())
        c2_l.append(r["c2"].long())
    nn = torch.cat(nn_l)
    c2 = forest.pos2id().long()[torch.cat(c2_l).clamp(min=0)]
    # per query, the C2 candidates (in Hamming order) that are not positives
    isneg = ~(c2.unsqueeze(2) == nn.unsqueeze(1)).any(2)
    rank = torch.cumsum(isneg.int(), 1) - 1
    negs = torch.full((ntr, kn), -1, dtype=torch.long, device=x.device)
    pick = isneg & (rank < kn)
    rows_i = torch.arange(ntr, device=x.device).unsqueeze(1).expand_as(c2)
    negs[rows_i[pick], rank[pick]] = c2[pick]
    negs = torch.where(negs < 0, nn, negs)  # (never short at these budgets)
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t
    nn_np = nn.cpu().numpy()
    e = forest.info["quant_exp"]
    qi, pi = hf.hilbert_pairs(hf.quantize(qt, e), nn_np, 5, args.learned_batch)
    # the negative of pair (query, r-th positive) is the query's r-th negative
    rk = np.repeat(np.arange(kn), len(qi) // kn)
    ni = negs.cpu().numpy()[qi, rk]
    A = qt[torch.from_numpy(qi).to(x.device)].contiguous()
    B = x[torch.from_numpy(pi).to(x.device)].contiguous()
    Nn = x[torch.from_numpy(ni).to(x.device)].contiguous()
    L = hf.LHash.init(ws["d"], 256, seed=7)
    torch.cuda.synchronize()
    t = time.perf_counter()
    curve = L.train(A, B, hf.train_params(epochs=args.learned_epochs, batch=args.learned_batch, lr=1e-3, tau=0.1,
                                          slope=2.0, balance=0.05, keep_blocks=True), N=Nn)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t
    log("learned hash trained on %d pairs (+ as many hard negatives) in %.2f s, loss per epoch %s"
        % (A.shape[0], train_s, np.round(curve, 3)))
    del A, B, Nn
    # encode of all N rows: one untimed call, then the median of three
    forest.set_sketch("learned", L)
    torch.cuda.synchronize()
    enc_t = []
    for _ in range(3):
        t = time.perf_counter()
        forest.set_sketch("learned", L)
        torch.cuda.synchronize()
        enc_t.append(time.perf_counter() - t)
    enc_s = float(np.median(enc_t))
    enc_flop = 2.0 * x.shape[0] * (ws["d"] * 256 + 256 * 512)
    forest.search(q, args.k, args.k1, args.k2, args.h)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(args.steps):
        lid, _ = forest.search(q, args.k, args.k1, args.k2, args.h)
    torch.cuda.synchronize()
    ldt = time.perf_counter() - t
    lrec = recall(lid, gt)
    forest.set_sketch("srp")
    srid, _ = forest.search(q, args.k, args.k1, args.k2, args.h)
    srec = recall(srid, gt)
    log("learned sketches: recall %.4f vs SRP %.4f at k1=%d k2=%d h=%d" % (lrec, srec, args.k1, args.k2, args.h))
    return ({"recall": lrec, "recall_srp_same_budget": srec, "gain_over_srp": lrec - srec,
             "qps": nq * args.steps / ldt, "train_pairs": int(len(qi)), "hard_negatives": int(len(qi)),
             "pairs_from": "forest search k1=%d k2=%d h=%d (positives: its top %d; negatives: C2 entries not "
                           "among them, in Hamming order)" % (g1, g2, gh, kn),
             "pair_generation_s": gen_s, "train_s": train_s, "encode_23M_s": enc_s,
             # the encoder's two dense layers over every row: 2 (d 256 + 256 512) flops a row
             "encode_tflop_per_s": enc_flop / enc_s / 1e12,
             "encode_frac_bf16_peak": enc_flop / enc_s / 1e12 / MFMA_F16_PEAK_TFLOPS,  # bf16 peak = fp16 peak
             "loss_per_epoch": [float(v) for v in curve],
             "sketch_in_use": "srp" if lrec <= srec else "learned"}, L)


def bench_graph(args, hf, torch, ws, k, lhash):
    import datagen

    N = (args.n if args.workload.startswith("graph") else None) or ws["n"]
    d = ws["d"]
    log("drawing %d x %d data on the device" % (N, d))
    x = datagen.mixture_device(N, d, ws["n_comp"], ws["sigma"], ws["seed"], ws["unit"])
    torch.cuda.synchronize()
    if args.sweep and args.workload.startswith("graph"):
        rows = torch.randperm(N, generator=torch.Generator(device="cpu").manual_seed(4))[:10000].to(x.device)
        gt = ground_truth_graph(x, rows, k)
        for cfg in args.sweep.split(";"):
            v = [int(u) for u in cfg.split(",")]
            no, wi, k2 = v[0], v[1], (v[2] if len(v) > 2 else 0)
            torch.cuda.synchronize()
            hf.timing_enable(True)
            hf.timing_read()
            t = time.perf_counter()
            ids, _ = hf.knn_graph(x, no, wi, k, 3, k2=k2, sketch_seed=6)
            torch.cuda.synchronize()
            el = time.perf_counter() - t
            st = hf.timing_read()
            hf.timing_enable(False)
            log("graph sweep orders=%d w=%d k2=%d: recall %.4f, %.3f s %s" % (
                no, wi, k2, recall(ids[rows], gt), el,
                {k_: round(v_[0], 1) for k_, v_ in st.items() if v_[1]}))
    for _ in range(args.warmup):
        hf.knn_graph(x, args.orders, args.window, k, 3)
    torch.cuda.synchronize()
    hf.timing_enable(True)
    hf.timing_read()
    t = time.perf_counter()
    for _ in range(args.steps):
        ids, sc = hf.knn_graph(x, args.orders, args.window, k, 3)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    stages = hf.timing_read()
    hf.timing_enable(False)
    rows = torch.randperm(N, generator=torch.Generator(device="cpu").manual_seed(4))[:10000].to(x.device)
    gt = ground_truth_graph(x, rows, k)
    rec = recall(ids[rows], gt)
    log("graph %.3f s, recall %.4f, stages %s" % (dt / args.steps, rec,
                                                   {k: round(v[0] / args.steps, 2) for k, v in stages.items()}))
    band_ms, band_n = stages["graph_band"]
    # per band launch (one order): every position reads its re-laid row once
    # (2d B), its norm and id (8 B), and reads and writes its top-k list
    # (16k B); neighbours' rows come through the caches
    bytes_launch = N * (d * 2 + 4 + 4 + k * 8 * 2)
    achieved = bytes_launch / (band_ms / band_n * 1e-3) / 1e9
    src = os.path.join(ROOT, "paper_2508_21682_amd", "csrc", "hf_graph.hip")
    cfg = {"n": N, "orders": args.orders, "window": args.window, "k": k}
    rec_t = measured_traffic("k_band_graph-3Mx384_counters.json", src, cfg)
    roof = {"bound": "hbm", "kernel": "k_band", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": rec_t[0] if rec_t else None,
            "bytes_per_launch": bytes_launch, "ms_per_launch": band_ms / band_n}
    prefilter = None
    if lhash is not None:
        # the sketch stage of Alg. 2 with learned sketches against SRP and the
        # plain form, at each setting of orders, window and k2 (the first is
        # the learned form's graph shape: 32 orders, window +-32)
        prefilter = []
        for pcfg in args.prefilter.split(";"):
            po, pw, pk2 = (int(v) for v in pcfg.split(","))
            forms = {}
            for name, kw in [("learned", dict(k2=pk2, sketch="learned", lhash=lhash)),
                             ("srp", dict(k2=pk2, sketch_seed=6)), ("plain", dict())]:
                hf.knn_graph(x, po, pw, k, 3, **kw)
                torch.cuda.synchronize()
                t = time.perf_counter()
                pids, _ = hf.knn_graph(x, po, pw, k, 3, **kw)
                torch.cuda.synchronize()
                forms[name] = {"k2": kw.get("k2", 0), "recall": recall(pids[rows], gt), "s": time.perf_counter() - t}
            prefilter.append({"orders": po, "window": pw, "forms": forms})
            log("graph sketch stage (%d orders, +-%d, k2=%d): %s" % (po, pw, pk2, {
                n_: (round(v_["recall"], 3), round(v_["s"], 3)) for n_, v_ in forms.items()}))
    table2 = None
    if args.tables:
        table2 = []
        for (psec, prec_, tn, tk1, tk2) in TABLE2:
            torch.cuda.synchronize()
            t = time.perf_counter()
            tids, _ = hf.knn_graph(x, tn, tk1 // 2, k, 3, k2=min(tk2, 256), sketch_seed=6)
            torch.cuda.synchronize()
            tdt = time.perf_counter() - t
            table2.append({"orders": tn, "window": tk1 // 2, "k2": min(tk2, 256), "recall": recall(tids[rows], gt),
                           "s": tdt, "paper_recall": prec_, "paper_s": psec, "paper_k1": tk1, "paper_k2": tk2})
        log("Table 2 rows on the stand-in: %s" % [(r_["orders"], r_["window"], round(r_["recall"], 3),
                                                    round(r_["s"], 2)) for r_ in table2])
    return {"metric": "kNN-graph build s (3Mx384, k=15)", "value": dt / args.steps, "unit": "s",
            "ms_per_step": dt * 1e3 / args.steps, "recall": rec, "higher_is_better": False,
            "config": {"workload": "graph-3Mx384", "n": N, "d": d, "orders": args.orders,
                       "window": args.window, "k": k}, "roofline": roof,
            "stages_ms_per_step": {k: v[0] / args.steps for k, v in stages.items()}, "table2": table2,
            "prefilter": prefilter}


def bench_configs(args, hf, torch):
    """The two small configurations: the 10,000 x 32 search (8 trees, recall@10
    against the exact inner-product top-10) and the 1M x 384 graph (16 orders,
    +-32, recall@15 on 10,000 sampled rows)."""
    import numpy as np

    import datagen

    out = {}
    w = datagen.WORKLOADS["search-10Kx32"]
    x, q = datagen.mixture(w["n"], w["d"], w["n_comp"], w["sigma"], w["seed"], unit=w["unit"], dtype=np.float32,
                           query_seed=w["query_seed"], nq=w["nq"])
    x, q = torch.from_numpy(x).cuda(), torch.from_numpy(q).cuda()
    fo = hf.Forest(x, n_trees=8, leaf_max=100, seed=1, sketch_seed=2)
    gt = ground_truth_ip(x, q, 10)
    k1, k2, h = 256, 64, 1
    fo.search(q, 10, k1, k2, h)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(args.steps):
        ids, _ = fo.search(q, 10, k1, k2, h)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / args.steps
    fo.free()
    out["search-10Kx32"] = {"trees": 8, "leaf_max": 100, "k": 10, "k1": k1, "k2": k2, "h": h,
                            "recall": recall(ids, gt), "qps": q.shape[0] / dt, "ms_per_step": dt * 1e3}
    log("search-10Kx32: recall@10 %.4f, %.3f ms per 1,000 queries" % (out["search-10Kx32"]["recall"], dt * 1e3))
    w = datagen.WORKLOADS["graph-1Mx384"]
    x = datagen.mixture_device(w["n"], w["d"], w["n_comp"], w["sigma"], w["seed"], w["unit"])
    hf.knn_graph(x, 16, 32, 15, 3)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(args.steps):
        gids, _ = hf.knn_graph(x, 16, 32, 15, 3)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / args.steps
    rows = torch.randperm(w["n"], generator=torch.Generator(device="cpu").manual_seed(4))[:10000].to(x.device)
    gr = recall(gids[rows], ground_truth_graph(x, rows, 15))
    out["graph-1Mx384"] = {"orders": 16, "window": 32, "k": 15, "recall": gr, "build_s": dt}
    log("graph-1Mx384: recall@15 %.4f in %.4f s" % (gr, dt))
    del x, gids
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="search-23Mx384", choices=["search-23Mx384", "graph-3Mx384"])
    ap.add_argument("--n", type=int, default=None, help="override N (development runs only)")
    ap.add_argument("--nq", type=int, default=None)
    ap.add_argument("--trees", type=int, default=1280)
    ap.add_argument("--leaf", type=int, default=100)
    ap.add_argument("--k", type=int, default=None)
    ap.add_argument("--k1", type=int, default=70)
    ap.add_argument("--k2", type=int, default=1000)
    ap.add_argument("--h", type=int, default=0)
    ap.add_argument("--alt", default="65,1000,1",
                    help="search: a second budget 'k1,k2,h' timed on the same forest ('' for none); the default "
                         "is the fastest found at recall >= 0.7 that keeps the +-h expansion")
    ap.add_argument("--orders", type=int, default=228)
    ap.add_argument("--window", type=int, default=160)
    ap.add_argument("--sweep", default=None,
                    help="extra configs: search 'k1,k2,h;...', graph 'orders,w[,k2];...'")
    ap.add_argument("--forms", default="bf16,fp8,c4",
                    help="forms measured after the plain search: bf16, fp8 (low-precision scoring, FP32 rerank), "
                         "c4 (sign sketches and 4-bit codes, the paper's layout)")
    ap.add_argument("--learned", type=int, default=1, help="also train and measure the learned sketch form")
    ap.add_argument("--learned-queries", type=int, default=66667,
                    help="training queries; pairs = queries x --learned-nn (2M by default)")
    ap.add_argument("--learned-budget", default="140,3000,1",
                    help="'k1,k2,h' of the forest search that generates the training pairs and negatives")
    ap.add_argument("--learned-nn", type=int, default=30)
    ap.add_argument("--learned-batch", type=int, default=500)
    ap.add_argument("--learned-epochs", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--graph", type=int, default=1,
                    help="search workload: also time the 3M x 384 graph (--orders, --window) in the same line")
    ap.add_argument("--configs", type=int, default=1,
                    help="search workload: also run the 10K x 32 search and the 1M x 384 graph configurations")
    ap.add_argument("--prefilter", default="32,32,128;128,128,256",
                    help="graph: 'orders,window,k2[;...]' at which learned and SRP sketch stages are compared with the plain form")
    ap.add_argument("--tables", type=int, default=1,
                    help="also re-run the paper's Table 1 (search) and Table 2 (graph) parameters once each")
    ap.add_argument("--exact", type=int, default=1,
                    help="search: also time the main budget with exact query positions (insertion ranks)")
    ap.add_argument("--c3", default="2400,1100,2,160",
                    help="search: 'k1,k2,h,trees' timed on the forest's first trees ('' for none): the budget "
                         "at 160 trees")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (counter calibration for rocprofv3)")
    ap.add_argument("--peaks", action="store_true",
                    help="only run the ceiling probes (copy, random gathers, fp16 MFMA)")
    args = ap.parse_args()
    if args.peaks:
        import subprocess

        from paper_2508_21682_amd import build as hb

        if not os.path.exists(hb.PEAKS):
            sys.exit("%s is not built: run build() first" % hb.PEAKS)
        out = subprocess.run([hb.PEAKS], check=True, capture_output=True, text=True).stdout
        rows = [json.loads(line) for line in out.splitlines() if line.startswith("{")]
        print(json.dumps({"peaks": rows, "published": {"hbm_gb_per_s": HBM_PEAK_GBS,
                                                       "mfma_f16_tflop_per_s": MFMA_F16_PEAK_TFLOPS}}),
              flush=True)
        return
    if args.calibrate_copy:
        import torch

        n = args.calibrate_copy << 20
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n, "launches": 3}), flush=True)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU; the library has no multi-GPU path (got --gpus %d)"
              % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.k is None:
        args.k = 30 if args.workload.startswith("search") else 15
    import torch

    import datagen
    import paper_2508_21682_amd as hf

    hf.lib()
    ws = datagen.WORKLOADS[args.workload]
    if args.workload.startswith("search"):
        res, lhash = bench_search(args, hf, torch, ws)
        torch.cuda.empty_cache()
        if args.graph:
            # the other half of the metric: the 3M x 384 k-NN graph
            log("graph-3Mx384: %d orders, window +-%d" % (args.orders, args.window))
            res["graph"] = bench_graph(args, hf, torch, datagen.WORKLOADS["graph-3Mx384"], 15, lhash)
            torch.cuda.empty_cache()
        if lhash is not None:
            lhash.free()
        if args.configs:
            res["configs"] = bench_configs(args, hf, torch)
    else:
        res = bench_graph(args, hf, torch, ws, args.k, None)
    res.update({"n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "scaling": "weak",
                "vs_baseline": None, "dtype": "f16", "data": "synthetic"})
    if not args.no_cpu_baseline:
        log("cpu baselines (the oracle on bounded samples; all cores, then 8 pinned cores)")
        if args.workload.startswith("search"):
            res["cpu_baseline"] = cpu_baseline_search(args, res["window_entries_per_s"])
            if "graph" in res:
                res["graph"]["cpu_baseline"] = cpu_baseline_graph(args, res["graph"]["config"]["n"])
        else:
            res["cpu_baseline"] = cpu_baseline_graph(args, res["config"]["n"])
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
