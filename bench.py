#!/usr/bin/env python3
"""Benchmark of the GPU filtering stage on one MI355X.

Workload (default): 100M int8 vectors of dimension 100 drawn from a seeded
Gaussian mixture (8192 centres U[-128,127]^100, sigma 10, rounded and
clipped), IVF with 65536 lists (Eq. 2 replication, at most 2 lists per
vector), PQ with 50 subspaces x 256 codewords (5 GB of codes, raw vectors in
HBM), 10,000 queries, nprobe 64, k 10, rerank_n at the recall@10 >= 0.9
operating point.  The index is built on the host first (about 2.5 minutes).
A step is one pass of the whole path (probe, distance table, gather + dedup,
Eq. 1 scan, top-n, exact re-rank) over all queries, with the index and the
queries already in HBM.  --workload ivf_u8_10m runs the 10M uint8 one.

Forms timed:
  plain    one ann_search call per batch of 256 queries (default work split);
           also the latency of single-query calls
  batched  the whole batch as one HIP-graph launch (ann_graph_launch) with the
           work split the autotuner picked; its per-stage times come from an
           event-bracketed eager run of the same search ("batched_eager")
  served   Poisson arrivals of requests of U{1..256} queries into the
           continuous-batching server at several offered loads, then saturation
The headline value is the batched form's queries/s.

Also reported: candidates/s, recall@10 against exact kNN of a query sample,
bit-exact parity of a query sample against the CPU oracle, the scan kernel's
roofline (HBM: code bytes of the scored candidates plus 4 bytes per replica
entry walked, over the scan's per-launch time from HIP events), and the CPU
oracle's own throughput on a bounded sample (all host threads, and one).
Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "PQ-ADC candidates/s + QPS at recall@10>=0.9, batched vs plain, 1 MI355X"
HBM_PEAK_GBS = 8000.0
SCAN_SOURCES = ["paper_2409_16576_amd/csrc/ann_kernels.hip"]


# Per-workload defaults, sized so a default run (index build included) ends
# within a few minutes: oracle sample, brute-force sample, served loads
# (million queries/s) and window, heuristic (rerank_n, batch, eps, beta).
WORKLOAD_DEFAULTS = {
    "serve_i8_100m": dict(cpu_queries=2000, recall_queries=200,
                          served_rates="0.005,0.01,0.02,0.05,0.2,0.5", served_seconds=2.0,
                          heur="400,100,0,2"),
    "ivf_u8_10m": dict(cpu_queries=10000, recall_queries=500,
                       served_rates="0.25,0.5,1,1.5,2,3", served_seconds=1.5,
                       heur="2000,200,0,2"),
    "zipf_f32_5m": dict(cpu_queries=2000, recall_queries=200, served_rates="0.1,0.2,0.5",
                        served_seconds=1.5, heur="3200,400,0,2"),
    "ivf_f32_100k": dict(cpu_queries=1000, recall_queries=1000, served_rates="0.1,0.5,1",
                         served_seconds=1.0, heur="800,100,0,2"),
}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    h = hashlib.sha256()
    for s in SCAN_SOURCES:
        with open(os.path.join(ROOT, s), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def load_traffic(stage: str, workload: str):
    """HBM traffic per launch of a stage's kernel from the committed counter
    summary, if it was taken on the current kernel source; else None."""
    p = os.path.join(ROOT, "profiles", f"traffic_{stage}_{workload}.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        t = json.load(f)
    if t.get("kernel_sha") != kernel_hash():
        return None
    return t


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="serve_i8_100m")
    ap.add_argument("--plain-batch", type=int, default=256)
    ap.add_argument("--cpu-queries", type=int, default=None)
    ap.add_argument("--recall-queries", type=int, default=None)
    ap.add_argument("--rerank-n", type=int, default=0,
                    help="top-n re-ranked (default: the workload's recall>=0.9 operating point)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle leg (profiling runs)")
    ap.add_argument("--forms", default="plain,batched,served,heuristic")
    ap.add_argument("--heur", default=None,
                    help="heuristic form: rerank_n,batch_size,eps,beta (Alg. 1)")
    ap.add_argument("--served-rates", default=None,
                    help="offered loads of the served form, million queries/s")
    ap.add_argument("--served-seconds", type=float, default=None,
                    help="arrival window per offered load")
    ap.add_argument("--lut16", action="store_true",
                    help="half-precision distance table (binary16 entries, float32 sums)")
    ap.add_argument("--split", type=int, default=0,
                    help="batched form: this work split instead of the autotuner's")
    ap.add_argument("--tile", type=int, default=65536, help="with --split: entries per item")
    ap.add_argument("--lm", default="",
                    help="with --split: list-major alpha,rows,blocks[,min_rows] instead of "
                         "per-query only")
    ap.add_argument("--page-bytes", type=int, default=4096,
                    help="host_raw form: bytes per page of the host-memory raw tier")
    ap.add_argument("--build-only", action="store_true")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="first run one device-to-device copy of this size (counter calibration)")
    args = ap.parse_args()
    known = {"plain", "batched", "served", "heuristic", "host_raw"}
    names = [f for f in args.forms.split(",") if f]
    if not set(names) <= known:
        ap.error(f"--forms: unknown form(s) {sorted(set(names) - known)}")
    if not set(names) - {"served"}:
        ap.error("--forms: the stage times and the roofline need plain, batched or heuristic too")
    for key, v in WORKLOAD_DEFAULTS.get(args.workload, WORKLOAD_DEFAULTS["ivf_u8_10m"]).items():
        if getattr(args, key) is None:
            setattr(args, key, v)
    return args


def run_served(ann, g, Qh, npq, w, k, n, args):
    """Served form: Poisson request arrivals (sizes U{1..256}) at several
    offered loads into a continuous-batching server; per load the achieved
    queries/s and the p50/p99 request latency, then a saturation run (every
    request waiting at once).  A load is sustained when it achieves at least
    95% of the offered rate with a p99 latency at most ten times the p50 of
    the lightest load.  The form's qps is the best sustained rate or the
    saturation rate, whichever is higher."""
    import queue
    import threading

    import numpy as np

    nq = Qh.shape[0]
    fixed_np = isinstance(w.nprobe, int)
    np_all = np.full(nq, int(w.nprobe), np.int32) if fixed_np else npq.astype(np.int32)
    srv = ann.Server(g, hbm_budget_bytes=4 << 30, max_slots=4, max_batch=1024,
                     max_nprobe=int(np_all.max()), max_k=k, max_rerank_n=n)
    rng = np.random.default_rng(1_000_003 * 2 + 7)

    def play(arrivals, sizes):
        tickets = queue.Queue()
        done = {"q": 0, "t_end": 0.0}

        def collect():
            while True:
                t = tickets.get()
                if t is None:
                    break
                srv.poll(t, wait=True)
            done["t_end"] = time.perf_counter()

        th = threading.Thread(target=collect)
        th.start()
        pos = 0
        t0 = time.perf_counter()
        for a, sz in zip(arrivals, sizes):
            while True:
                dt = t0 + a - time.perf_counter()
                if dt <= 0:
                    break
                if dt > 3e-4:
                    time.sleep(dt - 2e-4)
            rows = (np.arange(pos, pos + sz) % nq)
            pos += sz
            tickets.put(srv.submit(Qh[rows], np_all[rows], k, n))
        tickets.put(None)
        th.join()
        return done["t_end"] - t0, pos

    # warm-up (kernels of every launch shape, pinned pages): a burst, then a
    # short stream of single arrivals of mixed sizes, none of it measured
    play(np.zeros(8), [256] * 8)
    wr = np.random.default_rng(17)
    play(np.cumsum(wr.exponential(1.0, size=400)) * 5e-4, wr.integers(1, 257, size=400))
    srv.stats(reset=True)
    loads = []
    for rate_m in [float(x) for x in args.served_rates.split(",") if x]:
        lam = rate_m * 1e6
        nreq = max(8, int(lam * args.served_seconds / 128.5))
        sizes = rng.integers(1, 257, size=nreq)
        gaps = rng.exponential(1.0, size=nreq) * (sizes.mean() / lam)
        arrivals = np.cumsum(gaps) - gaps[0]
        el, nqs = play(arrivals, sizes)
        st = srv.stats(reset=True)
        ach = nqs / el
        loads.append({"offered_qps": lam, "achieved_qps": round(ach, 1),
                      "p50_ms": round(st["latency_p50_ms"], 3),
                      "p99_ms": round(st["latency_p99_ms"], 3),
                      "requests": int(st["requests_done"]), "launches": int(st["launches"]),
                      "mean_launch_queries": round(st["queries_done"] / max(1, st["launches"]), 1),
                      "max_in_flight": int(st["max_in_flight"]),
                      "sustained": bool(ach >= 0.95 * lam)})
        if len(loads) == 1:
            p99_bound = 10.0 * loads[0]["p50_ms"]
        loads[-1]["p99_bound_ms"] = round(p99_bound, 3)
        loads[-1]["sustained"] = bool(loads[-1]["sustained"] and loads[-1]["p99_ms"] <= p99_bound)
        log(f"served @ {rate_m:g}M q/s offered: {ach:.0f} q/s, p50 {st['latency_p50_ms']:.2f} ms, "
            f"p99 {st['latency_p99_ms']:.2f} ms, {st['launches']} launches")
    # saturation: all requests waiting at once
    sizes = rng.integers(1, 257, size=max(8, int(3 * nq / 128.5)))
    el, nqs = play(np.zeros(len(sizes)), sizes)
    st = srv.stats(reset=True)
    sat = {"achieved_qps": round(nqs / el, 1), "p50_ms": round(st["latency_p50_ms"], 3),
           "p99_ms": round(st["latency_p99_ms"], 3), "launches": int(st["launches"]),
           "mean_launch_queries": round(st["queries_done"] / max(1, st["launches"]), 1),
           "max_in_flight": int(st["max_in_flight"]), "queries": int(nqs)}
    log(f"served saturation: {nqs / el:.0f} q/s over {nqs} queries, {st['launches']} launches")
    srv.stop()
    best = max([x["achieved_qps"] for x in loads if x["sustained"]] + [sat["achieved_qps"]])
    return {"qps": best, "ms_per_step": nq / best * 1e3, "loads": loads, "saturation": sat,
            "max_slots": 4, "max_batch": 1024, "request_sizes": "U{1..256}",
            "arrivals": "Poisson"}


def run_host_raw(ann, path, Q, nprobe_arg, k, n, opts, args, out, heur):
    """The search with the raw vectors kept in pinned host memory on pages
    (Sec. 4.3 layout; raw_tier 1): the same tuned batched search, with step 8
    reading whole pages over PCIe -- each page once per query, shared by its
    candidates on it.  Reports queries/s, pages read per query and the PCIe
    bytes they move, for the fixed re-rank and the heuristic one (Alg. 1)."""
    import numpy as np
    import torch

    t0 = time.time()
    gh = ann.Index(path, 0, raw_tier=1, page_bytes=args.page_bytes)
    log(f"host raw tier: {gh.desc['pages']} pages of {args.page_bytes} B "
        f"({gh.desc['host_bytes'] / 2**30:.2f} GiB pinned) in {time.time() - t0:.1f}s")
    for o, v in opts.items():
        gh.set_option(o, v)
    st = torch.cuda.current_stream(Q.device)
    nq = Q.shape[0]
    res = {"page_bytes": args.page_bytes, "pages": int(gh.desc["pages"])}
    for label, (bs, eps, beta, nn) in (("fixed", (0, 0.0, 1, n)),
                                       ("heuristic", (heur[1], heur[2], heur[3], heur[0]))):
        for _ in range(max(1, args.warmup)):
            r = gh.search_pages(Q, nprobe_arg, k, nn, bs, eps, beta)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(args.steps):
            r = gh.search_pages(Q, nprobe_arg, k, nn, bs, eps, beta)
        e1.record(st)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        ids, d, rr, pr = r
        reads = float(pr.double().mean())
        item = {"ms_per_step": round(ms, 4), "qps": round(nq / (ms / 1e3), 1),
                "rerank_n": nn, "reranked_per_query": round(float(rr.double().mean()), 1),
                "page_reads_per_query": round(reads, 1),
                "pcie_gb_per_s": round(reads * nq * args.page_bytes / (ms / 1e3) / 1e9, 2)}
        ref = out.get("graph_res") if label == "fixed" else out.get("heur_res")
        if ref is not None:
            item["results_equal_hbm_tier"] = bool(torch.equal(ids, ref[0]) and
                                                  torch.equal(d.view(torch.int32),
                                                              ref[1].view(torch.int32)))
        res[label] = item
        log(f"host raw tier, {label}: {ms:.3f} ms/step, {item['qps']:.0f} q/s, "
            f"{reads:.1f} pages per query, {item['pcie_gb_per_s']} GB/s over PCIe")
    gh.close()
    res["qps"] = res["fixed"]["qps"]
    res["ms_per_step"] = res["fixed"]["ms_per_step"]
    return res


def run_diff(args):
    """Differentiable PQ distance on the differentiation workload: 1M x 96-d
    float32 (1024-centre Gaussian mixture, centres U[0,100]^96, sigma 5), PQ 24
    x 256 x 4-d trained on a seeded sample, codes fixed; batches of 4096 queries
    x 2048 candidates.  Times forward + backward (dL/dcodebooks and dL/dqueries
    of L = mean (Dhat - exact)^2) per batch, reports pairs/s and the fp32 MFMA
    rate of the backward's two GEMMs, then fine-tunes the codebooks and
    reports the distortion and the ADC recall before and after."""
    import numpy as np
    import torch

    from paper_2409_16576_amd import ann, builder, finetune, inputs

    wid, n, dim, M = 4, 1_000_000, 96, 24
    t0 = time.time()
    C0 = inputs.mixture_centres(inputs.seed_for(wid, 1), 1024, dim, 0.0, 100.0)
    X = inputs.mixture_points(inputs.seed_for(wid, 2), n, C0, 5.0, "f32")
    Qh = inputs.mixture_points(inputs.seed_for(wid, 3), 16384, C0, 5.0, "f32")
    p = builder.BuildParams(nlist=1, M=M, seed=inputs.seed_for(wid, 5))
    CB = builder.train_pq(X, "f32", p)
    codes = builder.encode_pq(X, CB)
    log(f"diff workload ready in {time.time() - t0:.1f}s")
    dev = torch.device("cuda", 0)
    B, Cn = 4096, 2048
    rng = np.random.default_rng(inputs.seed_for(wid, 8))
    ci = rng.choice(n, size=Cn, replace=False)
    qi = rng.choice(len(Qh), size=B, replace=False)
    Q = torch.from_numpy(Qh[qi]).to(dev)
    Xc = torch.from_numpy(X[ci]).to(dev)
    cc = torch.from_numpy(codes[ci]).to(dev)
    CBt = torch.from_numpy(CB).to(dev)
    ex = finetune.exact_sq(Q, Xc)

    def step():
        Qg = Q.clone().requires_grad_(True)
        CBg = CBt.clone().requires_grad_(True)
        d = ann.adc_distance(Qg, CBg, cc)
        g = d.detach() - ex
        d.backward(2.0 * g / g.numel())
        return Qg.grad, CBg.grad

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    st = torch.cuda.current_stream(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(args.steps):
        step()
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    # the backward alone (both GEMMs + the codeword scatter), event-timed
    Qg = Q.clone().requires_grad_(True)
    CBg = CBt.clone().requires_grad_(True)
    d = ann.adc_distance(Qg, CBg, cc)
    G = torch.randn_like(d)
    torch.cuda.synchronize()
    e0.record(st)
    for _ in range(args.steps):
        torch.autograd.grad(d, (Qg, CBg), G, retain_graph=True)
    e1.record(st)
    torch.cuda.synchronize()
    bwd_ms = e0.elapsed_time(e1) / args.steps
    gemm_flops = 2 * 2.0 * B * Cn * dim
    Qall = torch.from_numpy(Qh).to(dev)
    rows = np.sort(rng.choice(n, size=8192, replace=False))
    Xs = torch.from_numpy(X[rows]).to(dev)
    cs = torch.from_numpy(codes[rows]).to(dev)
    Qe = Qall[:1024]
    l0 = float(finetune.distortion_loss(Qe, CBt, cs, Xs))
    r0 = finetune.adc_recall(Qe, CBt, cs, Xs, k=10, n=100)
    CB1, hist = finetune.finetune_codebooks(CBt, cs, Xs, Qall[1024:], steps=50, batch_q=B,
                                            batch_c=Cn, lr=0.05, seed=1)
    l1 = float(finetune.distortion_loss(Qe, CB1, cs, Xs))
    r1 = finetune.adc_recall(Qe, CB1, cs, Xs, k=10, n=100)
    log(f"diff: {ms:.3f} ms per fwd+bwd batch, backward {bwd_ms:.3f} ms; "
        f"distortion {l0:.1f} -> {l1:.1f}, ADC recall 10@100 {r0:.3f} -> {r1:.3f}")
    achieved = gemm_flops / (bwd_ms / 1e3) / 1e12
    line = {"metric": "differentiable PQ distance, forward+backward pairs/s", "value":
            round(B * Cn / (ms / 1e3), 1), "unit": "pairs/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "diff_f32_1m", "n": n, "dim": dim, "M": M, "dsub": 4,
                       "batch_queries": B, "batch_candidates": Cn},
            "roofline": {"bound": "mfma", "achieved": round(achieved, 2), "peak": 157.3,
                         "unit": "TFLOP/s", "frac": round(achieved / 157.3, 4), "traffic": None,
                         "kernel": "backward (two fp32 MFMA GEMMs + codeword scatter)",
                         "backward_ms": round(bwd_ms, 4), "gemm_flops": gemm_flops},
            "finetune": {"steps": 50, "distortion_before": round(l0, 2),
                         "distortion_after": round(l1, 2), "recall10_at100_before": round(r0, 4),
                         "recall10_at100_after": round(r1, 4)}}
    print(json.dumps(line), flush=True)


def run_nav(args):
    """Navigation-graph probe (Sec. 4.1) at the paper's list count, where the
    exact probe stops being cheap: 2M x 100-d int8 vectors (8192-centre
    mixture), 200,000 lists (0.1 N), PQ 50 x 256; 10,000 queries, nprobe 256,
    rerank_n 200, k 10.  Builds the centroid graph (32 edges per vertex), then
    times step 2 alone and the whole search (one ann_search over the batch)
    with the exact probe and with graph walks of several beam widths, each
    bracketed by HIP events on the launch stream; reports the share of the
    exact top-nprobe lists each walk finds.  The CPU leg adds recall@10
    against exact kNN and the bit-exact parity of the GPU graph search with
    the oracle's on a query sample."""
    import numpy as np
    import torch

    from paper_2409_16576_amd import ann, builder, workloads

    w = workloads.ALL["nav_i8_2m"]
    t0 = time.time()
    path = workloads.ensure_index(w, verbose=True)
    log(f"index ready in {time.time() - t0:.1f}s")
    C = builder.read_centroids(path)
    graphs = []
    for deg, pool, gprobe in ((32, 128, 8), (64, 256, 16)):
        t0 = time.time()
        adj, entry = builder.build_nav_graph(C, deg=deg, seed=1, gprobe=gprobe, pool=pool)
        graphs.append({"deg": deg, "pool": pool, "gprobe": gprobe, "adj": adj, "entry": entry,
                       "build_s": round(time.time() - t0, 1)})
        log(f"navigation graph: {C.shape[0]} vertices, {deg} edges each (pool {pool}, "
            f"{gprobe} groups), {len(entry)} entries, {time.time() - t0:.1f}s")
    if args.build_only:
        return
    dev = torch.device("cuda", 0)
    g = ann.Index(path, 0)
    Qh = workloads.queries(w)
    Q = torch.from_numpy(Qh).to(dev)
    nq, npr, k, n = len(Qh), int(w.nprobe), w.k, w.rerank_n
    st = torch.cuda.current_stream(dev)

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(reps):
            out = fn()
        e1.record(st)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps, out

    reps = max(1, args.steps)
    g.set_option(g.OPT_PROBE_BEAM, 0)
    p_ms, (ex_lists, _) = timed(lambda: g.probe(Q, npr, with_dists=False), reps)
    s_ms, (ex_ids, _) = timed(lambda: g.search(Q, npr, k, n), reps)
    exact = {"probe_ms": round(p_ms, 4), "search_ms": round(s_ms, 4),
             "qps": round(nq / (s_ms / 1e3), 1)}
    log(f"exact probe: probe {p_ms:.3f} ms, search {s_ms:.3f} ms per {nq} queries")
    exs = ex_lists.cpu().numpy()
    walks = []
    for gi_, gr in enumerate(graphs):
        g.set_nav_graph(gr["adj"], gr["entry"])
        for beam in (256, 512):
            g.set_option(g.OPT_PROBE_BEAM, beam)
            p_ms, (gl, _) = timed(lambda: g.probe(Q, npr, with_dists=False), reps)
            s_ms, (gi, _) = timed(lambda: g.search(Q, npr, k, n), reps)
            gls = gl.cpu().numpy()
            found = np.mean([len(np.intersect1d(a, b)) / npr for a, b in zip(gls, exs)])
            same10 = float((gi.cpu().numpy() == ex_ids.cpu().numpy()).mean())
            walks.append({"graph": gi_, "degree": gr["deg"], "beam": beam,
                          "probe_ms": round(p_ms, 4), "search_ms": round(s_ms, 4),
                          "qps": round(nq / (s_ms / 1e3), 1), "exact_lists_found": round(found, 4),
                          "top10_equal_exact_probe": round(same10, 4)})
            log(f"graph {gi_} (degree {gr['deg']}) beam {beam}: probe {p_ms:.3f} ms, search "
                f"{s_ms:.3f} ms, {found:.4f} of the exact lists")
    best = max(walks, key=lambda x: (x["exact_lists_found"] >= 0.9, x["qps"]))
    line = {"metric": "navigation-graph probe vs exact probe at nlist = 0.1 N, queries/s",
            "value": best["qps"], "unit": "queries/s", "n_gpus": 1, "steps": reps,
            "warmup": 1, "ms_per_step": best["search_ms"], "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "i32", "data": "synthetic",
            "config": {**w.describe(), "graphs": [{kk: vv for kk, vv in gr.items()
                                                    if kk not in ("adj", "entry")} |
                                                   {"entries": int(len(gr["entry"]))}
                                                   for gr in graphs]},
            "exact_probe": exact, "graph_probe": walks, "chosen": best}
    if not args.no_cpu:
        import oracle
        oracle.build(force=False)
        ix = oracle.read_index(path)
        m = 200
        t0 = time.time()
        truth, _ = oracle.bruteforce(ix, Qh[:m], k)
        beam, gr = best["beam"], graphs[best["graph"]]
        g.set_nav_graph(gr["adj"], gr["entry"])
        g.set_option(g.OPT_PROBE_BEAM, beam)
        gi, gd = g.search(Q[:m], npr, k, n)
        r = oracle.search(ix, Qh[:m], npr, k, n,
                          graph=oracle.NavGraph(gr["adj"], gr["entry"], beam))
        parity = {"queries": m, "graph": best["graph"], "beam": beam,
                  "ids_equal": bool(np.array_equal(gi.cpu().numpy(), r.ids)),
                  "dists_equal": bool(np.array_equal(gd.cpu().numpy().view(np.int32),
                                                     r.dists.view(np.int32)))}
        g.set_option(g.OPT_PROBE_BEAM, 0)
        ei, _ = g.search(Q[:m], npr, k, n)
        rec = {"exact_probe": round(oracle.recall_at_k(ei.cpu().numpy(), truth, k), 4)}
        for wk in walks:
            gr = graphs[wk["graph"]]
            g.set_nav_graph(gr["adj"], gr["entry"])
            g.set_option(g.OPT_PROBE_BEAM, wk["beam"])
            gi, _ = g.search(Q[:m], npr, k, n)
            wk["recall_at_10"] = round(oracle.recall_at_k(gi.cpu().numpy(), truth, k), 4)
            rec[f"graph{wk['graph']}_beam{wk['beam']}"] = wk["recall_at_10"]
        line["recall_at_10"] = rec
        line["parity_sample"] = parity
        log(f"recall@10 {rec}, parity {parity} ({time.time() - t0:.1f}s)")
    g.close()
    print(json.dumps(line), flush=True)


def run_repl(args):
    """How the replication of Eq. 2 (and balanced clustering) drives the
    filtering stage's work: 4M x 100-d int8 vectors (4096-centre mixture),
    8192 lists, PQ 50 x 256, 10,000 queries, nprobe 32, rerank_n 200, k 10.
    Centroids and PQ are trained once; each variant re-assigns the vectors on
    the GPU (exact R nearest lists, Eq. 2 with eps) and writes its own index:
    R = 1, 2, 4, 8 at eps 0.1, R = 8 at eps 0.3, and R = 2 with hierarchical
    balanced clustering.  Per variant: list entries per vector, list-size
    spread, per query the list entries gathered, the replica entries the scan
    walks (the rest are skipped whole by the ownership rule) and the distinct
    candidates scored, the search time of one ann_search over the batch
    (HIP events), and recall@10 against exact kNN on a query sample."""
    import numpy as np
    import torch

    from paper_2409_16576_amd import ann, builder, inputs, workloads

    w = workloads.ALL["repl_i8_4m"]
    t0 = time.time()
    X = workloads.base_vectors(w)
    Qh = workloads.queries(w)
    log(f"data ready in {time.time() - t0:.1f}s")
    base = workloads.build_params(w)
    C, hier = builder.train_ivf(X, w.kind, base)
    CB = builder.train_pq(X, w.kind, base)
    codes = builder.encode_pq(X, CB)
    log(f"centroids and PQ trained in {time.time() - t0:.1f}s")
    variants = [("R1", 1, 0.1, 0.0), ("R2", 2, 0.1, 0.0), ("R4", 4, 0.1, 0.0),
                ("R8", 8, 0.1, 0.0), ("R8_eps0.3", 8, 0.3, 0.0), ("R2_balanced", 2, 0.1, 0.1)]
    dev = torch.device("cuda", 0)
    Q = torch.from_numpy(Qh).to(dev)
    nq, npr, k, n = len(Qh), int(w.nprobe), w.k, w.rerank_n
    st = torch.cuda.current_stream(dev)
    truth = None
    out = []
    tmpd = workloads.cache_dir()
    Cb = None
    for name, R, eps, bal in variants:
        t1 = time.time()
        Cv = C
        if bal > 0:
            if Cb is None:
                pb = workloads.build_params(w)
                pb.balance = bal
                Cb, _ = builder.train_ivf(X, w.kind, pb)
            Cv = Cb
        A = builder.assign_lists_gpu(X, Cv, w.kind, R, eps)
        off, ent = builder.lists_from_assignment(A, w.nlist)
        path = os.path.join(tmpd, f"repl_{name}.fidx")
        builder.write_index(path, builder.IndexArrays(w.kind, Cv, CB, codes, X, off, ent, A, eps,
                                                      True))
        sizes = np.diff(off)
        prim = np.bincount(A[:, 0], minlength=w.nlist)
        g = ann.Index(path, 0)
        ids, dd = g.search(Q, npr, k, n)  # warm-up
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = max(1, args.steps)
        e0.record(st)
        for _ in range(reps):
            ids, dd = g.search(Q, npr, k, n)
        e1.record(st)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        _, _, nc, nw = g.search_topn(Q, npr, n, walked=True)
        nc, nw = nc.cpu().numpy(), nw.cpu().numpy()
        # list entries gathered per query (with duplicates), from the probe
        lists, _ = g.probe(Q, npr, with_dists=False)
        ls = lists.cpu().numpy()
        gathered = np.where(ls >= 0, sizes[np.maximum(ls, 0)], 0).sum(1)
        first = np.where(ls >= 0, prim[np.maximum(ls, 0)], 0).sum(1)
        rec = {"name": name, "R": R, "eps": eps, "balanced": bal,
               "entries_per_vector": round(float(len(ent) / w.n), 4),
               "list_size": {"max": int(sizes.max()), "median": float(np.median(sizes)),
                             "p99": float(np.percentile(sizes, 99))},
               "per_query": {"entries_gathered": round(float(gathered.mean()), 1),
                             "replica_entries_listed": round(float((gathered - first).mean()), 1),
                             "replica_entries_walked": round(float((nw - first).mean()), 1),
                             "candidates_scored": round(float(nc.mean()), 1)},
               "search_ms": round(ms, 4), "qps": round(nq / (ms / 1e3), 1),
               "build_s": round(time.time() - t1, 1)}
        if not args.no_cpu:
            import oracle
            oracle.build(force=False)
            m = 200
            if truth is None:
                ix0 = oracle.read_index(path)
                truth, _ = oracle.bruteforce(ix0, Qh[:m], k)
            rec["recall_at_10"] = round(oracle.recall_at_k(ids[:m].cpu().numpy(), truth, k), 4)
        g.close()
        os.remove(path)
        out.append(rec)
        log(f"replication {rec}")
    base_ms = out[0]["search_ms"]
    line = {"metric": "replication study: search time and dedup work per query vs Eq. 2's R",
            "value": out[1]["qps"], "unit": "queries/s", "n_gpus": 1, "steps": max(1, args.steps),
            "warmup": 1, "ms_per_step": out[1]["search_ms"], "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "i32", "data": "synthetic",
            "config": w.describe(), "variants": out,
            "search_time_vs_R1": {r["name"]: round(r["search_ms"] / base_ms, 3) for r in out}}
    print(json.dumps(line), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}): the search path "
              "runs on a single MI355X and uses no collectives.", file=sys.stderr)
        sys.exit(2)

    import numpy as np

    from paper_2409_16576_amd import builder, workloads

    if args.workload == "diff_f32_1m":
        return run_diff(args)
    if args.workload == "nav_i8_2m":
        return run_nav(args)
    if args.workload == "repl_i8_4m":
        return run_repl(args)
    w = workloads.ALL[args.workload]
    t0 = time.time()
    path = workloads.ensure_index(w, verbose=True)
    log(f"index ready in {time.time() - t0:.1f}s: {path}")
    if args.build_only:
        return

    import torch

    from paper_2409_16576_amd import ann

    dev = torch.device("cuda", 0)
    if args.copy_calibration_mib:
        nb = args.copy_calibration_mib << 20
        src = torch.ones(nb, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy of {nb} bytes done")
        del src, dst
    t0 = time.time()
    g = ann.Index(path, 0)
    log(f"index loaded to HBM in {time.time() - t0:.1f}s, {g.desc['hbm_bytes'] / 2**30:.2f} GiB")
    if args.lut16:
        g.set_option(g.OPT_LUT_F16, 1)
    Qh = workloads.queries(w)
    nq = Qh.shape[0]
    Q = torch.from_numpy(Qh).to(dev)
    npq = workloads.nprobe_per_query(w)
    fixed_np = isinstance(w.nprobe, int)
    nprobe_arg = int(w.nprobe) if fixed_np else torch.from_numpy(npq).to(dev)
    k = w.k
    n = args.rerank_n or w.rerank_n_op or w.rerank_n
    st = torch.cuda.current_stream(dev)

    # ---- work counts (untimed): candidates scored and list entries walked.
    # A probed list's first-list members are a contiguous row range (no ID is
    # read); its replica entries (8 B each) are walked unless their whole
    # group is skipped because the group's first list is probed too.
    _, _, ncand, nwalk = g.search_topn(Q, nprobe_arg, n, walked=True)
    lists, _ = g.probe(Q, nprobe_arg, with_dists=False)
    torch.cuda.synchronize()
    ncand = ncand.cpu().numpy()
    nwalk = nwalk.cpu().numpy()
    lists = lists.cpu().numpy()
    sizes, primary = builder.read_list_meta(path)
    valid = lists >= 0
    lsafe = np.where(valid, lists, 0)
    entries_q = (sizes[lsafe] * valid).sum(1)
    prim_q = (primary[lsafe] * valid).sum(1)
    rep_q = entries_q - prim_q
    rep_walked = int((nwalk - prim_q).sum())
    cand_per_step = int(ncand.sum())
    # algorithmic bytes of the scan: M code bytes per scored candidate and a
    # 4-byte ID per replica entry walked (first-list members are a row range:
    # no ID read); the distance table is built on chip and not counted
    M = g.desc["m"]
    scan_alg_bytes = cand_per_step * M + rep_walked * 4
    log(f"per step: {cand_per_step} candidates, {int(entries_q.sum())} list entries "
        f"({int(rep_q.sum())} replica), {int(nwalk.sum())} walked ({rep_walked} replica); "
        f"scan algorithmic bytes {scan_alg_bytes / 1e9:.2f} GB")

    def step_plain():
        for b0 in range(0, nq, args.plain_batch):
            b1 = min(nq, b0 + args.plain_batch)
            npb = nprobe_arg if fixed_np else nprobe_arg[b0:b1]
            g.search(Q[b0:b1], npb, k, n)

    out = {}
    graph = None
    tuned = None

    def step_eager():
        out["res"] = g.search(Q, nprobe_arg, k, n)

    def step_graph():
        out["graph_res"] = graph.launch(st)

    hn, hb, heps, hbeta = (float(x) for x in args.heur.split(","))
    hn, hb, hbeta = int(hn), int(hb), int(hbeta)

    def step_heur():
        out["heur_res"] = g.search_heuristic(Q, nprobe_arg, k, hn, hb, heps, hbeta)

    forms = {"plain": step_plain, "batched": step_graph, "batched_eager": step_eager,
             "heuristic": step_heur}
    names = args.forms.split(",")
    # tuning options (none changes results): the index's defaults for the
    # plain form, the autotuner's choice for the batched form
    OPTS = (g.OPT_SCAN_TILE, g.OPT_SCAN_SPLIT, g.OPT_LIST_MAJOR, g.OPT_LM_ALPHA, g.OPT_LM_TILE,
            g.OPT_LM_BLOCKS, g.OPT_LM_MIN_ROWS)

    def get_opts():
        return {o: g.get_option(o) for o in OPTS}

    def set_opts(d):
        for o, v in d.items():
            g.set_option(o, v)

    default_opts = get_opts()
    if "batched" in names:
        # the batched form: options picked by the autotuner for this batch (or
        # a given per-query split), then the whole search captured once into a
        # HIP graph; its stage times (and the roofline) come from an eager,
        # event-bracketed run of the same search right after
        if args.split:
            g.set_option(g.OPT_SCAN_TILE, args.tile)
            g.set_option(g.OPT_SCAN_SPLIT, args.split)
            tuned = {"tile": args.tile, "split": args.split, "tried": 0, "ms": 0.0,
                     "list_major": 0}
            if args.lm:
                la, lt, lb, *lmin = (int(x) for x in args.lm.split(","))
                lmin = lmin[0] if lmin else 0
                for o, v in ((g.OPT_LIST_MAJOR, 1), (g.OPT_LM_ALPHA, la), (g.OPT_LM_TILE, lt),
                             (g.OPT_LM_BLOCKS, lb), (g.OPT_LM_MIN_ROWS, lmin)):
                    g.set_option(o, v)
                tuned.update(list_major=1, lm_alpha=la, lm_tile=lt, lm_blocks=lb,
                             lm_min_rows=lmin)
        else:
            tuned = ann.autotune(g, Q, nprobe_arg, k, n, reps=2)
        log(f"autotuned: {tuned}")
        graph = ann.Graph(g, Q, nprobe_arg, k, n)
        names.insert(names.index("batched") + 1, "batched_eager")
    batched_opts = get_opts()
    results = {}
    for name in names:
        if name == "host_raw":
            results[name] = run_host_raw(ann, path, Q, nprobe_arg, k, n, batched_opts, args, out,
                                         (hn, hb, heps, hbeta))
            continue
        if name == "served":  # the server launches with the tuned work split
            set_opts({**batched_opts, g.OPT_LIST_MAJOR: 0})
            results[name] = run_served(ann, g, Qh, npq, w, k, n, args)
            continue
        fn = forms[name]
        set_opts(batched_opts if name.startswith("batched") or name == "heuristic"
                 else default_opts)
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        g.set_profiling(True)
        g.get_profile(reset=True)
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record(st)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            fn()
        ev1.record(st)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms = ev0.elapsed_time(ev1) / args.steps
        prof = g.get_profile(reset=True)
        g.set_profiling(False)
        if name == "batched":  # graph launches carry no stage events
            prof = {s_: {"ms": 0.0, "launches": 0} for s_ in prof}
        results[name] = {"ms_per_step": ms, "qps": nq / (ms / 1e3),
                         "candidates_per_s": cand_per_step / (ms / 1e3),
                         "wall_ms_per_step": wall * 1e3 / args.steps,
                         "stage_ms_per_step": {s: v["ms"] / args.steps for s, v in prof.items()},
                         "stage_launches_per_step": {s: v["launches"] // args.steps
                                                     for s, v in prof.items()}}
        log(f"{name}: {ms:.3f} ms/step, {results[name]['qps']:.0f} q/s, "
            f"{results[name]['candidates_per_s'] / 1e9:.2f} G cand/s, stages "
            + ", ".join(f"{s} {v['ms'] / args.steps:.3f}ms" for s, v in prof.items()))

    if "plain" in results:
        # latency of single-query calls (plain form, batch of one): each call is
        # timed from submission to completion on the host clock
        set_opts(default_opts)
        lat = []
        for i in range(220):
            npb = nprobe_arg if fixed_np else nprobe_arg[i % nq:i % nq + 1]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            g.search(Q[i % nq:i % nq + 1], npb, k, n)
            torch.cuda.synchronize()
            if i >= 20:
                lat.append((time.perf_counter() - t0) * 1e3)
        lat = np.array(lat)
        results["plain"]["batch1_latency_ms"] = {
            "p50": round(float(np.percentile(lat, 50)), 4),
            "p99": round(float(np.percentile(lat, 99)), 4),
            "mean": round(float(lat.mean()), 4), "calls": int(lat.size)}
        log(f"plain, one query per call: p50 {np.percentile(lat, 50):.3f} ms, "
            f"p99 {np.percentile(lat, 99):.3f} ms")

    head = "batched" if "batched" in results else [f for f in results if f != "served"][0]
    R = results[head]
    RS = results["batched_eager"] if head == "batched" else R  # stage times (events)
    st_ms, st_n = RS["stage_ms_per_step"], RS["stage_launches_per_step"]
    lm_on = head == "batched" and batched_opts[g.OPT_LIST_MAJOR] == 1
    lm = None
    if lm_on:
        # the list-major pass's work, from the probe lists and the same split
        # rule the kernels apply (first-list rows of each query's leading lists
        # until alpha * n rows stay with the per-query scan, and those of lists
        # shorter than min_rows)
        alpha = batched_opts[g.OPT_LM_ALPHA]
        npv = valid.sum(1)
        plen = np.where(valid, primary[lsafe], 0)
        csum = np.cumsum(plen, axis=1)
        reach = csum >= alpha * n
        first = np.where(reach.any(1), reach.argmax(1) + 1, lists.shape[1])
        walkp = np.minimum(first, npv)
        slot = np.arange(lists.shape[1])[None, :]
        min_rows = batched_opts[g.OPT_LM_MIN_ROWS]
        in2 = valid & (slot >= walkp[:, None]) & (plen > 0) & (plen >= min_rows)
        cnt_l = np.bincount(lists[in2], minlength=len(primary))
        G = 16 if g.desc["int_grid"] else (8 if args.lut16 else 4)
        groups = (cnt_l + G - 1) // G
        lm = {"pairs_per_step": int((plen * in2).sum()),
              "rows_distinct_per_step": int(primary[cnt_l > 0].sum()),
              "rows_read_per_step": int((groups * primary).sum()),
              "query_groups_per_step": int(groups.sum()), "alpha": int(alpha)}
        log(f"list-major: {lm}")
    # dominant kernel: the per-query scan or the list-major launch
    kern = "scan"
    if lm_on and st_ms.get("list_major", 0.0) > st_ms["scan"]:
        kern = "list_major"
    launches = max(1, st_n[kern])
    if kern == "scan":
        cand_q = cand_per_step - (lm["pairs_per_step"] if lm else 0)
        alg_bytes = cand_q * M + rep_walked * 4
        kname = "k_scan (fused gather/dedup/Eq.1/top-n)"
        extra = {"replica_entries_walked_per_step": rep_walked,
                 "replica_entries_listed_per_step": int(rep_q.sum()),
                 "candidates_scored_per_step": cand_q}
    else:
        # each probed list's code rows read once (M bytes a row)
        alg_bytes = lm["rows_distinct_per_step"] * M
        kname = ("k_lm_mfma (list-major decode + int8 MFMA Eq. 1 + threshold)"
                 if g.desc["int_grid"] else
                 "k_lm_lut (list-major Eq. 1 by interleaved LDS tables + threshold)")
        extra = dict(lm)
    # bytes per launch / average launch time = bytes per step / kernel time per step
    achieved = alg_bytes / (st_ms[kern] / 1e3) / 1e9
    tr = load_traffic(kern, w.name)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": (tr["bytes_per_launch"] if tr else None),
                "kernel": kname, "stage": kern,
                "ms_per_launch": round(st_ms[kern] / launches, 4),
                "launches_per_step": launches,
                "algorithmic_bytes_per_launch": alg_bytes // launches, **extra}

    line = {
        "metric": METRIC, "value": round(R["qps"], 1), "unit": "queries/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(R["ms_per_step"], 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {**w.describe(), "rerank_n": n, "rerank_n_config": w.rerank_n,
                   "data_dtype": w.kind, "form": head, "plain_batch": args.plain_batch,
                   "lut": "f16" if args.lut16 else "f32"},
        "candidates_per_s": round(R["candidates_per_s"], 1),
        "candidates_per_query": round(cand_per_step / nq, 1),
        "forms": {k_: {kk: (round(v, 4) if isinstance(v, float) else v) for kk, v in r.items()}
                  for k_, r in results.items()},
        "roofline": roofline,
    }
    if tuned:
        line["config"]["tuned"] = {kk: vv for kk, vv in tuned.items() if kk not in ("ms", "tried")}
    if "plain" in results and "batched" in results:
        line["batched_over_plain"] = round(results["batched"]["qps"] / results["plain"]["qps"], 3)
    if "plain" in results and "served" in results:
        line["served_over_plain"] = round(results["served"]["qps"] / results["plain"]["qps"], 3)
    if "heuristic" in results:
        rr = out["heur_res"][2].float()
        results["heuristic"]["params"] = {"rerank_n": hn, "batch_size": hb, "eps": heps,
                                          "beta": hbeta}
        results["heuristic"]["mean_reranked"] = round(float(rr.mean()), 1)
        line["forms"]["heuristic"] = {kk: (round(v, 4) if isinstance(v, float) else v)
                                      for kk, v in results["heuristic"].items()}

    if not args.no_cpu:
        import oracle

        log("oracle leg: reading the index on the host")
        oracle.build(force=False)
        oracle.use_native()  # -march=native copy for this host (same arithmetic)
        oix = oracle.read_index(path, verify=False)
        # the host's CPU share for this GPU (OMP_NUM_THREADS where the host sets it)
        threads = min(len(os.sched_getaffinity(0)),
                      int(os.environ.get("OMP_NUM_THREADS") or 0) or 1 << 30) or 1
        ns = min(args.cpu_queries, nq)
        t0 = time.perf_counter()
        r = oracle.search(oix, Qh[:ns], npq[:ns], k, n, threads=threads, lut_f16=args.lut16)
        cpu_s = time.perf_counter() - t0
        log(f"oracle: {ns} queries in {cpu_s:.2f}s on {threads} threads")
        # parity of the headline form's own output (the graph's), else an eager search
        ids_gpu, d_gpu = out.get("graph_res") or out.get("res") or g.search(Q, nprobe_arg, k, n)
        ids_gpu = ids_gpu[:ns].cpu().numpy()
        d_gpu = d_gpu[:ns].cpu().numpy()
        line["parity_sample"] = {"queries": ns, "ids_equal": bool(np.array_equal(ids_gpu, r.ids)),
                                 "dists_equal": bool(np.array_equal(d_gpu, r.dists))}
        line["cpu_baseline"] = {"value": round(ns / cpu_s, 1), "unit": "queries/s",
                                "cores": threads, "kind": "oracle",
                                "sample": f"first {ns} of {nq} queries, full index, same knobs",
                                "candidates_per_s": round(float(r.ncand.sum()) / cpu_s, 1)}
        # the same oracle on one thread, on a smaller sample
        n1 = max(1, ns // max(1, threads) // 2)
        t0 = time.perf_counter()
        oracle.search(oix, Qh[:n1], npq[:n1], k, n, threads=1, lut_f16=args.lut16)
        cpu1_s = time.perf_counter() - t0
        line["cpu_baseline"]["one_thread"] = {"value": round(n1 / cpu1_s, 2), "unit": "queries/s",
                                              "sample": f"first {n1} queries"}
        log(f"oracle, one thread: {n1} queries in {cpu1_s:.2f}s")
        nr = min(args.recall_queries, nq)
        t0 = time.perf_counter()
        gt, _ = oracle.bruteforce(oix, Qh[:nr], k, threads=threads)
        log(f"brute force of {nr} queries in {time.perf_counter() - t0:.1f}s")
        line["recall_at_10"] = round(oracle.recall_at_k(ids_gpu[:nr], gt, k), 4)
        line["recall_queries"] = nr
        # Per-query minimum re-ranking number (the paper's Sec. 2.3 study): a
        # query's exact top-k comes out of re-ranking its top-n ADC candidates
        # once all k true neighbours are among them, i.e. from n = 1 + the
        # largest ADC rank of a true neighbour (never, when one lies outside
        # the probed lists).  Ranks from the GPU's top-4096 ADC candidates.
        nmax = min(4096, g.desc["max_rerank_n"])
        tids, _, _ = g.search_topn(Q[:nr], nprobe_arg if fixed_np else nprobe_arg[:nr], nmax)
        tids = tids.cpu().numpy()
        need = np.full(nr, np.inf)
        for i in range(nr):
            pos = {int(v): r_ for r_, v in enumerate(tids[i]) if v >= 0}
            rk = [pos.get(int(v), None) for v in gt[i][:k]]
            if all(x is not None for x in rk):
                need[i] = 1 + max(rk)
        grid = [10, 20, 40, 100, 200, 400, 1000, 2000, 4096]
        line["min_rerank_n"] = {
            "queries": nr, "n_max": nmax,
            "share_exact_at_n": {str(x): round(float((need <= x).mean()), 4) for x in grid},
            "never": round(float(np.isinf(need).mean()), 4),
            "median": (float(np.median(need)) if np.isfinite(np.median(need)) else None),
            "p90": (float(np.percentile(need, 90)) if np.isfinite(np.percentile(need, 90))
                    else None)}
        log(f"minimum re-ranking number: {line['min_rerank_n']}")
        if "heur_res" in out:
            hid = out["heur_res"][0][:nr].cpu().numpy()
            line["forms"]["heuristic"]["recall_at_10"] = round(oracle.recall_at_k(hid, gt, k), 4)
            rh = oracle.search(oix, Qh[:nr], npq[:nr], k, hn, threads=threads,
                               lut_f16=args.lut16, heuristic=(hb, heps, hbeta))
            line["forms"]["heuristic"]["parity_sample"] = {
                "queries": nr, "ids_equal": bool(np.array_equal(hid, rh.ids)),
                "dists_equal": bool(np.array_equal(out["heur_res"][1][:nr].cpu().numpy(), rh.dists)),
                "reranked_equal": bool(np.array_equal(
                    out["heur_res"][2][:nr].cpu().numpy().astype(np.int64), rh.reranked))}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
