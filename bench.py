#!/usr/bin/env python3
"""Benchmark of the ternary EVP search path on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload large|mid|small]

Workload (default "large"): a database of N = 10,000,000 l2-normalised
d = 1024 float32 embeddings from the seeded 4,096-component anisotropic
Gaussian mixture, encoded on the GPU to {256,1024} EVP codes (256 bytes per
vector, 2.56 GB resident), and 10,000 queries of the same mixture; k = 10.
A step is one batch of 100 queries through the whole query path: tq_encode of
the float queries, then tq_search_knn on the plain path (one full database
scan per query, the paper's "exhaustive queries") with top-k; the float
queries are already resident in HBM when timing starts.

Prints one JSON line: queries/s, the roofline of the scan kernel (algorithmic
bytes per launch / measured launch time, against 8 TB/s HBM), recall@10
against an exact FP64 cosine ground truth, and the CPU oracle timed on a
bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
METRIC = "queries/sec + HBM GB/s (% peak) at recall@10; p50/p99 latency served vs plain"


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--workload", default="large", choices=["small", "mid", "large"])
    p.add_argument("--x", type=int, default=0, help="EVP x (default: the workload's)")
    p.add_argument("--k", type=int, default=0, help="neighbours per query of the timed steps (default: the workload's)")
    p.add_argument("--batch", type=int, default=100, help="queries per step")
    p.add_argument("--path", default="plain", choices=["plain", "batched", "auto"])
    p.add_argument("--engine", default="matrix", choices=["matrix", "popcount"],
                   help="batched path: engine timed by --path batched")
    p.add_argument("--grid", type=int, default=0)
    p.add_argument("--recall-queries", type=int, default=100)
    p.add_argument("--rerank", type=int, default=512,
                   help="refine the top-N Delta candidates of the recall queries with the float vectors "
                        "(keeps the float database resident on the GPU); 0 = off")
    p.add_argument("--sparse-x", type=int, default=-1,
                   help="x of a second database (same vectors) scanned with the index-list engine; "
                        "-1 = d/32, 0 = off")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-sample-rows", type=int, default=1 << 20)
    p.add_argument("--cpu-sample-queries", type=int, default=160)
    p.add_argument("--copy-probe", action="store_true",
                   help="also run a plain 1 GiB device copy (reference for HBM byte counters)")
    p.add_argument("--no-batching", action="store_true", help="skip the batching workload")
    p.add_argument("--batches", type=int, default=500)
    p.add_argument("--no-serving", action="store_true", help="skip the serving workload")
    p.add_argument("--no-mid", action="store_true", help="skip the mid-workload x sweep")
    p.add_argument("--serve-requests", type=int, default=2000, help="requests per arrival rate")
    p.add_argument("--serve-segments", type=int, default=0, help="database segments per pass (0: library default)")
    return p.parse_args()


def pct(v, q):
    return float(np.percentile(np.asarray(v, dtype=np.float64), q)) if len(v) else None


def run_batching(tq, torch, db, queries, x, n, W, plain_qps, args, log):
    """Batching workload: seeded batches of U{1..1024} queries with k in {1,10,100}
    on the batched path (autotuned shapes, one hipGraph per batch-size bucket)."""
    from workloads import datagen
    dev = queries.device
    batches = datagen.batch_stream(args.batches, 1024, (1, 10, 100))
    t0 = time.time()
    tq.tq_autotune(db, 1024, [1, 10, 100])
    tune_s = time.time() - t0
    nq_pool = queries.shape[0]
    qc = torch.empty((1024, 2 * W), dtype=torch.int32, device=dev)
    outs = {k: (torch.empty((1024, k), dtype=torch.int32, device=dev),
                torch.empty((1024, k), dtype=torch.int32, device=dev)) for k in (1, 10, 100)}
    offs = np.cumsum([0] + [b for b, _ in batches]) % max(1, nq_pool - 1024)

    def one(i, engine=tq.TQ_ENGINE_AUTO):
        b, k = batches[i]
        q0 = int(offs[i])
        tq.tq_encode(queries[q0:q0 + b], x, qc[:b])
        ids, sc = outs[k]
        tq.tq_search_knn(db, qc[:b], k, path=tq.TQ_PATH_BATCHED, ids=ids[:b], scores=sc[:b], engine=engine)

    def stream(engine):
        # untimed: every (batch-size bucket, k) graph of this engine once
        for b in sorted({1 << j for j in range(11)}):
            for k in (1, 10, 100):
                tq.tq_search_knn(db, qc[:b], k, path=tq.TQ_PATH_BATCHED, ids=outs[k][0][:b],
                                 scores=outs[k][1][:b], engine=engine)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for i in range(len(batches)):
            one(i, engine)
        torch.cuda.synchronize()
        return time.perf_counter() - t

    dt = stream(tq.TQ_ENGINE_AUTO)
    total_q = sum(b for b, _ in batches)
    # the same stream on the popcount engine alone (the AND / popcount form of
    # the paper's b2sp), for comparison with the default engine choice
    dt_pop = stream(tq.TQ_ENGINE_POPCOUNT)
    # rooflines on the first 50 batches (direct launches, HIP events around each scan):
    # the matrix engine on the batches the tuned path gives it (k <= 128 from 16
    # queries), against the fp4 MFMA peak, and the popcount engine on all 50,
    # against the integer VALU peak
    nb = min(50, len(batches))
    d_pad = 128 * ((W * 32 + 127) // 128)  # K of the fp4 products (d padded to 128)
    on_matrix = [i for i in range(nb) if batches[i][1] <= 128 and batches[i][0] >= 16]

    def timed(engine, which):
        """HIP-event time of the scan launch(es) of each batch, in ms."""
        per = []
        tq.tq_timing_read(1, reset=True)
        tq.tq_timing_enable(True)
        for i in which:
            b, k = batches[i]
            q0 = int(offs[i])
            tq.tq_encode(queries[q0:q0 + b], x, qc[:b])
            ids, sc = outs[k]
            tq.tq_search_knn(db, qc[:b], k, path=tq.TQ_PATH_BATCHED, engine=engine, ids=ids[:b], scores=sc[:b])
            ms, _ = tq.tq_timing_read(1, reset=True)
            per.append(ms)
        tq.tq_timing_enable(False)
        return per

    per_m = timed(tq.TQ_ENGINE_MATRIX, on_matrix)
    per_p = timed(tq.TQ_ENGINE_POPCOUNT, range(nb))
    kms_m, launches_m = sum(per_m), len(per_m)
    kms_p, launches_p = sum(per_p), len(per_p)
    pairs_m = sum(batches[i][0] for i in on_matrix) * n
    pairs = sum(b for b, _ in batches[:nb]) * n
    flops = 2.0 * pairs_m * d_pad
    tflops = flops / (kms_m * 1e-3) / 1e12
    fp4_peak = 10100.0  # dense fp4 MFMA, TFLOP/s
    ops_per_pair = 5 * 4 * ((W + 3) // 4)
    valu_peak = 256 * 64 * 2.4e9 / 1e12
    tops = pairs * ops_per_pair / (kms_p * 1e-3) / 1e12
    # The bound of each batch: one pass reads the whole database (HBM floor)
    # and does 2 d_pad flops per pair (fp4 floor); a batch of b queries cannot
    # finish before the larger of the two.  Sum of the floors over the sum of
    # the measured times = the fraction of its own bound the mix reaches.
    db_bytes = n * 8 * W
    floor_m = [max(db_bytes / (HBM_PEAK_GBPS * 1e9), 2.0 * batches[i][0] * n * d_pad / (fp4_peak * 1e12)) * 1e3
               for i in on_matrix]
    hbm_bound_m = sum(1 for i in on_matrix
                      if db_bytes / (HBM_PEAK_GBPS * 1e9) >= 2.0 * batches[i][0] * n * d_pad / (fp4_peak * 1e12))
    floor_p = [max(db_bytes / (HBM_PEAK_GBPS * 1e9), batches[i][0] * n * ops_per_pair / (valu_peak * 1e12)) * 1e3
               for i in range(nb)]
    # One 1 024-query k = 10 batch on the popcount engine (16-query tiles):
    # the launch whose vector-instruction count rocprofv3 measured
    # (profiles/popcount_counters.json, valid while the kernel sources hash
    # the same).  Rates: the algorithmic count at 5 lane-ops per plane word
    # (and, xor, and, two popcount-accumulates), the same at a 6-per-word
    # estimate, the 4 instructions per word the kernel needs (the xor and the
    # second and are one three-input instruction, so the first two rates can
    # exceed the instruction peak), and the instructions the kernel actually
    # issues (SQ_INSTS_VALU x 64 lanes).
    pc = None
    q1 = queries[:1024]
    tq.tq_encode(q1, x, qc)
    ids1, sc1 = outs[10]
    tq.tq_search_knn(db, qc, 10, path=tq.TQ_PATH_BATCHED, engine=tq.TQ_ENGINE_POPCOUNT, qtile=16, ids=ids1, scores=sc1)
    tq.tq_timing_read(1, reset=True)
    tq.tq_timing_enable(True)
    for _ in range(2):
        tq.tq_search_knn(db, qc, 10, path=tq.TQ_PATH_BATCHED, engine=tq.TQ_ENGINE_POPCOUNT, qtile=16, ids=ids1,
                         scores=sc1)
    torch.cuda.synchronize()
    tq.tq_timing_enable(False)
    p_ms, p_l = tq.tq_timing_read(1, reset=True)
    p_s = p_ms / max(1, p_l) * 1e-3
    pairs1 = 1024 * n
    pc = {"kernel": "scan_batched_kernel<NC, 1, 16>", "queries": 1024, "k": 10, "avg_launch_ms": round(p_s * 1e3, 4),
          "algorithmic_5_per_word_tops": round(pairs1 * ops_per_pair / p_s / 1e12, 2),
          "algorithmic_6_per_word_tops": round(pairs1 * 6 * 4 * ((W + 3) // 4) / p_s / 1e12, 2),
          "instructions_4_per_word_tops": round(pairs1 * 4 * 4 * ((W + 3) // 4) / p_s / 1e12, 2),
          "peak_tops": round(valu_peak, 2)}
    cf = os.path.join(ROOT, "profiles", "popcount_counters.json")
    crec = json.load(open(cf)).get("scan_batched/large/k10/qt16") if os.path.exists(cf) else None
    if crec and crec.get("source_sha") == source_sha("batched_kernels.hip", "tq_device.h") and W == 32:
        issued = crec["valu_lane_ops_per_pair"] * pairs1 / p_s / 1e12
        pc.update({"issued_valu_lane_ops_per_pair": crec["valu_lane_ops_per_pair"], "issued_tops": round(issued, 2),
                   "issued_frac": round(issued / valu_peak, 4), "counters": "profiles/popcount_counters.json"})
    # consistency: a few batches against the plain path
    ok = True
    for i in (0, 7, 123):
        b, k = batches[i]
        q0 = int(offs[i])
        tq.tq_encode(queries[q0:q0 + b], x, qc[:b])
        a = tq.tq_search_knn(db, qc[:b], k, path=tq.TQ_PATH_BATCHED)
        p = tq.tq_search_knn(db, qc[:b], k, path=tq.TQ_PATH_PLAIN)
        ok &= bool(torch.equal(a[0], p[0]) and torch.equal(a[1], p[1]))
    log(f"batching: {len(batches)} batches, {total_q} queries in {dt:.2f}s (tuning {tune_s:.1f}s); "
        f"popcount engine alone {dt_pop:.2f}s")
    return {"workload": f"batching: {len(batches)} seeded batches, sizes U{{1..1024}}, k in {{1,10,100}}, "
                        f"on the N={n} d={W * 32} x={x} database",
            "queries": total_q, "seconds": round(dt, 3), "qps": round(total_q / dt, 1),
            "vs_plain": round(total_q / dt / plain_qps, 2), "autotune_s": round(tune_s, 1),
            "popcount_engine": {"seconds": round(dt_pop, 3), "qps": round(total_q / dt_pop, 1),
                                "vs_plain": round(total_q / dt_pop / plain_qps, 2)},
            "same_results_as_plain": ok,
            "roofline": {"kernel": "scan_mfma_group_kernel (k <= 16); sample pass + sample_floor_kernel + scan_mfma_kernel (k > 16)", "bound": "mfma", "achieved": round(tflops, 1),
                         "peak": fp4_peak, "unit": "TFLOP/s", "frac": round(tflops / fp4_peak, 4),
                         "flops_per_pair": 2 * d_pad, "batches": len(on_matrix), "launches": launches_m,
                         "avg_launch_ms": round(kms_m / max(1, launches_m), 4),
                         "bound_ms": round(sum(floor_m), 3), "measured_ms": round(kms_m, 3),
                         "frac_of_bound": round(sum(floor_m) / kms_m, 4), "hbm_bound_batches": hbm_bound_m},
            "roofline_popcount": {"kernel": "scan_batched_kernel", "bound": "alu", "achieved": round(tops, 2),
                                  "peak": round(valu_peak, 2), "unit": "Tops/s", "frac": round(tops / valu_peak, 4),
                                  "ops_per_pair": ops_per_pair, "batches": nb, "launches": launches_p,
                                  "avg_launch_ms": round(kms_p / max(1, launches_p), 4),
                                  "bound_ms": round(sum(floor_p), 3), "measured_ms": round(kms_p, 3),
                                  "frac_of_bound": round(sum(floor_p) / kms_p, 4)},
            "popcount_1024": pc}


def run_mid_sweep(tq, torch, args, log):
    """Mid workload (N=1e6, d=768, anisotropic 1 024-component mixture): the x
    sweep {96, 192, 384} -- recall@10 and 10@100 against the FP64 exact-cosine
    top-10 of 200 queries, and the plain path's queries/s at k=100 over the
    1 000 queries.  The 192 MB database fits the 256 MB Infinity Cache, so the
    scan rate is an effective GB/s, not an HBM figure."""
    from workloads import datagen, metrics
    wl = datagen.WORKLOADS["mid"]
    dev = torch.device("cuda", 0)
    n, d, k, xs = wl["n"], wl["d"], wl["k"], wl["xs"]
    W = tq.tq_code_words(d)
    queries = datagen.rows(wl["spec"], datagen.QUERIES, 0, wl["nq"], dev)
    nrec = wl["recall_nq"]
    gt = metrics.ExactTopK(queries[:nrec], 10)
    codes = {x: torch.empty((n, 2 * W), dtype=torch.int32, device=dev) for x in xs}
    # the encoders compared on the same vectors (Table 2 / Fig. 5: EVP at its
    # default x, 1-bit = x = d, b1.58 absmean)
    x_def = tq.tq_default_x(d)
    enc_codes = {name: torch.empty((n, 2 * W), dtype=torch.int32, device=dev)
                 for name in ("evp_default", "one_bit", "b158")}
    for r0, X in datagen.iter_rows(wl["spec"], datagen.DB, 0, n, dev):
        m = X.shape[0]
        for x in xs:
            tq.tq_encode(X, x, codes[x][r0:r0 + m])
        tq.tq_encode(X, x_def, enc_codes["evp_default"][r0:r0 + m])
        tq.tq_encode(X, d, enc_codes["one_bit"][r0:r0 + m])
        tq.tq_encode_b158(X, enc_codes["b158"][r0:r0 + m])
        gt.add(X, r0)
    tq.tq_sync()
    gt_ids, _ = gt.result()
    out = {"workload": f"mid: N={n} d={d}, {wl['nq']} queries, k={k}, plain path; recall on {nrec} queries",
           "rows": []}
    for x in xs:
        db = tq.tq_db_create(codes[x], d, x)
        codes[x] = None
        q = tq.tq_encode(queries, x)
        i10, _ = tq.tq_search_knn(db, q[:nrec], 10, path=tq.TQ_PATH_PLAIN)
        i100, _ = tq.tq_search_knn(db, q[:nrec], 100, path=tq.TQ_PATH_PLAIN)
        ids = torch.empty((q.shape[0], k), dtype=torch.int32, device=dev)
        sc = torch.empty_like(ids)
        tq.tq_search_knn(db, q[:16], k, path=tq.TQ_PATH_PLAIN, ids=ids[:16], scores=sc[:16])
        torch.cuda.synchronize()
        tq.tq_timing_read(0, reset=True)
        tq.tq_timing_enable(True)
        t0 = time.perf_counter()
        tq.tq_search_knn(db, q, k, path=tq.TQ_PATH_PLAIN, ids=ids, scores=sc)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        tq.tq_timing_enable(False)
        kms, launches = tq.tq_timing_read(0, reset=True)
        per_q = kms / q.shape[0]  # scan-kernel time per query (with its sample scan, where taken)
        row = {"x": x, "recall_at_10": round(metrics.recall_at(gt_ids, i10.cpu().numpy(), 10, 10), 4),
               "recall_10_at_100": round(metrics.recall_at(gt_ids, i100.cpu().numpy(), 10, 100), 4),
               "qps": round(q.shape[0] / dt, 1), "scan_ms_per_query": round(per_q, 4),
               "scan_launches_per_query": round(launches / q.shape[0], 2),
               "effective_gbps": round(n * 8 * W / (per_q * 1e-3) / 1e9, 1)}
        out["rows"].append(row)
        log(f"mid x={x}: recall@10 {row['recall_at_10']}, 10@100 {row['recall_10_at_100']}, "
            f"{row['qps']} q/s at k={k} ({row['scan_ms_per_query']} ms of scan kernels per query)")
        db.destroy()
    # encoders on the same vectors: recall of the proxy top-10 / top-100
    qr = queries[:nrec]
    enc = []
    for name, label, x_db, q_codes, metric in (
            ("evp_default", f"EVP {{{x_def},{d}}} (default x), Delta", x_def, tq.tq_encode(qr, x_def),
             tq.TQ_METRIC_DELTA),
            ("one_bit", f"1-bit (x = d = {d}), Delta", d, tq.tq_encode(qr, d), tq.TQ_METRIC_DELTA),
            ("b158", "b1.58 absmean, l2 between ternary vectors (2 Delta - nnz(v))", 0, tq.tq_encode_b158(qr),
             tq.TQ_METRIC_L2),
            ("b158", "b1.58 absmean, raw Delta (no norm correction)", 0, None, tq.TQ_METRIC_DELTA)):
        if q_codes is None:
            q_codes = tq.tq_encode_b158(qr)
        db = tq.tq_db_create(enc_codes[name], d, x_db)
        i10, _ = tq.tq_search_knn(db, q_codes, 10, path=tq.TQ_PATH_PLAIN, metric=metric)
        i100, _ = tq.tq_search_knn(db, q_codes, 100, path=tq.TQ_PATH_PLAIN, metric=metric)
        torch.cuda.synchronize()
        row = {"encoder": label, "recall_at_10": round(metrics.recall_at(gt_ids, i10.cpu().numpy(), 10, 10), 4),
               "recall_10_at_100": round(metrics.recall_at(gt_ids, i100.cpu().numpy(), 10, 100), 4)}
        enc.append(row)
        log(f"mid encoders: {label}: recall@10 {row['recall_at_10']}, 10@100 {row['recall_10_at_100']}")
        db.destroy()
    out["encoders"] = enc
    del enc_codes
    torch.cuda.empty_cache()
    return out


def run_serving(tq, torch, args, log):
    """Serving workload: N=5M d=768 x=192 database; Poisson arrivals at 0.3 / 0.6 / 0.9
    of the plain path's request capacity; sizes geometric (mean 16) in 1..256; k in {10,100}."""
    import threading
    from workloads import datagen, metrics
    wl = datagen.WORKLOADS["serving"]
    dev = torch.device("cuda", 0)
    n, d, x = wl["n"], wl["d"], wl["x"]
    W = tq.tq_code_words(d)
    t0 = time.time()
    queries = datagen.rows(wl["spec"], datagen.QUERIES, 0, 4096, dev)
    gt = metrics.ExactTopK(queries[:200], 10)
    codes = torch.empty((n, 2 * W), dtype=torch.int32, device=dev)
    for r0, X in datagen.iter_rows(wl["spec"], datagen.DB, 0, n, dev):
        tq.tq_encode(X, x, codes[r0:r0 + X.shape[0]])
        gt.add(X, r0)
    tq.tq_sync()
    db = tq.tq_db_create(codes, d, x)
    del codes
    qcodes = tq.tq_encode(queries, x)
    tq.tq_sync()
    qhost = qcodes.cpu().numpy().view(np.uint32)
    ids10, _ = tq.tq_search_knn(db, qcodes[:200], 10, path=tq.TQ_PATH_PLAIN)
    recall = metrics.recall_at(gt.result()[0], ids10.cpu().numpy(), 10, 10)
    log(f"serving database ready in {time.time() - t0:.1f}s")
    # plain capacity on this database
    for _ in range(2):
        tq.tq_search_knn(db, qcodes[:64], 100, path=tq.TQ_PATH_PLAIN)
    torch.cuda.synchronize()
    t = time.perf_counter()
    tq.tq_search_knn(db, qcodes[:512], 100, path=tq.TQ_PATH_PLAIN)
    torch.cuda.synchronize()
    plain_qps = 512 / (time.perf_counter() - t)
    cap_req = plain_qps / wl["mean_size"]
    out = {"workload": f"serving: N={n} d={d} x={x}, Poisson arrivals, request sizes geometric mean 16 in 1..256, "
                       f"k in {{10,100}}, {args.serve_requests} requests per rate",
           "plain_qps": round(plain_qps, 1), "plain_capacity_req_s": round(cap_req, 1),
           "recall_at_10": round(recall, 4), "rates": []}
    srv = tq.tq_server(db, max_k=100, max_slots=8192, max_request_nq=256, budget_bytes=1 << 30,
                       n_segments=args.serve_segments)

    def served_run(server, reqs, offs):
        """The requests submitted at their arrival times by a thread; latency
        from the library's own time stamps."""
        tickets = [None] * len(reqs)
        start = time.perf_counter() + 0.05

        def submitter():
            for i, (ta, nq, k) in enumerate(reqs):
                delay = start + ta - time.perf_counter()
                if delay > 0:
                    time.sleep(delay)
                tickets[i] = server.submit(qhost[offs[i]:offs[i] + nq], k)

        th = threading.Thread(target=submitter)
        th.start()
        lat, nqs, first, last = [], 0, None, 0
        for i in range(len(reqs)):
            while tickets[i] is None:
                time.sleep(0.0002)
            r = server.wait(tickets[i], 600000)
            lat.append((r[2].complete_ns - r[2].submit_ns) / 1e6)
            nqs += reqs[i][1]
            first = r[2].submit_ns if first is None else min(first, r[2].submit_ns)
            last = max(last, r[2].complete_ns)
        th.join()
        span = (last - first) / 1e9  # library time stamps (CLOCK_MONOTONIC)
        return {"p50_ms": round(pct(lat, 50), 3), "p99_ms": round(pct(lat, 99), 3),
                "qps": round(nqs / max(span, 1e-9), 1)}

    for frac in wl["rates"]:
        rate = frac * cap_req
        reqs = datagen.request_stream(args.serve_requests, rate, wl["mean_size"], wl["max_size"], wl["ks"])
        offs = [(i * 37) % (4096 - 256) for i in range(len(reqs))]
        served = served_run(srv, reqs, offs)
        nqs = sum(nq for _, nq, _ in reqs)
        # plain: the same arrivals served first-come first-served, one request at a time
        plat = []
        pstart = time.perf_counter()
        for i, (ta, nq, k) in enumerate(reqs):
            now = time.perf_counter() - pstart
            if now < ta:
                time.sleep(ta - now)
            q = qcodes[offs[i]:offs[i] + nq]
            tq.tq_search_knn(db, q, k, path=tq.TQ_PATH_PLAIN)
            torch.cuda.synchronize()
            plat.append((time.perf_counter() - pstart - ta) * 1e3)
        pspan = time.perf_counter() - pstart
        plain = {"p50_ms": round(pct(plat, 50), 3), "p99_ms": round(pct(plat, 99), 3),
                 "qps": round(nqs / pspan, 1)}
        row = {"load": frac, "req_per_s": round(rate, 1), "served": served, "plain": plain}
        if frac == wl["rates"][1]:
            # the same arrivals on a server pinned to the popcount engine
            psrv = tq.tq_server(db, max_k=100, max_slots=8192, max_request_nq=256, budget_bytes=1 << 30,
                                n_segments=args.serve_segments, engine=tq.TQ_ENGINE_POPCOUNT)
            row["served_popcount_engine"] = served_run(psrv, reqs, offs)
            psrv.destroy()
        out["rates"].append(row)
        log(f"serving load {frac}: served p50 {served['p50_ms']} ms p99 {served['p99_ms']} ms; "
            f"plain p50 {plain['p50_ms']} ms p99 {plain['p99_ms']} ms"
            + (f"; popcount engine p50 {row['served_popcount_engine']['p50_ms']} ms p99 "
               f"{row['served_popcount_engine']['p99_ms']} ms" if "served_popcount_engine" in row else ""))
    st = srv.stats()
    srv.destroy()
    out["ticks"] = st["ticks"]
    out["segments"] = args.serve_segments or "default"
    db.destroy()
    return out


def source_sha(*names):
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_2506_00528_amd", "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import torch

    from paper_2506_00528_amd import tq
    from workloads import datagen, metrics

    if not os.path.exists(tq.LIB_PATH):
        from paper_2506_00528_amd.build import build
        build()
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    wl = datagen.WORKLOADS[args.workload]
    n, d, k = wl["n"], wl["d"], args.k or wl["k"]
    x = args.x or wl["x"]
    nq_total = wl["nq"]
    spec = wl["spec"]
    W = tq.tq_code_words(d)
    log = lambda m: print(f"[bench] {m}", file=sys.stderr, flush=True)

    # ---- database: generate on the GPU chunk by chunk, encode, ground truth
    t0 = time.time()
    queries = datagen.rows(spec, datagen.QUERIES, 0, nq_total, dev)
    nrec = min(args.recall_queries, nq_total)
    gt = metrics.ExactTopK(queries[:nrec], 10)
    codes = torch.empty((n, 2 * W), dtype=torch.int32, device=dev)
    # the same vectors at a small x, for the index-list engine (kept when 8x <= d)
    xs = d // 32 if args.sparse_x < 0 else args.sparse_x
    sp_codes = torch.empty((n, 2 * W), dtype=torch.int32, device=dev) if 0 < xs and 8 * xs <= d else None
    cpu_rows = min(args.cpu_sample_rows, n) if not args.no_cpu_baseline else 0
    cpu_X = np.empty((cpu_rows, d), dtype=np.float32) if cpu_rows else None
    for r0, X in datagen.iter_rows(spec, datagen.DB, 0, n, dev):
        tq.tq_encode(X, x, codes[r0:r0 + X.shape[0]])
        if sp_codes is not None:
            tq.tq_encode(X, xs, sp_codes[r0:r0 + X.shape[0]])
        gt.add(X, r0)
        if cpu_rows and r0 < cpu_rows:
            m = min(X.shape[0], cpu_rows - r0)
            cpu_X[r0:r0 + m] = X[:m].cpu().numpy()
    tq.tq_sync()
    log(f"database generated+encoded: n={n} d={d} x={x} in {time.time() - t0:.1f}s")

    # encode rate of the kernel alone on one resident block
    blk = datagen.rows(spec, datagen.DB, 0, min(n, 1 << 18), dev)
    enc_out = torch.empty((blk.shape[0], 2 * W), dtype=torch.int32, device=dev)
    tq.tq_encode(blk, x, enc_out)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        tq.tq_encode(blk, x, enc_out)
    e1.record()
    torch.cuda.synchronize()
    enc_ms = e0.elapsed_time(e1) / 5
    enc_bytes = blk.numel() * 4 + enc_out.numel() * 4
    del blk, enc_out

    db = tq.tq_db_create(codes, d, x)
    del codes
    torch.cuda.empty_cache()
    qcodes_all = tq.tq_encode(queries, x)
    tq.tq_sync()

    path = {"plain": tq.TQ_PATH_PLAIN, "batched": tq.TQ_PATH_BATCHED, "auto": tq.TQ_PATH_AUTO}[args.path]

    # ---- recall on the ground-truth subsample (k=10 and 10@100)
    ids10, _ = tq.tq_search_knn(db, qcodes_all[:nrec], 10, path=path, grid=args.grid)
    ids100, _ = tq.tq_search_knn(db, qcodes_all[:nrec], 100, path=path, grid=args.grid)
    gt_ids, _ = gt.result()
    recall10 = metrics.recall_at(gt_ids, ids10.cpu().numpy(), 10, 10)
    recall10_100 = metrics.recall_at(gt_ids, ids100.cpu().numpy(), 10, 100)
    # ---- masked addition (float queries against the codes): recall and HBM rate
    tq.tq_search_masked(db, queries[:2], 10)
    torch.cuda.synchronize()
    tq.tq_timing_read(2, reset=True)
    tq.tq_timing_enable(True)
    t_m = time.perf_counter()
    m_ids, _ = tq.tq_search_masked(db, queries[:nrec], 10)
    torch.cuda.synchronize()
    t_m = time.perf_counter() - t_m
    tq.tq_timing_enable(False)
    m_ms, m_launches = tq.tq_timing_read(2, reset=True)
    m_avg = m_ms / max(1, m_launches)
    masked = {"recall_at_10": round(metrics.recall_at(gt_ids, m_ids.cpu().numpy(), 10, 10), 4),
              "queries": nrec, "qps": round(nrec / t_m, 1),
              "roofline": {"kernel": "scan_masked_kernel", "bound": "hbm",
                           "achieved": round(n * 8 * W / (m_avg * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBPS,
                           "unit": "GB/s", "frac": round(n * 8 * W / (m_avg * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
                           "avg_launch_ms": round(m_avg, 4), "launches": m_launches}}
    log(f"masked addition: recall@10 {masked['recall_at_10']}, {m_avg:.3f} ms per query scan "
        f"({masked['roofline']['frac'] * 100:.1f}% of HBM)")

    # ---- index-list engine on the small-x database: recall, QPS and HBM rate
    sparse = None
    if sp_codes is not None:
        sdb = tq.tq_db_create(sp_codes, d, xs)
        del sp_codes
        torch.cuda.empty_cache()
        sq = tq.tq_encode(queries[:nrec], xs)
        s_ids, _ = tq.tq_search_knn(sdb, sq, 10, path=tq.TQ_PATH_PLAIN, engine=tq.TQ_ENGINE_SPARSE)
        b_ids, b_sc = tq.tq_search_knn(sdb, sq, 10, path=tq.TQ_PATH_PLAIN, engine=tq.TQ_ENGINE_POPCOUNT)
        s_ids2, s_sc2 = tq.tq_search_knn(sdb, sq, 10, path=tq.TQ_PATH_PLAIN, engine=tq.TQ_ENGINE_SPARSE)
        torch.cuda.synchronize()
        same = bool(torch.equal(s_ids2, b_ids) and torch.equal(s_sc2, b_sc))
        timing = {}
        for name, eng, fam in (("index_list", tq.TQ_ENGINE_SPARSE, 3), ("bit_planes", tq.TQ_ENGINE_POPCOUNT, 0)):
            tq.tq_timing_read(fam, reset=True)
            tq.tq_timing_enable(True)
            t_s = time.perf_counter()
            tq.tq_search_knn(sdb, sq, 10, path=tq.TQ_PATH_PLAIN, engine=eng)
            torch.cuda.synchronize()
            t_s = time.perf_counter() - t_s
            tq.tq_timing_enable(False)
            ms_s, l_s = tq.tq_timing_read(fam, reset=True)
            timing[name] = (nrec / t_s, ms_s / max(1, l_s), l_s)
        sc_chunks = (xs + 7) // 8
        s_bytes = n * 16 * sc_chunks  # 8 two-byte entries per 16-byte chunk, every vector once
        s_avg = timing["index_list"][1]
        s_gbps = s_bytes / (s_avg * 1e-3) / 1e9
        sparse = {"workload": f"same N={n} d={d} vectors encoded at x={xs}, index-list engine, k=10",
                  "x": xs, "recall_at_10": round(metrics.recall_at(gt_ids, s_ids.cpu().numpy(), 10, 10), 4),
                  "queries": nrec, "qps": round(timing["index_list"][0], 1),
                  "bit_planes_qps": round(timing["bit_planes"][0], 1),
                  "bit_planes_avg_launch_ms": round(timing["bit_planes"][1], 4),
                  "same_results_as_bit_planes": same,
                  "roofline": {"kernel": "scan_sparse_kernel", "bound": "hbm", "achieved": round(s_gbps, 1),
                               "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": round(s_gbps / HBM_PEAK_GBPS, 4),
                               "bytes_per_launch": s_bytes, "avg_launch_ms": round(s_avg, 4),
                               "launches": timing["index_list"][2]}}
        log(f"index list x={xs}: recall@10 {sparse['recall_at_10']}, {s_avg:.4f} ms per scan "
            f"({sparse['roofline']['frac'] * 100:.1f}% of HBM), {sparse['qps']} q/s vs "
            f"{sparse['bit_planes_qps']} q/s on the bit planes, same results: {same}")
        sdb.destroy()
        del sq, s_ids, b_ids, b_sc, s_ids2, s_sc2
        torch.cuda.empty_cache()

    # ---- timed steps
    B = args.batch
    out_ids = torch.empty((B, k), dtype=torch.int32, device=dev)
    out_sc = torch.empty((B, k), dtype=torch.int32, device=dev)
    qc = torch.empty((B, 2 * W), dtype=torch.int32, device=dev)

    def step(i):
        q0 = (i * B) % max(1, nq_total - B + 1)
        tq.tq_encode(queries[q0:q0 + B], x, qc)
        tq.tq_search_knn(db, qc, k, path=path, grid=args.grid, ids=out_ids, scores=out_sc, engine=engine)

    engine = {"matrix": tq.TQ_ENGINE_MATRIX, "popcount": tq.TQ_ENGINE_POPCOUNT}[args.engine] \
        if args.path == "batched" else tq.TQ_ENGINE_AUTO
    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    sclk_before = tq.tq_clock_mhz()
    tq.tq_timing_read(0, reset=True)
    tq.tq_timing_read(1, reset=True)
    tq.tq_timing_enable(True)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        step(args.warmup + i)
    torch.cuda.synchronize()
    t_end = time.perf_counter()
    tq.tq_timing_enable(False)
    fam = 1 if args.path == "batched" else 0
    kern_ms, launches = tq.tq_timing_read(fam, reset=True)
    tq.tq_sync()

    elapsed = t_end - t_start
    nqueries = args.steps * B
    # ---- refinement of the top-N Delta candidates (after the timed region)
    rerank = None
    if args.rerank:
        # the float database (40.96 GB), regenerated here rather than kept from
        # the set-up: with it resident the timed scans ran a few percent slower
        Xall = torch.empty((n, d), dtype=torch.float32, device=dev)
        for r0, X in datagen.iter_rows(spec, datagen.DB, 0, n, dev):
            Xall[r0:r0 + X.shape[0]].copy_(X)
        R = min(args.rerank, tq.TQ_MAX_K, n)
        # the candidates: the library's own path choice for nrec queries at k = R
        cand, cand_sc = tq.tq_search_knn(db, qcodes_all[:nrec], R, path=tq.TQ_PATH_AUTO)
        rr_ids, rr_sc = tq.tq_rerank(Xall, queries[:nrec], cand, 10)
        torch.cuda.synchronize()
        c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        c0.record()
        tq.tq_search_knn(db, qcodes_all[:nrec], R, path=tq.TQ_PATH_AUTO, ids=cand, scores=cand_sc)
        c1.record()
        torch.cuda.synchronize()
        cand_ms = c0.elapsed_time(c1)
        recall_rr = metrics.recall_at(gt_ids, rr_ids.cpu().numpy(), 10, 10)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            tq.tq_rerank(Xall, queries[:nrec], cand, 10, ids=rr_ids, scores=rr_sc)
        e1.record()
        torch.cuda.synchronize()
        rr_ms = e0.elapsed_time(e1) / 5
        rr_bytes = nrec * R * d * 4  # every candidate row read once
        rerank = {"candidates": R, "k": 10, "recall_at_10": round(recall_rr, 4), "queries": nrec,
                  "ms": round(rr_ms, 4), "gbps": round(rr_bytes / (rr_ms * 1e-3) / 1e9, 1),
                  "candidate_scan_ms": round(cand_ms, 3), "candidate_scan_path": "auto"}
        log(f"rerank top-{R} -> 10: recall@10 {recall_rr:.4f} (proxy alone {recall10:.4f}), "
            f"{rr_ms:.3f} ms for {nrec} queries; the top-{R} candidate scan {cand_ms:.1f} ms")
        del Xall
        torch.cuda.empty_cache()

    qps = nqueries / elapsed
    ms_per_step = elapsed * 1e3 / args.steps
    db_bytes = n * 2 * W * 4  # algorithmic bytes of one full scan: both bit planes of every vector
    avg_launch_ms = kern_ms / launches if launches else float("nan")
    achieved = db_bytes / (avg_launch_ms * 1e-3) / 1e9 if launches else float("nan")

    # batched path: dominant kernel is bound by integer VALU issue, not HBM
    valu_peak_tops = 256 * 64 * 2.4e9 / 1e12  # 32-bit lane-ops/s: 256 CUs x 64 lanes x 2.4 GHz
    ops_per_pair = 5 * 4 * ((W + 3) // 4)  # and, xor, and + two popcount-accumulates per plane word
    traffic = None
    tf = os.path.join(ROOT, "profiles", "traffic.json")
    key = f"scan_plain/{args.workload}"
    if os.path.exists(tf):
        rec = json.load(open(tf)).get(key)
        if rec and rec.get("source_sha") == source_sha("scan.hip", "tq_device.h"):
            traffic = rec.get("hbm_bytes_per_launch")

    result = {
        "metric": METRIC,
        "value": round(qps, 2),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: N={n} d={d} x={x} k={k}, {B} queries/step, "
                               f"{args.path} path (one full database scan per query)",
                   "n": n, "d": d, "x": x, "k": k, "queries_per_step": B, "path": args.path,
                   "global_batch": B, "parallelism": "single GPU"},
        "hbm_gbps": round(achieved, 1),
        "hbm_frac": round(achieved / HBM_PEAK_GBPS, 4),
        "recall_at_10": round(recall10, 4),
        "recall_10_at_100": round(recall10_100, 4),
        "recall_queries": nrec,
        "rerank": rerank,
        "masked": masked,
        "sparse": sparse,
        "encode": {"kernel": "encode_kernel", "bound": "hbm", "rows_per_s": round(enc_bytes / (4 * (d + 2 * W)) / (enc_ms * 1e-3), 1),
                   "gbps": round(enc_bytes / (enc_ms * 1e-3) / 1e9, 1),
                   "frac": round(enc_bytes / (enc_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4)},
        "roofline": {"kernel": "scan_plain_kernel", "bound": "hbm", "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                     "traffic": traffic, "bytes_per_launch": db_bytes,
                     "avg_launch_ms": round(avg_launch_ms, 5), "launches": launches},
    }
    if args.path == "batched" and args.engine == "popcount":
        ops = B * n * ops_per_pair
        tops = ops / (avg_launch_ms * 1e-3) / 1e12
        result["hbm_gbps"] = None
        result["hbm_frac"] = None
        result["roofline"] = {"kernel": "scan_batched_kernel", "bound": "alu", "achieved": round(tops, 2),
                              "peak": round(valu_peak_tops, 2), "unit": "Tops/s", "frac": round(tops / valu_peak_tops, 4),
                              "traffic": None, "ops_per_launch": ops, "ops_per_pair": ops_per_pair,
                              "avg_launch_ms": round(avg_launch_ms, 5), "launches": launches}
    elif args.path == "batched":
        d_pad = 128 * ((W * 32 + 127) // 128)
        tflops = 2.0 * B * n * d_pad / (avg_launch_ms * 1e-3) / 1e12
        result["hbm_gbps"] = None
        result["hbm_frac"] = None
        result["roofline"] = {"kernel": "scan_mfma_group_kernel (k <= 16); sample pass + sample_floor_kernel + scan_mfma_kernel (k > 16)", "bound": "mfma", "achieved": round(tflops, 1),
                              "peak": 10100.0, "unit": "TFLOP/s", "frac": round(tflops / 10100.0, 4),
                              "traffic": None, "flops_per_pair": 2 * d_pad,
                              "avg_launch_ms": round(avg_launch_ms, 5), "launches": launches}

    if args.copy_probe:
        a = torch.empty(1 << 28, dtype=torch.int32, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        result["copy_probe_bytes"] = a.numel() * 4

    if not args.no_batching and args.workload == "large":
        result["batched"] = run_batching(tq, torch, db, queries, x, n, W, qps, args, log)
    # the shader clock under load (device counters), before the timed steps
    # and now; the vector-ALU and matrix-core peaks above assume 2 400 MHz
    result["sclk_mhz"] = {"before_steps": round(sclk_before, 1), "after_batching": round(tq.tq_clock_mhz(), 1),
                          "peak_assumed": 2400.0}

    # ---- CPU oracle on a bounded sample (rank 0, N=1 only)
    if cpu_rows:
        import oracle
        o = oracle.default()
        threads = o.num_threads()
        Vs = o.encode(cpu_X, x)  # set-up: the sample database, encoded once
        nqs = args.cpu_sample_queries
        Qs = queries[:nqs].cpu().numpy()
        t = time.perf_counter()
        VQ = o.encode(Qs, x)
        o.knn(VQ, Vs, k)
        dt = time.perf_counter() - t
        per_query_full = dt / nqs * (n / cpu_rows)
        result["cpu_baseline"] = {
            "value": round(1.0 / per_query_full, 4), "unit": "queries/s", "cores": threads, "kind": "oracle",
            "sample": f"{nqs} queries encoded + exhaustive top-{k} over the first {cpu_rows} database rows "
                      f"({dt:.1f}s), scaled by N/{cpu_rows} to the full N={n}"}
    db.destroy()
    torch.cuda.empty_cache()
    if not args.no_serving and args.workload == "large":
        result["serving"] = run_serving(tq, torch, args, log)
    if not args.no_mid and args.workload == "large":
        result["mid_sweep"] = run_mid_sweep(tq, torch, args, log)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
