"""Benchmark: exact induced 4- and 5-vertex subgraph counts on one MI355X.

One step = one call of esc_count_subgraphs(k=5) on the whole graph: degree
order and relabelled CSR, triangles and per-arc triangle lists, 4-cycles,
the per-triangle pass (4- and 5-cliques, triangle-cut sums), vertex and edge
sums, the pattern 13/17 and wheel pair passes, 5-cycles and the final exact
linear map; the 45 counts end on the host.  The CSR is resident in HBM when
the timed region starts.

Headline workload: the largest single-GPU graph, Chung-Lu n = 4e6, exponent
1.9, mean degree 40, max expected degree 5e4 (seed 0, 7.65e7 edges, a
near-clique core of some 1.4e3 hubs), standing in for the paper's
web/social/technology graphs; value = undirected edges / second.  One call
takes minutes, so this leg times min(--steps, --headline-steps) calls with
--headline-warmup warm-up calls before them (the line reports both the
requested and the timed numbers); the library prints each stage as it ends
(ESC_TRACE).  The 1M-vertex graph (exponent 2.1, mean degree 20, max expected
degree 1e4) runs the full --steps / --warmup under the key "chung_lu_1m",
beside the batched and serving workloads.

Prints one JSON line (see the keys below).  --gpus above 1 is refused: this
build runs on one GPU.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP4_PEAK_TOPS = 10100.0  # dense 4-bit-float matrix-core peak (10.1 POP/s; one multiply-add = 2 ops)
BYTES_PER_VISIT = 4     # one int32 neighbour / triangle-list entry per visited element
TRAFFIC_FILES = {"chung_lu_4m": os.path.join(ROOT, "profiles", "traffic_chung_lu_4m.json"),
                 "chung_lu_1m": os.path.join(ROOT, "profiles", "traffic_chung_lu_1m.json")}


def kernel_sources_sha(source_file):
    """sha256 over (name, bytes) of ctx.h, device.h and the kernel's file."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1610_09411_amd", "csrc")
    for name in ("ctx.h", "device.h", source_file):
        h.update(name.encode())
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(workload, stage):
    """HBM bytes per launch of a stage's kernel from the committed rocprofv3
    FETCH_SIZE/WRITE_SIZE summary of the workload, or None when that kernel's
    sources have changed since it was taken (or no summary covers it)."""
    try:
        with open(TRAFFIC_FILES[workload]) as f:
            t = json.load(f)
        e = t["stages"][stage]
        if e["sources_sha256"] != kernel_sources_sha(e["source_file"]):
            return None
    except (OSError, ValueError, KeyError):
        return None
    e = t["stages"][stage]
    return e["fetch_bytes"] + e["write_bytes"]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--headline-steps", type=int, default=1,
                    help="timed calls on the 4M-vertex graph at most (each takes minutes)")
    ap.add_argument("--headline-warmup", type=int, default=0,
                    help="warm-up calls on the 4M-vertex graph (0: buffer allocation is inside the timed call)")
    ap.add_argument("--headline", choices=["chung_lu_4m", "chung_lu_1m"], default="chung_lu_4m")
    ap.add_argument("--small", type=int, default=1,
                    help="also time the 1M-vertex graph when the headline is the 4M one (0 = skip)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu-sample", type=int, default=128,
                    help="oracle timing sample: 1/N of sources and edges (0 = skip the CPU leg)")
    ap.add_argument("--cpu-threads", type=int, default=0)
    ap.add_argument("--cpu-one-thread", type=int, default=0,
                    help="also time the oracle on one thread (about 150 s more: its setup stage alone takes 2 min)")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="only run a plain device-to-device copy of this many bytes (counter calibration)")
    ap.add_argument("--batched", type=int, default=1,
                    help="also measure the 10^4-graph batched workload against one graph per launch (0 = skip)")
    ap.add_argument("--plain-sample", type=int, default=500,
                    help="graphs of the batched workload timed one graph per launch")
    ap.add_argument("--serving-rate", type=float, default=200.0,
                    help="Poisson arrival rate (requests/s) of the serving latency measurement (0 = skip serving)")
    ap.add_argument("--serving-seconds", type=float, default=4.0)
    ap.add_argument("--serving-inflight", type=int, default=8)
    ap.add_argument("--workload", choices=["single", "serving-sweep"], default="single",
                    help="serving-sweep: only the serving loop, one JSON line per rate in --rates")
    ap.add_argument("--rates", default="100,200,500,1000,2000,5000")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(--gpus %d refused)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    rank = int(os.environ.get("RANK", "0"))

    import torch
    if args.copy_probe > 0:
        # a copy kernel of known size: rocprofv3 FETCH_SIZE / WRITE_SIZE on it
        # give the factor between counter units and bytes moved
        src = torch.ones(args.copy_probe, dtype=torch.uint8, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": args.copy_probe}), flush=True)
        return
    import synth
    import paper_1610_09411_amd as esc

    if args.workload == "serving-sweep":
        ctx = esc.Context(0)
        pool = serving_pool(synth, args.seed)
        cap = bench_serving_capacity(esc, ctx, pool, args.serving_inflight)
        print(json.dumps(dict(cap, metric="serving capacity (burst)", n_gpus=1)), flush=True)
        for rate in [float(x) for x in args.rates.split(",")]:
            res = bench_serving(esc, ctx, pool, rate, args.serving_seconds, args.serving_inflight, args.seed)
            print(json.dumps(dict(res, metric="serving latency and throughput", n_gpus=1)), flush=True)
        ctx.close()
        return

    # the headline context reports every stage as it ends (a call on the 4M
    # graph takes minutes), one launch per stage so the per-launch roofline
    # figures hold
    os.environ["ESC_TRACE"] = "1"
    os.environ["ESC_SLICE_MS"] = "0"
    ctx_h = esc.Context(0)
    del os.environ["ESC_TRACE"]
    del os.environ["ESC_SLICE_MS"]
    ctx = esc.Context(0)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)

    big = args.headline == "chung_lu_4m"
    g = synth.chung_lu_4m(args.seed) if big else synth.chung_lu_1m(args.seed)
    print("headline graph n=%d m=%d generated" % (g.n, g.m), file=sys.stderr, flush=True)
    h_steps = min(args.steps, args.headline_steps) if big else args.steps
    h_warm = min(args.warmup, args.headline_warmup) if big else args.warmup
    head = run_single(esc, ctx_h if big else ctx, torch, g, args.headline, h_steps, h_warm, stream)
    head_g = g
    ctx_h.close()
    del g

    small = None
    if big and (args.small or args.cpu_sample > 0):
        g1 = synth.chung_lu_1m(args.seed)
        if args.small:
            # at least one warm-up call: the first call on a context sizes
            # its buffers (seconds for the per-workgroup tables)
            small = run_single(esc, ctx, torch, g1, "chung_lu_1m", args.steps, max(args.warmup, 1), stream)
    else:
        g1 = head_g

    cpu = None
    if rank == 0 and args.cpu_sample > 0:
        cpu = cpu_baseline(g1, args.cpu_sample, args.cpu_threads, args.cpu_one_thread)

    batched = None
    if args.batched:
        batched = bench_batched(esc, ctx, synth, torch, stream, args.steps, args.seed, args.plain_sample)
    serving = None
    if args.serving_rate > 0:
        pool = serving_pool(synth, args.seed)
        serving = bench_serving(esc, ctx, pool, args.serving_rate, args.serving_seconds, args.serving_inflight,
                                args.seed)
        serving["capacity"] = bench_serving_capacity(esc, ctx, pool, args.serving_inflight)

    line = {
        "metric": "edges/sec for all induced 4+5-vertex counts (bit-exact)",
        "value": head["value"],
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": h_steps,
        "warmup": h_warm,
        "steps_requested": args.steps,
        "warmup_requested": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": head["config"],
        "roofline": head["roofline"],
        "cpu_baseline": cpu,
        "stages_ms": head["stages_ms"],
        "walks_ms": head["walks_ms"],
        "stages_visits": head["stages_visits"],
        "products": head["products"],
        "work": head["work"],
        "launch_params": head["launch_params"],
        "checksum": head["checksum"],
        "chung_lu_1m": small,
        "batched": batched,
        "serving": serving,
    }
    if rank == 0:
        print(json.dumps(line), flush=True)
    ctx.close()


WORKLOADS = {
    "chung_lu_4m": "chung_lu n=4000000 gamma=1.9 mean_degree=40 max_expected_degree=50000 seed=%d",
    "chung_lu_1m": "chung_lu n=1000000 gamma=2.1 mean_degree=20 max_expected_degree=10000 seed=%d",
}


def run_single(esc, ctx, torch, g, name, steps, warmup, stream, seed=0):
    """`warmup` untimed then `steps` timed k = 5 calls on graph g (CSR resident
    on the device); per-stage device times and visits averaged over the timed
    calls, each stage split into its walk and its matrix-core product
    (esc_last_products; HIP events on the call's stream); the roofline of
    the longest of those kernels: a walk against the HBM peak (4 bytes per
    visited element), a product against the matrix-core peak of its operand
    type (4-bit floats)."""
    n, m = g.n, g.m
    dev = torch.device("cuda:0")
    rp = torch.from_numpy(g.row_ptr).to(dev)
    col = torch.from_numpy(g.col).to(dev)
    counts = None
    for _ in range(warmup):
        counts = esc.esc_count_subgraphs(ctx.ptr, n, rp, col, 5, stream=stream)
    prof_sum = {k: [0.0, 0] for k in esc.STAGES}
    prod_sum = {k: [0.0, 0.0, 0] for k in esc.STAGES}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        counts = esc.esc_count_subgraphs(ctx.ptr, n, rp, col, 5, stream=stream)
        for k, (ms, vis) in esc.esc_last_profile(ctx.ptr).items():
            prof_sum[k][0] += ms
            prof_sum[k][1] += vis
        for k, (wms, pms, macs) in esc.esc_last_products(ctx.ptr).items():
            prod_sum[k][0] += wms
            prod_sum[k][1] += pms
            prod_sum[k][2] += macs
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1000.0 / steps
    prof = {k: (v[0] / steps, v[1] / steps) for k, v in prof_sum.items()}
    prods = {k: (v[0] / steps, v[1] / steps, v[2] / steps) for k, v in prod_sum.items()}
    # the dominant kernel: a stage's walk (the whole stage where it has no
    # matrix-core product; HBM-bound list reads) or a stage's product (fp4
    # matrix cores), whichever takes longest
    walk_dom = max(prods, key=lambda k: prods[k][0])
    prod_dom = max(prods, key=lambda k: prods[k][1])
    products = {k: {"ms": round(v[1], 3), "multiply_adds": int(v[2]),
                    "achieved_tops": 2 * v[2] / (v[1] / 1000.0) / 1e12 if v[1] > 0 else 0.0,
                    "frac": 2 * v[2] / (v[1] / 1000.0) / 1e12 / FP4_PEAK_TOPS if v[1] > 0 else 0.0}
                for k, v in prods.items() if v[2] > 0}
    if prods[prod_dom][1] > prods[walk_dom][0] and prods[prod_dom][2] > 0:
        pk = products[prod_dom]
        roofline = {"bound": "mfma", "kernel": prod_dom + " product", "achieved": pk["achieved_tops"],
                    "peak": FP4_PEAK_TOPS, "unit": "TOP/s", "frac": pk["frac"], "traffic": None,
                    "traffic_bytes_per_launch": None, "algorithmic_ops": 2 * prods[prod_dom][2]}
    else:
        dom = walk_dom
        dom_ms, dom_vis = prods[dom][0], prof[dom][1]
        achieved = dom_vis * BYTES_PER_VISIT / (dom_ms / 1000.0) / 1e9 if dom_ms > 0 else 0.0
        tbytes = measured_traffic(name, dom)
        traffic = tbytes / (dom_ms / 1000.0) / 1e9 if (tbytes is not None and dom_ms > 0) else None
        roofline = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "traffic_bytes_per_launch": tbytes,
                    "algorithmic_bytes_per_launch": dom_vis * BYTES_PER_VISIT}
    del rp, col
    return {"value": m / (ms_per_step / 1000.0), "ms_per_step": ms_per_step, "steps": steps, "warmup": warmup,
            "config": {"workload": WORKLOADS[name] % seed, "n": n, "m": m, "k": 5, "parallelism": "single GPU"},
            "roofline": roofline,
            "stages_ms": {k: round(v[0], 3) for k, v in prof.items()},
            "walks_ms": {k: round(v[0], 3) for k, v in prods.items()},
            "stages_visits": {k: int(v[1]) for k, v in prof.items()},
            "products": products,
            "work": esc.esc_last_work(ctx.ptr),
            "launch_params": ctx.last_params(),
            "checksum": {"sum_4": str(sum(counts[:11])), "sum_5": str(sum(counts[11:])),
                         "p8_5cycles": str(counts[11 + 7]), "p21_5cliques": str(counts[31])}}


def cpu_baseline(g, sample, threads, one_thread):
    """The oracle on the host cores, timed on a bounded sample of the 1M-vertex
    graph's job (its per-edge triangle lists for the 4M-vertex graph, 12 B x
    2.8e10 entries, do not fit host memory): degree order, triangle stage and
    triangle lists in full, every later per-source / per-edge loop on 1/sample
    of the ids (two sample offsets, their spread reported); with one_thread,
    also on one thread at 4x the sampling."""
    import platform
    import oracle
    threads = threads or len(os.sched_getaffinity(0))
    runs = []
    for off in (0, sample // 2):
        setup_s, sampled_s = oracle.timed_sample(g, 5, sample, threads, off)
        runs.append((setup_s, sampled_s))
    est = [s + x * sample for s, x in runs]
    mean = sum(est) / len(est)
    one = None
    if one_thread:
        s1 = 4 * sample
        setup1, sampled1 = oracle.timed_sample(g, 5, s1, 1, 0)
        est1 = setup1 + sampled1 * s1
        one = {"value": g.m / est1, "setup_s": setup1, "sampled_s": sampled1, "sample": s1, "estimated_s": est1}
    cpu_model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    cpu_model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        cpu_model = platform.processor()
    return {"value": g.m / mean, "unit": "edges/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model,
            "workload": "chung_lu n=1000000 gamma=2.1 mean_degree=20 max_expected_degree=10000 (the oracle "
                        "cannot hold the 4M-vertex graph's triangle lists in host memory)",
            "sample": "degree order, triangle stage and triangle lists in full (%.1f s), every later "
                      "per-source/per-edge loop on 1/%d of the ids at offsets 0 and %d (%.1f s, %.1f s, scaled "
                      "x%d); estimated whole job %.0f s and %.0f s"
                      % (runs[0][0], sample, sample // 2, runs[0][1], runs[1][1], sample, est[0], est[1]),
            "spread": abs(est[0] - est[1]) / mean,
            "one_thread": one}


def bench_batched(esc, ctx, synth, torch, stream, steps, seed, plain_sample):
    """The batched workload: 10^4 graphs, n log-uniform in [20, 2000], half
    Erdos-Renyi (mean degree 4-30), half Chung-Lu (exponent 2.0-2.8), in one
    esc_count_batched call with the concatenated CSR resident in HBM; against
    the same graphs one esc_count_subgraphs call each (a sample of them)."""
    specs = synth.batch_specs(10_000, seed)
    graphs = [synth.from_spec(x) for x in specs]
    vo, ao, rp, ci = esc.pack_batch(graphs)
    rp_d = torch.from_numpy(rp).cuda()
    ci_d = torch.from_numpy(ci).cuda()
    esc.esc_count_batched(ctx.ptr, vo, ao, rp_d, ci_d, 5, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        rows, ovf = esc.esc_count_batched(ctx.ptr, vo, ao, rp_d, ci_d, 5, stream=stream)
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / steps
    prof = {k: round(v[0], 3) for k, v in esc.esc_last_profile(ctx.ptr).items()}
    sums_ok = all(int(rows[i][11:].sum(dtype=object)) == _comb5(graphs[i].n) for i in range(len(graphs)))
    sample = graphs[:plain_sample]
    dev = [(x.n, torch.from_numpy(x.row_ptr).cuda(), torch.from_numpy(x.col).cuda()) for x in sample]
    esc.esc_count_subgraphs(ctx.ptr, dev[0][0], dev[0][1], dev[0][2], 5, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain_rows = [esc.esc_count_subgraphs(ctx.ptr, n, r, c, 5, stream=stream) for n, r, c in dev]
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    same = all([int(v) for v in rows[i]] == plain_rows[i] for i in range(len(sample)))
    m_total = int(ao[-1]) // 2
    return {"workload": "batched: 10000 graphs, n log-uniform [20,2000], half ER mean degree 4-30, "
                        "half Chung-Lu exponent 2.0-2.8, seed %d" % seed,
            "graphs": len(graphs), "sum_n": int(vo[-1]), "sum_m": m_total,
            "graphs_per_s": len(graphs) / t_batch, "edges_per_s": m_total / t_batch, "ms_per_batch": t_batch * 1e3,
            "stages_ms": prof,
            "plain_graphs_per_s": len(sample) / t_plain, "plain_sample": len(sample),
            "speedup_vs_plain": (len(graphs) / t_batch) / (len(sample) / t_plain),
            "rows_sum_to_C(n,5)": sums_ok, "sample_equal_to_plain": same}


def _comb5(n):
    from math import comb
    return comb(n, 5)


def serving_pool(synth, seed, size=400):
    """Request graphs: Chung-Lu, n log-uniform in [50, 50000], exponent
    2.0-2.5, mean degree 8-32; arrivals draw from this pool."""
    return [synth.from_spec(x) for x in synth.request_specs(size, seed)]


def bench_serving_capacity(esc, ctx, pool, inflight, count=2000):
    """Saturated throughput: `count` requests submitted at once."""
    srv = esc.Server(ctx, max_inflight=inflight)
    for t in [srv.submit(g, 5) for g in pool[:16]]:
        srv.wait(t)
    st0 = srv.stats()
    t0 = time.perf_counter()
    tickets = [srv.submit(pool[i % len(pool)], 5) for i in range(count)]
    for t in tickets:
        srv.wait(t)
    t1 = time.perf_counter()
    st = srv.stats()
    srv.stop()
    edges = sum(pool[i % len(pool)].m for i in range(count))
    return {"requests": count, "graphs_per_s": count / (t1 - t0), "edges_per_s": edges / (t1 - t0),
            "launches": st["launches"] - st0["launches"], "peak_inflight": st["peak_inflight"]}


def bench_serving(esc, ctx, pool, rate, seconds, inflight, seed):
    """Poisson arrivals at `rate` for `seconds`; latency = submit to result,
    measured by the server; throughput = completed requests / elapsed."""
    import random
    import threading
    rng = random.Random(seed)
    srv = esc.Server(ctx, max_inflight=inflight)
    for t in [srv.submit(g, 5) for g in pool[:16]]:     # warm the worker contexts
        srv.wait(t)
    st0 = srv.stats()
    tickets = []
    lat = []
    done_evt = threading.Event()

    def collect():
        i = 0
        while True:
            if i < len(tickets):
                lat.append(srv.wait(tickets[i])[1])
                i += 1
            elif done_evt.is_set():
                break
            else:
                time.sleep(0.0005)
    th = threading.Thread(target=collect)
    th.start()
    t0 = time.perf_counter()
    nxt = t0
    edges = 0
    while True:
        nxt += rng.expovariate(rate)
        if nxt - t0 > seconds:
            break
        d = nxt - time.perf_counter()
        if d > 0:
            time.sleep(d)
        g = pool[rng.randrange(len(pool))]
        tickets.append(srv.submit(g, 5))
        edges += g.m
    done_evt.set()
    th.join()
    t1 = time.perf_counter()
    st = srv.stats()
    srv.stop()
    lat.sort()
    q = lambda p: lat[min(len(lat) - 1, int(p * len(lat)))] * 1e3 if lat else None
    return {"workload": "serving: Chung-Lu requests, n log-uniform [50,50000], exponent 2.0-2.5, mean degree 8-32 "
                        "(pool of %d graphs), Poisson arrivals" % len(pool),
            "rate_req_s": rate, "seconds": seconds, "requests": len(tickets),
            "graphs_per_s": len(tickets) / (t1 - t0), "edges_per_s": edges / (t1 - t0),
            "p50_ms": q(0.50), "p99_ms": q(0.99), "max_inflight": inflight,
            "launches": st["launches"] - st0["launches"],
            "batched_requests": st["batched_requests"] - st0["batched_requests"],
            "peak_inflight": st["peak_inflight"]}


if __name__ == "__main__":
    main()
