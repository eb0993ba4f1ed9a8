"""Benchmark of the ASCI determinant search on one MI355X.

One step = one whole search (every step of the path: inputs resident in HBM,
psi keys, class counts, generation, sort, accumulation, exclusion, diagonal +
score, top-k) on the Cr2-shaped (24e,30o) workload: 30 orbitals, 12 alpha +
12 beta electrons, 10^5 core determinants, k = 10^6 (6.7e9 pairs, the
largest single-GPU configuration).  The metric is H_ai C_i contributions per
second: the closed-form number of (core, target) pairs divided by the search
wall time.  The (16e,20o) workload (10^4 cores, k = 10^5) is timed as well
and reported under "extra_workloads".

    python bench.py [--steps K] [--warmup W] [--workload 24e30o] [--no-cpu-baseline]
"""
import argparse
import json
import os
import sys
import time
from math import comb

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "H_ai·C_i contributions/sec + search wall-time; batched/served vs single, p50/p99"
HBM_PEAK_GBS = 8000.0


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` on `workload` from the committed
    rocprofv3 counter summary (FETCH_SIZE and WRITE_SIZE scaled by a plain
    copy), or None when the kernel's sources changed since the counters were
    taken."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "%s_%s_pmc.md" % (kernel, workload))
    if not os.path.exists(path):
        return None
    for line in open(path):
        parts = line.split()
        if not parts or parts[0] != "traffic_record":
            continue
        rec = dict(p.split("=", 1) for p in parts[1:])
        h = hashlib.sha256()
        for f in rec["sources"].split(","):
            h.update(open(os.path.join(ROOT, f), "rb").read())
        if h.hexdigest() != rec["sha256"]:
            return None
        return 1024.0 * (float(rec["fetch_kib"]) * float(rec["fetch_scale"]) +
                         float(rec["write_kib"]) * float(rec["write_scale"]))
    return None


def sd_per_det(n, na, nb):
    va, vb = n - na, n - nb
    return na * va + nb * vb + comb(na, 2) * comb(va, 2) + comb(nb, 2) * comb(vb, 2) + na * va * nb * vb


def cpu_info():
    """(CPU model, logical CPUs, CPUs this process may use)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count(), len(os.sched_getaffinity(0))


def cpu_baseline(case, E0, budget_s=8.0):
    """The oracle, as it stands, on a bounded sample: the first m input
    determinants of the same workload as the wave function (a smaller search
    of the same shape), through the oracle's bucketed search (generate, sort,
    accumulate, exclude, score, each bucket's top k, then the top k of their
    union), once on one thread and once on every host thread this process may
    use (at most 16).  Returns contributions/s with the thread counts and the
    CPU model."""
    import oracle

    oracle.build(force=False)
    n, na, nb, k = case["norb"], case["nalpha"], case["nbeta"], case["k"]
    per = sd_per_det(n, na, nb)
    model, ncpu, avail = cpu_info()
    threads = max(1, min(avail, 16))

    def run(m, th):
        dets, C = case["dets"][:m], case["coeffs"][:m]
        t0 = time.perf_counter()
        r, st = oracle.search_buckets(case["h"], case["eri"], n, na, nb, dets, C, E0, nbuckets=4 * th,
                                      threads=th, keep_top=k)
        oracle.topk_index(r["keys"], r["score"], k)
        return m * per / (time.perf_counter() - t0), time.perf_counter() - t0

    # size the one-thread sample from a short probe, then the all-thread one from it
    m0 = max(1, min(len(case["coeffs"]), int(2.0e5 / per) + 1))
    r0, _ = run(m0, 1)
    m1 = max(1, min(len(case["coeffs"]), int(r0 * budget_s / per)))
    r1, t1 = run(m1, 1)
    mt = max(1, min(len(case["coeffs"]), int(r1 * threads * budget_s / per)))
    rt, tt = run(mt, threads)
    return {"value": rt, "unit": "contributions/s", "cores": threads, "kind": "oracle",
            "sample": "first %d (all threads) and %d (one thread) of %d input determinants of %s as the wave "
                      "function; oracle bucketed search (generate, sort, accumulate, exclude, score, top-%d); "
                      "%.1f s and %.1f s" % (mt, m1, len(case["coeffs"]), case["name"], k, tt, t1),
            "single_thread_value": r1, "cpu_model": model, "nproc": ncpu, "threads_available": avail}


def _dev_case(case, torch, dev):
    import numpy as np

    return (torch.from_numpy(case["h"]).to(dev), torch.from_numpy(case["eri"]).to(dev),
            torch.from_numpy(np.ascontiguousarray(case["dets"]).view(np.int64)).to(dev).view(torch.uint64),
            torch.from_numpy(case["coeffs"]).to(dev))


def mode_levels(args, asci, syn, torch):
    """Search time and class skew by constraint level (the single-GPU analogue
    of the strong-scaling and per-element pair-count study by level)."""
    case = syn.workload(args.workload)
    n, na, nb, k = case["norb"], case["nalpha"], case["nbeta"], case["k"]
    dev = torch.device("cuda", 0)
    h, eri, dets, coeffs = _dev_case(case, torch, dev)
    ctx = asci.Context.get(0)
    E0 = asci.energy(h, eri, n, na, nb, dets, coeffs, ctx=ctx)
    P = len(case["coeffs"]) * sd_per_det(n, na, nb)
    rows = []
    configs = [(1, 0), (2, 0), (3, 0), (4, 0), (5, 0), (6, 0), (6, max(1, P // 4096)), (6, max(1, P // 65536))]
    for level, split in configs:
        m, counts = asci.class_counts(n, na, nb, dets, coeffs, constraint_level=level, split_pairs=split)
        st = asci.class_skew(counts, npes=(8, 64, 256, 1024, 4096))
        asci.search(h, eri, n, na, nb, dets, coeffs, E0, k, constraint_level=level, split_pairs=split, ctx=ctx)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            out = asci.search(h, eri, n, na, nb, dets, coeffs, E0, k, constraint_level=level, split_pairs=split,
                              ctx=ctx)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        rows.append({"level": level, "split_pairs": split, "search_ms": round(ms, 3),
                     "contributions_per_s": P / (ms * 1e-3), "batches": ctx.get_param("last_batches"),
                     "selected": int(out[0].shape[0]), **st})
        print("level %d split %d: %.2f ms, %d classes" % (level, split, ms, st["classes"]), file=sys.stderr,
              flush=True)
    return {"metric": "search wall time and class skew by constraint level", "workload": args.workload,
            "contributions": P, "steps": args.steps, "levels": rows}


def mode_loop(args, asci, syn, torch):
    """The ASCI loop (Alg. 1) from the Hartree-Fock determinant on the
    workload's integrals: per-iteration search / selection / H / Davidson."""
    import numpy as np

    case = syn.workload(args.workload)
    n, na, nb = case["norb"], case["nalpha"], case["nbeta"]
    dev = torch.device("cuda", 0)
    h = torch.from_numpy(case["h"]).to(dev)
    eri = torch.from_numpy(case["eri"]).to(dev)
    hf = np.array([syn.aufbau(n, na, nb)], dtype=np.uint64)
    d0 = torch.from_numpy(hf.view(np.int64)).to(dev).view(torch.uint64)
    c0 = torch.ones(1, dtype=torch.float64, device=dev)
    opts = asci.loop_options(ntdets=args.ntdets, ncore=args.ncore, max_iter=args.iters, e_tol=0.0, pt2=True,
                             davidson_tol=1e-6)
    t0 = time.perf_counter()
    r = asci.run(h, eri, n, na, nb, d0, c0, opts)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return {"metric": "ASCI loop wall time by phase", "workload": args.workload, "ntdets": args.ntdets,
            "ncore": args.ncore, "wall_s": round(wall, 3), "energy": r["energy"], "pt2": r["pt2"],
            "iterations": r["iterations"]}


def _requests(asci, syn, torch, specs, dev):
    reqs, pairs = [], 0
    for sp in specs:
        c = syn.make_case(sp["n"], sp["na"], sp["nb"], sp["ndets"], sp["seed"], sampler=sp["sampler"],
                          tau=sp["tau"], k=sp["k"])
        h, eri, dets, coeffs = _dev_case(c, torch, dev)
        E0 = asci.energy(h, eri, sp["n"], sp["na"], sp["nb"], dets, coeffs)
        reqs.append(asci.SearchRequest(h, eri, sp["n"], sp["na"], sp["nb"], dets, coeffs, E0, sp["k"]))
        pairs += sp["ndets"] * sd_per_det(sp["n"], sp["na"], sp["nb"])
    return reqs, pairs


def _batch_compare(asci, syn, torch, specs, label, solo_pairs=None, slots=None):
    """The searches of `specs` one by one on one context (each bracketed by
    device synchronisations; the total is the sum of those times), then as
    batches: every request on the worker streams, and the requests inside the
    asynchronous search's scope as one captured graph (replayed; the rest on
    the workers at the same time).  Every batch result is compared bit for bit
    with the one-by-one result.  Each batch timing follows an untimed pass
    that sizes the workspaces (and captures the graph)."""
    dev = torch.device("cuda", 0)
    reqs, P = _requests(asci, syn, torch, specs, dev)
    print("%s batch inputs ready: %d searches, %.3g pairs" % (label, len(reqs), P), file=sys.stderr, flush=True)
    ctx = asci.Context.get(0)
    gctx = asci.Context(0)
    if solo_pairs is not None:
        gctx.set_param("batch_solo_pairs", int(solo_pairs))
    if slots is not None:
        gctx.set_param("batch_slots", int(slots))

    def snapshot():
        return [(r.out_dets.view(torch.int64).cpu().numpy().copy(), r.out_scores.cpu().numpy().copy()) for r in reqs]

    for r, sp in zip(reqs, specs):  # warm-up: size the context's workspace
        h, eri, dets, coeffs = r.keep
        asci.search(h, eri, sp["n"], sp["na"], sp["nb"], dets, coeffs, r.c.E0, sp["k"], ctx=ctx)
    torch.cuda.synchronize()
    per, single_out = [], []
    for r, sp in zip(reqs, specs):
        h, eri, dets, coeffs = r.keep
        t1 = time.perf_counter()
        k_, s_ = asci.search(h, eri, sp["n"], sp["na"], sp["nb"], dets, coeffs, r.c.E0, sp["k"], ctx=ctx)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        single_out.append((k_.view(torch.int64).cpu().numpy().copy(), s_.cpu().numpy().copy()))
        pairs = sp["ndets"] * sd_per_det(sp["n"], sp["na"], sp["nb"])
        per.append({"norb": sp["n"], "nalpha": sp["na"], "ndets": sp["ndets"], "k": sp["k"], "pairs": pairs,
                    "single_ms": round(dt * 1e3, 3), "graph": bool(asci.graph_capable(r, ctx=gctx))})
    single = sum(p["single_ms"] for p in per) * 1e-3

    def identical(res):
        got = snapshot()
        return all(rr.status == 0 and int(rr.count) == len(w[0]) and (g[0][:rr.count] == w[0]).all() and
                   (g[1][:rr.count] == w[1]).all() for rr, g, w in zip(res, got, single_out))

    def timed_batch(graph, subset=None):
        gctx.set_param("batch_graph", 1 if graph else 0)
        rs = reqs if subset is None else [reqs[i] for i in subset]
        asci.search_batch(rs, ctx=gctx)  # untimed: workspaces sized, graph captured
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = asci.search_batch(rs, ctx=gctx)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, res

    batch_workers, res_w = timed_batch(False)
    same_w = identical(res_w)
    for p, rr in zip(per, res_w):  # each request's own time inside the batch
        p["batch_run_ms"] = round(rr.run_ms, 3)
    print("%s: one by one %.3f s, worker batch %.3f s (identical %s)" % (label, single, batch_workers, same_w),
          file=sys.stderr, flush=True)
    batch_graph, res_g = timed_batch(True)
    same_g = identical(res_g)
    print("%s: graph batch %.3f s (identical %s)" % (label, batch_graph, same_g), file=sys.stderr, flush=True)
    sub = [i for i, p in enumerate(per) if p["graph"]]
    out = {"searches": len(reqs), "contributions": P, "single_s": round(single, 4),
           "batch_s": round(batch_workers, 4), "batch_graph_s": round(batch_graph, 4),
           "single_contributions_per_s": P / single, "batch_contributions_per_s": P / batch_workers,
           "speedup": single / batch_workers, "speedup_graph": single / batch_graph,
           "identical_to_single": bool(same_g and same_w), "batch_slots": gctx.get_param("batch_slots"),
           "batch_solo_pairs": gctx.get_param("batch_solo_pairs")}
    if sub and len(sub) < len(reqs):
        sub_single = sum(per[i]["single_ms"] for i in sub) * 1e-3
        sub_graph, _ = timed_batch(True, sub)
        sub_workers, _ = timed_batch(False, sub)
        out["graph_subset"] = {"searches": len(sub), "contributions": sum(per[i]["pairs"] for i in sub),
                               "single_s": round(sub_single, 4), "graph_s": round(sub_graph, 4),
                               "workers_s": round(sub_workers, 4), "speedup_graph": sub_single / sub_graph,
                               "speedup_workers": sub_single / sub_workers}
    out["per_search"] = per
    gctx.close()
    return out


def mode_batch(args, asci, syn, torch):
    """Batched vs one-by-one searches on two batches: 64 searches of uneven
    active spaces and core counts (most fill the GPU alone), and 256 small
    searches (each far from filling it)."""
    solo = args.batch_solo_pairs if args.batch_solo_pairs >= 0 else None
    slots = args.batch_slots if args.batch_slots > 0 else None
    return {"metric": "batched vs single searches",
            "uneven": _batch_compare(asci, syn, torch, syn.batch_specs(args.batch_count, seed=64), "uneven", solo,
                                     slots),
            "small": _batch_compare(asci, syn, torch, syn.small_batch_specs(4 * args.batch_count, seed=65), "small",
                                    solo, slots)}


SERVE_MIX = [(0.70, dict(n=20, na=8, nb=8, ndets=1_000)), (0.25, dict(n=26, na=10, nb=10, ndets=10_000)),
             (0.05, dict(n=30, na=12, nb=12, ndets=100_000))]


def mode_serve(args, asci, syn, torch):
    """Poisson arrivals of a 70/25/5 mix of (16e,20o)/10^3, (20e,26o)/10^4 and
    (24e,30o)/10^5 searches (k = 10 x cores) against the request server:
    each class's time alone, saturated throughput (after a warm-up pass),
    then latency p50/p99 at fractions of it, overall and per class, against
    1.5 x the largest class's time alone."""
    import numpy as np

    dev = torch.device("cuda", 0)
    pools = []
    for frac, base in SERVE_MIX:
        npool = 4 if base["ndets"] <= 1000 else (2 if base["ndets"] <= 10_000 else 1)
        specs = [dict(base, seed=500 + 10 * len(pools) + j, sampler="level", tau=base["ndets"] / 10.0,
                      k=10 * base["ndets"]) for j in range(npool)]
        reqs, P = _requests(asci, syn, torch, specs, dev)
        pools.append((frac, reqs, P / len(reqs), "%de%do/%d" % (base["na"] + base["nb"], base["n"], base["ndets"])))
    print("serve pools ready", file=sys.stderr, flush=True)
    rng = np.random.default_rng(55)

    def draw(count):
        out = []
        for _ in range(count):
            u, acc = rng.random(), 0.0
            for ci, (frac, reqs, per, _) in enumerate(pools):
                acc += frac
                if u <= acc:
                    out.append((reqs[int(rng.integers(len(reqs)))], per, ci))
                    break
            else:
                out.append((pools[-1][1][0], pools[-1][2], len(pools) - 1))
        return out

    srv = asci.Server(device=0, slots=args.slots)
    # each class alone on the server (after one untimed run)
    solo = []
    for _, reqs, _, name in pools:
        srv.wait(srv.submit(reqs[0]))
        ts = []
        for _ in range(3):
            t0 = time.perf_counter()
            srv.wait(srv.submit(reqs[0]))
            ts.append((time.perf_counter() - t0) * 1e3)
        solo.append(min(ts))
        print("alone %s: %.1f ms" % (name, solo[-1]), file=sys.stderr, flush=True)
    bar_ms = 1.5 * max(solo)
    # saturated: everything queued at once, timed after an untimed pass of the
    # same requests that sizes the workers' workspaces
    batch = draw(args.requests)
    for i, t in enumerate([srv.submit(r) for r, _, _ in batch]):
        srv.wait(t)
        if (i + 1) % 250 == 0:
            print("saturated warm-up: %d done" % (i + 1), file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    tickets = [srv.submit(r) for r, _, _ in batch]
    for i, t in enumerate(tickets):
        srv.wait(t)
        if (i + 1) % 250 == 0:
            print("saturated: %d done" % (i + 1), file=sys.stderr, flush=True)
    sat_s = time.perf_counter() - t0
    sat_qps = len(batch) / sat_s
    sat_cps = sum(per for _, per, _ in batch) / sat_s
    print("saturated: %.2f requests/s" % sat_qps, file=sys.stderr, flush=True)
    points = []
    for f in (0.5, 0.75, 0.9):
        qps = f * sat_qps
        batch = draw(args.requests)
        gaps = rng.exponential(1.0 / qps, len(batch))
        due = time.perf_counter()
        sent = []
        for i, ((r, _, ci), g) in enumerate(zip(batch, gaps)):
            due += g
            now = time.perf_counter()
            if due > now:
                time.sleep(due - now)
            sent.append((srv.submit(r), ci))
            if (i + 1) % 500 == 0:
                print("load %.2f: %d sent" % (f, i + 1), file=sys.stderr, flush=True)
        res = [(srv.wait(t), ci) for t, ci in sent]
        st = srv.stats()
        lat = np.array([x.latency_ms for x, _ in res])
        cls = np.array([ci for _, ci in res])
        per_class = {}
        for ci, (_, _, _, name) in enumerate(pools):
            m = lat[cls == ci]
            if len(m):
                per_class[name] = {"requests": int(len(m)), "p50_ms": float(np.percentile(m, 50)),
                                   "p99_ms": float(np.percentile(m, 99)), "alone_ms": round(solo[ci], 2)}
        points.append({"load": f, "qps": round(qps, 3), "requests": len(batch),
                       "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                       "p99_over_bar": float(np.percentile(lat, 99)) / bar_ms, "per_class": per_class,
                       "max_running": st["max_running"], "bypassed": st["bypassed"]})
        print("load %.2f: p50 %.1f ms p99 %.1f ms (bar %.1f ms)" % (f, points[-1]["p50_ms"], points[-1]["p99_ms"],
                                                                  bar_ms), file=sys.stderr, flush=True)
    srv.close()
    return {"metric": "served searches: saturated throughput and latency under Poisson load",
            "mix": "70% (16e,20o)/1e3, 25% (20e,26o)/1e4, 5% (24e,30o)/1e5; k = 10 x cores",
            "requests_per_point": args.requests, "slots": args.slots,
            "alone_ms": [round(x, 2) for x in solo],
            "p99_bar_ms": bar_ms, "saturated_qps": sat_qps, "saturated_contributions_per_s": sat_cps,
            "points": points}


def mode_host(args, asci, syn, torch):
    """The host-buffer entry point (asci_search): inputs uploaded and results
    downloaded inside the timed call (PCIe included)."""
    case = syn.workload(args.workload)
    n, na, nb, k = case["norb"], case["nalpha"], case["nbeta"], case["k"]
    h, eri, dets, coeffs = _dev_case(case, torch, torch.device("cuda", 0))
    E0 = asci.energy(h, eri, n, na, nb, dets, coeffs)
    asci.search_host(case["h"], case["eri"], n, na, nb, case["dets"], case["coeffs"], E0, k)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        asci.search_host(case["h"], case["eri"], n, na, nb, case["dets"], case["coeffs"], E0, k)
    dt = (time.perf_counter() - t0) / args.steps
    P = len(case["coeffs"]) * sd_per_det(n, na, nb)
    return {"metric": "host-buffer search (PCIe inclusive)", "workload": args.workload, "ms": round(dt * 1e3, 3),
            "contributions_per_s": P / dt}


def mode_copy(args, asci, syn, torch):
    """A plain device-to-device copy of known size: the reference for scaling
    the FETCH_SIZE / WRITE_SIZE counters of the search kernels."""
    nbytes = 1 << 30
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        dst.copy_(src)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    return {"metric": "device copy (counter reference)", "bytes_read": nbytes, "bytes_written": nbytes,
            "copies": args.steps, "ms_per_copy": round(dt * 1e3, 4), "GB/s": 2 * nbytes / dt / 1e9}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="24e30o")
    ap.add_argument("--extra", default="16e20o", help="search mode: further workloads timed (comma list, 'none' for none)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--finish-cap", type=int, default=0, help="records per LDS bucket (tuning parameter)")
    ap.add_argument("--mode", default="search", choices=["search", "levels", "loop", "batch", "serve", "copy", "host"],
                    help="search: the benchmark line; the others print their own measurement")
    ap.add_argument("--ntdets", type=int, default=10_000, help="loop mode: N_tdets")
    ap.add_argument("--ncore", type=int, default=0, help="loop mode: N_cdets (0 = all)")
    ap.add_argument("--iters", type=int, default=4, help="loop mode: outer iterations")
    ap.add_argument("--batch-count", type=int, default=64, help="batch mode: searches")
    ap.add_argument("--batch-slots", type=int, default=0, help="batch mode: worker slots (0: the library default)")
    ap.add_argument("--batch-solo-pairs", type=int, default=-1,
                    help="batch mode: pairs at which a request runs alone (-1: the library default)")
    ap.add_argument("--requests", type=int, default=2000, help="serve mode: requests per load point")
    ap.add_argument("--slots", type=int, default=4, help="serve mode: server worker slots")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (the search shards by "
              "constraint class across GPUs only in design); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import asci_synth as syn
    import paper_2303_05688_amd as asci

    if args.mode != "search":
        fn = {"levels": mode_levels, "loop": mode_loop, "batch": mode_batch, "serve": mode_serve,
              "copy": mode_copy, "host": mode_host}[args.mode]
        print(json.dumps(fn(args, asci, syn, torch)), flush=True)
        return

    ctx = asci.Context.get(0)
    if args.finish_cap:
        ctx.set_param("finish_cap", args.finish_cap)
    line = measure_search(args, asci, syn, torch, np, ctx, args.workload, args.steps, args.warmup, full=True)
    extras = [w for w in args.extra.split(",") if w and w not in ("none", args.workload)]
    if extras:
        line["extra_workloads"] = {}
        for w in extras:
            print("extra workload %s ..." % w, file=sys.stderr, flush=True)
            line["extra_workloads"][w] = measure_search(args, asci, syn, torch, np, ctx, w, max(args.steps, 5),
                                                        max(args.warmup, 2), full=False)
    if not args.no_cpu_baseline:
        print("cpu baseline (oracle sample) ...", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(line.pop("_case"), line.pop("_E0"))
    else:
        line.pop("_case")
        line.pop("_E0")
    print(json.dumps(line), flush=True)


def measure_search(args, asci, syn, torch, np, ctx, workload, steps, warmup, full):
    """Time `steps` whole searches of `workload` after `warmup` untimed ones.
    full: the headline line (roofline of the dominant kernel, per-phase
    breakdown); otherwise the rate and wall time only."""
    case = syn.workload(workload)
    n, na, nb = case["norb"], case["nalpha"], case["nbeta"]
    nd, k = len(case["coeffs"]), case["k"]
    dev = torch.device("cuda", 0)
    h = torch.from_numpy(case["h"]).to(dev)
    eri = torch.from_numpy(case["eri"]).to(dev)
    dets = torch.from_numpy(np.ascontiguousarray(case["dets"]).view(np.int64)).to(dev).view(torch.uint64)
    coeffs = torch.from_numpy(case["coeffs"]).to(dev)
    E0 = asci.energy(h, eri, n, na, nb, dets, coeffs, ctx=ctx)
    P = nd * sd_per_det(n, na, nb)

    def step():
        return asci.search(h, eri, n, na, nb, dets, coeffs, E0, k, ctx=ctx)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    print("%s: warmup done" % workload, file=sys.stderr, flush=True)
    desc = "%s: (%de,%do) synthetic integrals, %d core determinants, keep %d" % (workload, na + nb, n, nd, k)
    if not full:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            out_k, out_s = step()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1000.0 / steps
        return {"workload": desc, "value": P / (ms * 1e-3), "unit": "contributions/s", "ms_per_step": round(ms, 4),
                "steps": steps, "contributions": P, "selected": int(out_k.shape[0])}
    # every kernel timed (outside the timed region): the per-phase breakdown and
    # the dominant kernel, the one with the largest total time
    nph = max(1, min(steps, 3))
    ctx.set_profiling(True)
    for _ in range(nph):
        step()
    torch.cuda.synchronize()
    allprof = ctx.profile()
    ctx.set_profiling(False)
    name = max(allprof.items(), key=lambda kv: kv[1][0])[0]
    # timed region: HIP events bracket only the dominant kernel's launches
    ctx.set_profiling(True, only=name)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        out_k, out_s = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = ctx.profile()
    ctx.set_profiling(False)
    ms = (t1 - t0) * 1000.0 / steps
    print("%s: timed steps done" % workload, file=sys.stderr, flush=True)

    kms, launches, kbytes = prof[name]
    avg_ms = kms / max(launches, 1)
    achieved = (kbytes / max(launches, 1)) / (avg_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "kernel": name, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(name, workload),
                "avg_launch_ms": round(avg_ms, 4), "launches_per_step": launches / steps,
                "algorithmic_bytes_per_launch": kbytes / max(launches, 1)}
    phases = {kname: {"ms_per_step": round(v[0] / nph, 4), "launches_per_step": v[1] / nph,
                      "GB/s": round((v[2] / max(v[0], 1e-9)) / 1e6, 1)} for kname, v in sorted(allprof.items())}
    return {
        "metric": METRIC,
        "value": P / (ms * 1e-3),
        "unit": "contributions/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": desc, "norb": n, "nalpha": na, "nbeta": nb, "ndets": nd, "k": k,
                   "contributions": P, "seed": case["seed"], "finish_cap": ctx.get_param("finish_cap")},
        "search_wall_ms": round(ms, 4),
        "diagnostics": {kk: ctx.get_param(kk) for kk in ("last_batches", "last_finals", "last_levels",
                                                          "last_candidates")},
        "selected": int(out_k.shape[0]),
        "roofline": roofline,
        "phases": phases,
        "phases_steps": nph,
        "_case": case,
        "_E0": E0,
    }


if __name__ == "__main__":
    main()
