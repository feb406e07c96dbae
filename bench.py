#!/usr/bin/env python3
"""Benchmark of the persistent-thread dispatch path on one MI355X.

Headline workload (one worker per CU, all CUs): every mailbox is fed fp32 SAXPY items
y <- alpha*x + y over 16,384 elements back-to-back, 10,000 items per mailbox in total
(10 steps of 1,000 items per mailbox).  One step = every mailbox receiving 1,000 items
through post -> poll -> execute -> complete -> wait; the context is booted before the
warm-up and disposed after the timed steps (boot and dispose times are reported apart).

Printed as one JSON line: items/s of the persistent path (value), its dispatch latency
percentiles, the same workload as one hipLaunchKernelGGL per item and as a relaunched
hipGraph, the serial single-worker comparison (1 CU, affine+sum over 4,096 int32), the
ping-pong latency floor, the HBM roofline of the worker kernel and the CPU oracle timed
on a bounded sample of the same workload.

Inputs are seeded synthetic data resident in HBM before the timed region.
"""
import argparse
import concurrent.futures as cf
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
METRIC = "dispatch latency p50/p99/max (µs) + work items/s, persistent vs per-launch"


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def pct(v, p):
    """Nearest-rank percentile: sorted[ceil(p*N) - 1]."""
    v = np.sort(np.asarray(v, dtype=np.float64).ravel())
    if v.size == 0:
        return float("nan")
    k = max(1, int(np.ceil(p * v.size)))
    return float(v[k - 1])


def lat_summary(v):
    return {"p50": round(pct(v, 0.50), 3), "p99": round(pct(v, 0.99), 3),
            "p999": round(pct(v, 0.999), 3), "max": round(pct(v, 1.0), 3),
            "jitter": round(pct(v, 1.0) - pct(v, 0.0), 3)}


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "lk_worker_allcu_saxpy_traffic.md")
WORKER_SOURCES = ["lk_worker.hip", "lk_ops.hpp", "lk_devutil.hpp", "lk_wire.h"]


def worker_source_digest():
    import hashlib
    h = hashlib.sha256()
    for f in WORKER_SOURCES:
        with open(os.path.join(ROOT, "paper_2310_01212_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_per_item(n):
    """HBM bytes per item of the worker kernel from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE passes, scaled by the copy-probe calibration);
    None when the summary is missing, was taken for another item size, or the worker's
    sources changed since."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    text = open(TRAFFIC_FILE).read()
    import re
    m = re.search(r"```json\n(.*?)\n```", text, re.S)
    if not m:
        return None
    d = json.loads(m.group(1))
    if d.get("worker_source_digest") != worker_source_digest() or d.get("n") != n:
        return None
    return {"bytes_per_item": d["hbm_bytes_per_item"], "source": os.path.relpath(TRAFFIC_FILE, ROOT)}


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--items-per-step", type=int, default=1000, help="items per mailbox per step")
    ap.add_argument("--n", type=int, default=16384, help="elements per item")
    ap.add_argument("--depth", type=int, default=1, help="ring slots per mailbox (in flight)")
    ap.add_argument("--threads", type=int, default=max(1, min(14, (os.cpu_count() or 2) - 2)),
                    help="host feeder threads (one producer per mailbox)")
    ap.add_argument("--poll-sleep", type=int, default=0)
    ap.add_argument("--baseline-steps", type=int, default=1, help="steps timed for each baseline")
    ap.add_argument("--streams", type=int, default=4, help="HIP streams of the per-launch baseline")
    ap.add_argument("--skip-baselines", action="store_true")
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--cpu-items", type=int, default=1000, help="items per mailbox in the CPU sample")
    ap.add_argument("--copy-probe-mib", type=int, default=1024)
    ap.add_argument("--workload", choices=["allcu", "isolation"], default="allcu",
                    help="allcu: the headline all-CU workload; isolation: cluster 0 critical "
                         "item every period beside streaming copies on the other XCDs")
    ap.add_argument("--periods", type=int, default=10000, help="isolation: periods per variant")
    ap.add_argument("--period-us", type=float, default=1000.0)
    ap.add_argument("--copy-mib", type=int, default=256, help="isolation: interference buffer size")
    return ap.parse_args()


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}): "
              "the dispatch path has no multi-GPU component; see DESIGN.md for how it would shard.",
              file=sys.stderr)
        sys.exit(2)
    if args.workload == "isolation":
        return bench_isolation(args)
    return bench_allcu(args)


def bench_isolation(args):
    """Cluster isolation: 8 clusters = 8 XCDs; cluster 0 gets a critical int32 affine +
    int64 sum item over 262,144 elements every period, released by a host busy-wait, while
    clusters 1-7 copy private fp32 buffers back-to-back (interference on) or idle-poll
    (interference off)."""
    import torch
    import oracle
    from paper_2310_01212_amd import lk, workloads

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    lk.lib()
    oracle.build(force=False)
    dev = torch.device("cuda:0")
    P = args.periods
    log(f"isolation: generating inputs ({P} periods, {args.copy_mib} MiB copies)")
    xh, AB = workloads.isolation(periods=P)
    x = torch.from_numpy(xh).to(dev)
    y = torch.zeros_like(x)
    elems = (args.copy_mib << 20) // 4
    srcs = [workloads.isolation_copy_source_device(c, elems, dev) for c in range(1, 8)]
    dsts = [torch.empty_like(s) for s in srcs]
    torch.cuda.synchronize()
    crit = lk.make_items(lk.OP_AFFINE_SUM_I32, xh.size, x.data_ptr(), y.data_ptr(), AB[:, 0], AB[:, 1])
    bg = lk.make_items(lk.OP_COPY_F32, elems, [s.data_ptr() for s in srcs], [d.data_ptr() for d in dsts])
    out = {"metric": "critical-item latency p50/p99/p99.9/max (µs) under cross-XCD interference",
           "unit": "us", "higher_is_better": False, "n_gpus": 1, "dtype": "int32/int64 (critical), f32 copy",
           "data": "synthetic (seeded)", "steps": P, "warmup": 0, "scaling": "weak", "vs_baseline": None,
           "config": {"workload": "cluster isolation: 8 clusters = 8 XCDs; cluster 0 critical affine+sum over "
                                  f"{xh.size} int32 every {args.period_us} us; clusters 1-7 copy private "
                                  f"{args.copy_mib} MiB fp32 buffers back-to-back", "periods": P}}
    with lk.Context(n_workers=0, clusters=lk.CLUSTERS_PER_XCD, idle_timeout_ms=600000) as ctx:
        ncl = ctx.info()["n_clusters"]
        assert ncl == 8, f"expected 8 XCD clusters, got {ncl}"
        ctx.run_isolation(0, crit[:200], args.period_us * 1e-6, [], bg[:0])  # warm-up, untimed
        for name, bgc in (("off", []), ("on", list(range(1, 8)))):
            log(f"isolation: interference {name}")
            r = ctx.run_isolation(0, crit, args.period_us * 1e-6, bgc, bg[:len(bgc)])
            wall = 1e8
            span = (r["info"]["t_done_max"] - r["info"]["t_pick_min"]) / wall * 1e6
            v = {"latency_us": lat_summary(r["lat_us"]), "device_span_us": lat_summary(span),
                 "release_lateness_us": lat_summary(r["late_us"]), "elapsed_s": round(r["elapsed_s"], 3)}
            if bgc:
                copied = float(r["bg_done"].sum()) * 2 * (elems * 4)
                v["interference_copy_gbps"] = round(copied / r["elapsed_s"] / 1e9, 1)
                v["interference_items"] = int(r["bg_done"].sum())
            # spot parity: sums of 20 sampled periods against the oracle
            idx = np.linspace(0, P - 1, 20).astype(int)
            bad = sum(int(r["results"][k] != oracle.affine_sum_i32(xh, int(AB[k, 0]), int(AB[k, 1]))[1]) for k in idx)
            v["sampled_sum_mismatches"] = bad
            out[name] = v
    out["value"] = out["on"]["latency_us"]["max"]
    out["ms_per_step"] = round(out["on"]["elapsed_s"] * 1e3 / P, 4)
    print(json.dumps(out), flush=True)


def bench_allcu(args):
    import torch
    from paper_2310_01212_amd import lk, workloads

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    lk.lib()
    dev = torch.device("cuda:0")
    props = torch.cuda.get_device_properties(0)
    lanes = props.multi_processor_count
    n, per = args.n, args.items_per_step
    total_items = (args.warmup + args.steps) * per

    # ---------------- inputs (seeded, resident in HBM before any timed region)
    log(f"generating inputs: {lanes} lanes, n={n}, {total_items} items per lane")
    X = np.empty((lanes, n), np.float32)
    Y0 = np.empty((lanes, n), np.float32)
    A = np.empty((lanes, max(total_items, workloads.ALLCU_ITEMS)), np.float32)
    for w in range(lanes):
        x, y, a = workloads.allcu_lane(w, items=A.shape[1], n=n)
        X[w], Y0[w], A[w] = x, y, a
    x_d = torch.from_numpy(X).to(dev)
    y_d = torch.from_numpy(Y0).to(dev)
    torch.cuda.synchronize()
    li = np.arange(lanes, dtype=np.uint64)[:, None]
    x_addr = x_d.data_ptr() + li * n * 4
    y_addr = y_d.data_ptr() + li * n * 4

    # every step's descriptors are built before any timed region
    steps_items = [lk.make_items(lk.OP_SAXPY_F32, n, x_addr, y_addr, alpha=A[:, s * per:(s + 1) * per])
                   for s in range(args.warmup + args.steps)]

    def step_items(s):
        return steps_items[s]

    bytes_per_item = 12 * n  # SAXPY: 8n read + 4n write

    # ---------------- persistent path
    log("persistent path: boot")
    ctx = lk.Context(n_workers=lanes, depth=args.depth, poll_sleep=args.poll_sleep, idle_timeout_ms=60000)
    info0 = ctx.info()
    for s in range(args.warmup):
        ctx.run_lanes(np.arange(lanes), step_items(s), in_flight=args.depth, threads=args.threads)
    log("persistent path: timed steps")
    torch.cuda.synchronize()
    lat_all = []
    t0 = time.perf_counter()
    for s in range(args.warmup, args.warmup + args.steps):
        _, lat, _ = ctx.run_lanes(np.arange(lanes), step_items(s), in_flight=args.depth, threads=args.threads)
        lat_all.append(lat)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ctx.close()
    info = ctx.info()
    lat_all = np.concatenate([l.ravel() for l in lat_all])
    timed_items = lanes * per * args.steps
    items_per_s = timed_items / elapsed
    # duration of the single worker dispatch: packet-processor timestamps, or (when a tool
    # intercepting the queue hides them) the span from first boot to last exit on the
    # device wall clock
    kernel_ms, kernel_clock = info["kernel_ms"], "dispatch timestamps"
    if kernel_ms <= 0:
        kernel_ms, kernel_clock = info["device_span_ms"], "device wall clock"
    session_items = lanes * per * (args.warmup + args.steps)
    achieved_gbps = session_items * bytes_per_item / (kernel_ms * 1e-3) / 1e9 if kernel_ms > 0 else 0.0
    log(f"persistent: {items_per_s:,.0f} items/s, p50 {pct(lat_all, .5):.2f} us, kernel {kernel_ms:.1f} ms")

    result = {
        "metric": METRIC,
        "value": round(items_per_s, 1),
        "unit": "items/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed * 1e3 / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded: x, y ~ N(0,1), alpha ~ U(-2,2) per mailbox)",
        "config": {"workload": "all-CU SAXPY: one worker per CU, each mailbox fed items back-to-back",
                   "workers": lanes, "items_per_mailbox": per * args.steps, "n": n,
                   "item_bytes": bytes_per_item, "queue_depth": args.depth,
                   "host_threads": args.threads, "poll_sleep": args.poll_sleep},
        "latency_us": lat_summary(lat_all),
        "init_ms": round(info0["init_ms"], 3),
        "dispose_ms": round(info["dispose_ms"], 3),
    }

    # ---------------- roofline of the worker kernel (one launch = the session)
    result["roofline"] = {"bound": "hbm", "achieved": round(achieved_gbps, 1), "peak": HBM_PEAK_GBPS,
                          "unit": "GB/s", "frac": round(achieved_gbps / HBM_PEAK_GBPS, 4), "traffic": None,
                          "kernel": "lk_worker", "kernel_ms": round(kernel_ms, 3), "kernel_clock": kernel_clock,
                          "items_per_launch": session_items, "algorithmic_bytes_per_item": bytes_per_item,
                          "algorithmic_bytes": session_items * bytes_per_item}
    tr = traffic_per_item(n)
    if tr is not None:
        result["roofline"]["traffic"] = round(tr["bytes_per_item"] * session_items)
        result["roofline"]["traffic_source"] = tr["source"]

    # ---------------- baselines on the same workload
    if not args.skip_baselines:
        base = {}
        for name, mode in (("launch", 0), ("graph", lk.USE_GRAPH)):
            bl = []
            t0 = time.perf_counter()
            for s in range(args.baseline_steps):
                _, lat, el = lk.launch_lanes(step_items(s), streams=args.streams, threads_host=args.threads,
                                             mode=mode)
                bl.append(lat)
            el = time.perf_counter() - t0
            bl = np.concatenate([b.ravel() for b in bl])
            base[name] = {"items_per_s": round(bl.size / el, 1), "latency_us": lat_summary(bl),
                          "streams": args.streams, "items": int(bl.size)}
            log(f"{name}: {bl.size / el:,.0f} items/s, p50 {pct(bl, .5):.2f} us")
        result["baselines"] = base
        result["speedup_items_per_s"] = {k: round(items_per_s / v["items_per_s"], 2) for k, v in base.items()}

        # serial single-worker comparison (1 CU, 1000 affine+sum items of 4096 int32)
        Xs, ABs = workloads.plain()
        xs = torch.from_numpy(Xs).to(dev)
        ys = torch.zeros_like(xs)
        torch.cuda.synchronize()
        rows = np.arange(Xs.shape[0], dtype=np.uint64)
        items = lk.make_items(lk.OP_AFFINE_SUM_I32, Xs.shape[1], xs.data_ptr() + rows * Xs.shape[1] * 4,
                              ys.data_ptr() + rows * Xs.shape[1] * 4, ABs[:, 0], ABs[:, 1])
        with lk.Context(n_workers=1, idle_timeout_ms=30000) as c1:
            c1.run_serial(0, items[:100])
            _, lat_p, trig_p, _ = c1.run_serial(0, items)
        serial = {"persistent": lat_summary(lat_p), "persistent_trigger": lat_summary(trig_p)}
        for name, mode in (("launch_sync", lk.COMPLETE_SYNC), ("launch_flag", lk.COMPLETE_FLAG),
                           ("graph_sync", lk.COMPLETE_SYNC | lk.USE_GRAPH),
                           ("graph_flag", lk.COMPLETE_FLAG | lk.USE_GRAPH)):
            lk.launch_serial(items[:100], mode=mode)
            _, lat_b, lau_b = lk.launch_serial(items, mode=mode)
            serial[name] = lat_summary(lat_b)
            serial[name + "_launch_call"] = lat_summary(lau_b)
        rtt = lk.pingpong(workers=1, iters=5000)[:, 500:]
        serial["pingpong_rtt"] = lat_summary(rtt)
        result["serial_1cu"] = {"workload": "1 worker on 1 CU, 1000 submit-then-wait items: int32 affine "
                                            "+ int64 sum over 4096 elements", **serial}
        result["latency_roofline"] = {"floor": "host<->device coherent ping-pong RTT p50",
                                      "floor_us": serial["pingpong_rtt"]["p50"],
                                      "dispatch_p50_us": serial["persistent"]["p50"],
                                      "frac": round(serial["pingpong_rtt"]["p50"] / serial["persistent"]["p50"], 3)}
        log(f"serial: persistent p50 {serial['persistent']['p50']} us, launch p50 {serial['launch_sync']['p50']} us")

    # ---------------- streaming-copy probe (HBM roofline reference, known-size kernel)
    nbytes = args.copy_probe_mib << 20
    src = torch.empty(nbytes // 4, dtype=torch.int32, device=dev)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    ms, gbps = lk.copy_bandwidth(src, dst, nbytes, grid=lanes * 8, reps=5)
    result["copy_probe"] = {"bytes": nbytes, "ms": round(ms, 4), "gbps": round(gbps, 1),
                            "frac_of_peak": round(gbps / HBM_PEAK_GBPS, 4)}
    del src, dst

    # ---------------- CPU oracle on a bounded sample of the same workload
    if not args.skip_cpu:
        import oracle
        oracle.build(force=False)
        cores = min(16, os.cpu_count() or 1)
        per_cpu = args.cpu_items

        ys = [Y0[w].copy() for w in range(lanes)]
        jobs = [[dict(op=oracle.SAXPY_F32, inp=X[w], out=ys[w], alpha=a) for a in A[w, :per_cpu]]
                for w in range(lanes)]

        def lane_job(w):
            oracle.run_fifo(jobs[w])

        t0 = time.perf_counter()
        with cf.ThreadPoolExecutor(max_workers=cores) as ex:
            list(ex.map(lane_job, range(lanes)))
        el = time.perf_counter() - t0
        result["cpu_baseline"] = {"value": round(lanes * per_cpu / el, 1), "unit": "items/s", "cores": cores,
                                  "kind": "oracle",
                                  "sample": f"{lanes} mailboxes x {per_cpu} SAXPY items of {n} fp32 "
                                            f"({lanes * per_cpu} items), lanes spread over {cores} threads",
                                  "seconds": round(el, 3)}
        log(f"cpu oracle: {lanes * per_cpu / el:,.0f} items/s on {cores} threads")

    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
