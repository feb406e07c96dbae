#!/usr/bin/env python3
"""Benchmark of the persistent-thread dispatch path on one MI355X.

Headline workload (one worker per CU, all CUs): every mailbox is fed fp32 SAXPY items
y <- alpha*x + y over 16,384 elements back-to-back, 10,000 items per mailbox in total
(10 steps of 1,000 items per mailbox).  One step = every mailbox receiving 1,000 items
through post -> poll -> execute -> complete -> wait; the warm-up steps run first, then
the timed steps run as one stream per mailbox (no pause at step boundaries); the context
is booted before the warm-up and disposed after the timed steps (boot and dispose times
are reported apart).

Printed as one JSON line: items/s of the persistent path (value), its dispatch latency
percentiles and their split into device span and host link, the latency bound it is
measured against (roofline), the same workload as one hipLaunchKernelGGL per item, as a
relaunched hipGraph and as captured per-lane graph chains, its variants (ring kept ahead,
two workers per CU, operands streaming from HBM with their HBM roofline, x pinned in
LDS), the serial single-worker comparison (1 CU, affine+sum over 4,096 int32), the
ping-pong latency floors, the streaming-copy probes, shortened runs of the cluster
isolation, serving, batching and replay workloads, and the CPU oracle timed on a bounded
sample of the same workload.

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
    v = np.asarray(v, dtype=np.float64).ravel()
    return {"p50": round(pct(v, 0.50), 3), "p99": round(pct(v, 0.99), 3),
            "p999": round(pct(v, 0.999), 3), "max": round(pct(v, 1.0), 3),
            "jitter": round(pct(v, 1.0) - pct(v, 0.0), 3),
            "mean": round(float(v.mean()), 3) if v.size else float("nan")}


def gb_per_s(bytes_total, ms):
    """Bytes over a duration in milliseconds, in GB/s (0 for a non-positive duration)."""
    return bytes_total / (ms * 1e-3) / 1e9 if ms > 0 else 0.0


def latency_bound(mailboxes, echo_us, item_us, depth):
    """Items/s bound of mailboxes fed back-to-back: at depth 1 each item of a mailbox costs
    at least one host round trip (the echo) plus the item's device span; with the ring kept
    ahead the round trip can hide behind the item.  Returns (floor_us, items_per_s)."""
    floor_us = (echo_us if depth == 1 else 0.0) + item_us
    return floor_us, mailboxes / (floor_us * 1e-6)


def hbm_roofline(bytes_per_launch, kernel_ms, copy_gbps=None, traffic=None, **extra):
    """Roofline object of a bandwidth-bound kernel launch against the HBM peak (and, when
    given, the best streaming copy measured in the same run)."""
    a = gb_per_s(bytes_per_launch, kernel_ms)
    r = {"bound": "hbm", "achieved": round(a, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
         "frac": round(a / HBM_PEAK_GBPS, 4), "traffic": traffic,
         "kernel_ms": round(kernel_ms, 3), **extra}
    if copy_gbps:
        r["copy_probe_gbps"] = copy_gbps
        r["frac_of_copy_probe"] = round(a / copy_gbps, 4)
    return r


def int_sum_check(x, a=None, b=None):
    """Sanity value for a sampled result: int64 sum of x (int32), or of the int32 affine
    map a*x + b mod 2^32 when a is given.  Parity proper is established by the tests."""
    if a is None:
        return int(x.astype(np.int64).sum())
    y = (x.view(np.uint32) * np.uint32(a & 0xffffffff) + np.uint32(b & 0xffffffff)).view(np.int32)
    return int(y.astype(np.int64).sum())


TRAFFIC_FILES = [os.path.join(ROOT, "profiles", f) for f in
                 ("lk_worker_allcu_saxpy_traffic.md", "lk_worker_allcu_saxpy_pinned_traffic.md",
                  "lk_worker_allcu_saxpy_depth4_traffic.md", "lk_worker_allcu_saxpy_cold_traffic.md",
                  "lk_worker_allcu_saxpy_cold_depth4_traffic.md")]
WORKER_SOURCES = ["lk_worker.hip", "lk_ops.hpp", "lk_devutil.hpp", "lk_wire.h", "lk_device.h", "lk_common.h"]


def worker_source_digest(csrc=os.path.join(ROOT, "paper_2310_01212_amd", "csrc")):
    """First 16 hex digits of the sha256 of the worker's sources with comments removed and
    whitespace collapsed, so that a counter summary stays valid across comment edits."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in WORKER_SOURCES:
        with open(os.path.join(csrc, f)) as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def traffic_per_item(n, threads_per_worker, pin_input=False, depth=1, cold_pairs=0):
    """Memory bytes per item of the worker kernel from a committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE passes, scaled by the copy-probe calibration); None
    when no summary was taken for this item size, workgroup size, pinning, ring depth and
    operand rotation, or the worker's sources changed since."""
    import re
    for path in TRAFFIC_FILES:
        if not os.path.exists(path):
            continue
        m = re.search(r"```json\n(.*?)\n```", open(path).read(), re.S)
        if not m:
            continue
        d = json.loads(m.group(1))
        if (d.get("worker_source_digest") == worker_source_digest() and d.get("n") == n and
                d.get("threads_per_worker", 256) == threads_per_worker and
                bool(d.get("pin_input", False)) == bool(pin_input) and d.get("queue_depth", 1) == depth and
                d.get("cold_pairs", 0) == cold_pairs):
            return {"bytes_per_item": d["hbm_bytes_per_item"], "source": os.path.relpath(path, ROOT)}
    return None


def host_cpu_model():
    """Model name of the host CPU as lscpu reports it (/proc/cpuinfo if lscpu is missing)."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.strip().startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        with open("/proc/cpuinfo") as fh:
            return next((l.split(":", 1)[1].strip() for l in fh if l.startswith("model name")), "")
    except OSError:
        return ""


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--items-per-step", type=int, default=1000, help="items per mailbox per step")
    ap.add_argument("--n", type=int, default=16384, help="elements per item")
    ap.add_argument("--depth", type=int, default=1, help="ring slots per mailbox (in flight)")
    ap.add_argument("--threads-per-worker", type=int, default=1024,
                    help="workgroup size of each persistent worker and of the per-launch baselines "
                         "(1024 = four wave64 per SIMD; the 1-CU serial comparison keeps 256)")
    ap.add_argument("--pipelined-depth", type=int, default=4,
                    help="ring depth of the pipelined variant reported beside the depth-1 headline (0 = skip)")
    ap.add_argument("--cold-pairs", type=int, default=16,
                    help="(x, y) pairs each mailbox rotates through in the cold variant, 512 MiB in "
                         "aggregate at 16 (0/1 = skip)")
    ap.add_argument("--no-pinned", dest="pinned", action="store_false",
                    help="skip the pinned-input (x kept in LDS) variants")
    ap.add_argument("--pin-input", action="store_true",
                    help="time the all-CU workload itself with x pinned in each worker's LDS "
                         "(its roofline then counts the 8n HBM bytes per item of y alone)")
    ap.add_argument("--cold", type=int, default=0, metavar="P",
                    help="time the all-CU workload itself in its cold form: each mailbox rotates through "
                         "P (x, y) pairs (item k uses pair k mod P; 512 MiB in aggregate at 16), so the "
                         "operands stream from HBM (0/1 = the headline's fixed pair)")
    ap.add_argument("--variant-per-cu", type=int, default=2,
                    help="workers per CU of the variant reported beside the one-per-CU headline (0/1 = skip)")
    ap.add_argument("--threads", type=int, default=None,
                    help="host feeder threads (one producer per mailbox; default: every host CPU but two, "
                         "at most 14)")
    ap.add_argument("--poll-sleep", type=int, default=0)
    ap.add_argument("--baseline-steps", type=int, default=1, help="steps timed for each baseline")
    ap.add_argument("--streams", type=int, default=4, help="HIP streams of the per-launch baseline")
    ap.add_argument("--skip-baselines", action="store_true")
    ap.add_argument("--no-graph-relaunch", action="store_true",
                    help="leave out the baselines that relaunch one single-node hipGraph per item (lanes and "
                         "plain forms); the per-launch and captured-chain baselines still run")
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--skip-floors", action="store_true",
                    help="leave out the latency floors (host<->device echo, the item alone) and the one-CU "
                         "workload: for counter-collection runs, where a kernel that waits on the host must not run")
    ap.add_argument("--skip-legs", action="store_true",
                    help="default workload: leave out the shortened isolation, serving, batching and replay runs")
    ap.add_argument("--leg-periods", type=int, default=5000, help="isolation periods per variant in the default run")
    ap.add_argument("--leg-serve-seconds", type=float, default=2.0,
                    help="serving trace length per rate in the default run")
    ap.add_argument("--leg-runs", type=int, default=100, help="replay runs per configuration in the default run")
    ap.add_argument("--cpu-items", type=int, default=10000,
                    help="items per mailbox in the CPU sample (capped at the workload's own)")
    ap.add_argument("--copy-probe-mib", type=int, default=1024)
    ap.add_argument("--workload", choices=["allcu", "isolation", "replay", "batching", "serving"], default="allcu",
                    help="allcu: the headline all-CU workload; isolation: cluster 0 critical "
                         "item every period beside streaming copies on the other XCDs; replay: the "
                         "paper's phase protocol with its compute-only item")
    ap.add_argument("--runs", type=int, default=100, help="replay: runs per configuration")
    ap.add_argument("--rates", type=str, default="10000,100000,1000000", help="serving: arrival rates (req/s)")
    ap.add_argument("--serve-seconds", type=float, default=3.0, help="serving: trace length per rate")
    ap.add_argument("--budget-gib", type=float, default=64.0, help="serving: device-memory budget for outputs")
    ap.add_argument("--tile", type=int, default=65536, help="serving: elements per tile")
    ap.add_argument("--serve-threads", type=int, default=1024, help="serving: threads per worker")
    ap.add_argument("--serve-schedulers", type=int, default=4,
                    help="serving: host scheduler threads (each owns an equal share of the workers)")
    ap.add_argument("--bursts", type=str, default="1,4,16,64,256,1024,4096", help="batching: burst sizes")
    ap.add_argument("--burst-reps", type=int, default=5, help="batching: timed repetitions per burst")
    ap.add_argument("--batch-threads", type=str, default="256,1024",
                    help="batching: worker sizes (threads per worker) the autotuner chooses from")
    ap.add_argument("--batch-spans", type=str, default="all,half,xcd",
                    help="batching: spans the autotuner chooses from (all: every CU, half: four XCDs' workers, "
                         "xcd: one XCD's workers)")
    ap.add_argument("--spin-iters", type=int, default=20000, help="replay: loop iterations of the item")
    ap.add_argument("--periods", type=int, default=10000, help="isolation: periods per variant")
    ap.add_argument("--period-us", type=float, default=1000.0)
    ap.add_argument("--copy-mib", type=int, default=256, help="isolation: interference buffer size")
    ap.add_argument("--iso-threads", type=int, default=256, help="isolation: threads per worker")
    args = ap.parse_args()
    if args.threads is None:
        from paper_2310_01212_amd import workloads
        args.threads = workloads.feeder_threads()
    return args


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}): "
              "the dispatch path has no multi-GPU component (each GPU would run a context of its own).",
              file=sys.stderr)
        sys.exit(2)
    run = {"isolation": bench_isolation, "replay": bench_replay, "batching": bench_batching,
           "serving": bench_serving, "allcu": bench_allcu}[args.workload]
    print(json.dumps(run(args)), flush=True)


# Host clock cycles per phase printed in the paper (Sec. 3): Table 2 averages (single SM,
# full GPU) and Table 3 worst case (single SM), NVIDIA GTX 980 + Intel i7 at 3.6 GHz.
# Context only, never a target.
PAPER_CYCLES = {
    ("avg", "single", "LK"): {"Init": 509e6, "Trigger": 239, "Wait": 190e3, "Dispose": 30e6},
    ("avg", "single", "CUDA"): {"Alloc": 496e6, "Spawn": 3.9e3, "Wait": 175e3, "Dispose": 274e3},
    ("avg", "full", "LK"): {"Init": 503e6, "Trigger": 210, "Wait": 190e3, "Dispose": 30e6},
    ("avg", "full", "CUDA"): {"Alloc": 497e6, "Spawn": 3.8e3, "Wait": 176e3, "Dispose": 247e3},
    ("worst", "single", "LK"): {"Init": 521e6, "Trigger": 1.1e3, "Wait": 203e3, "Dispose": 33e6},
    ("worst", "single", "CUDA"): {"Alloc": 501e6, "Spawn": 7.7e3, "Wait": 176e3, "Dispose": 893e3},
}


def bench_batching(args):
    """Bursts of uneven items (int32 affine / fp32 SAXPY 50/50, log-uniform 256 .. 2^20
    elements) as one persistent batch, with the tile size, the polling interval, the worker
    size and the span (every CU, four XCDs' or one XCD's workers) picked per burst size by the
    autotuner on training bursts (seed 50), against the same bursts as per-item launches
    and as a captured hipGraph."""
    import torch
    from paper_2310_01212_amd import autotune, lk, workloads

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    lk.lib()
    dev = torch.device("cuda:0")
    sizes = [int(v) for v in args.bursts.split(",")]
    reps = args.burst_reps

    def burst(count, seed):
        ops, n, ab, alpha = workloads.batching(count, seed=seed)
        off = np.concatenate([[0], np.cumsum((n + 255) // 256 * 256)]).astype(np.uint64)
        return ops, n, ab, alpha, off

    plans = {(c, s): burst(c, s) for c in sizes for s in (50, 5)}
    total = int(max(p[4][-1] for p in plans.values()))
    log(f"batching: arenas of {total} elements x 4 buffers")
    xi, xf = workloads.device_arena(total, seed=5, device=dev)
    yf = torch.randn(total, device=dev, dtype=torch.float32)
    z = torch.empty(total, device=dev, dtype=torch.int32)
    torch.cuda.synchronize()

    def items_of(p):
        ops, n, ab, alpha, off = p
        ins = np.where(ops == lk.OP_AFFINE_SUM_I32, xi.data_ptr(), xf.data_ptr()).astype(np.uint64) + off[:-1] * 4
        outs = np.where(ops == lk.OP_AFFINE_SUM_I32, z.data_ptr(), yf.data_ptr()).astype(np.uint64) + off[:-1] * 4
        return lk.make_items(ops, n, ins, outs, ab[:, 0], ab[:, 1], alpha)

    def item_bytes(p):
        ops, n = p[0], p[1].astype(np.float64)
        return float(np.sum(np.where(ops == lk.OP_AFFINE_SUM_I32, 8 * n + 8, 12 * n)))

    staged = {}

    def staged_tiles(key, tile):
        if (key, tile) not in staged:
            tiles, _ = lk.batch_plan(items_of(plans[key]), tile)
            d = torch.from_numpy(tiles.view(np.uint8)).to(dev)
            part = torch.zeros(tiles.size, dtype=torch.int64, device=dev)
            torch.cuda.synchronize()
            staged[(key, tile)] = (d, tiles.size, part)
        return staged[(key, tile)]

    ctxs = {}

    n_cu = torch.cuda.get_device_properties(0).multi_processor_count

    def ctx_for(cs):
        # one context at a time: each holds every CU until it is closed.  A burst runs on
        # cluster 0: every worker ("all"), the first half of the physically ordered workers
        # ("half": XCDs 0-3) or XCD 0's workers ("xcd")
        if cs not in ctxs:
            for old in list(ctxs):
                ctxs.pop(old).close()
            sleep, threads, span = cs
            kw = dict(poll_sleep=sleep, threads=threads, idle_timeout_ms=120000)
            if span == "all":
                kw.update(n_workers=0, clusters=lk.CLUSTERS_ONE)
            elif span == "half":
                kw.update(n_workers=n_cu, clusters=lk.CLUSTERS_EXPLICIT,
                          cluster_of_worker=(np.arange(n_cu) >= n_cu // 2).astype(np.uint32))
            else:
                kw.update(n_workers=0, clusters=lk.CLUSTERS_PER_XCD)
            ctxs[cs] = lk.Context(**kw)
        return ctxs[cs]

    def run_burst(size, tile, cs, r):
        d, nt, part = staged_tiles((size, 50), tile)
        ctx = ctx_for(cs)
        ctx.run_batch(0, d, nt, part, reps=1)  # warm-up
        return ctx.run_batch(0, d, nt, part, reps=r)

    log("batching: autotuning on training bursts (seed 50)")
    worker_sizes = tuple(int(v) for v in args.batch_threads.split(","))
    spans = tuple(args.batch_spans.split(","))
    if not spans or not set(spans) <= set(autotune.SPAN_CANDIDATES):
        sys.exit(f"--batch-spans: give spans from {autotune.SPAN_CANDIDATES}, not {args.batch_spans!r}")
    table = autotune.tune(run_burst, sizes, ctx_settings=autotune.contexts(threads=worker_sizes, spans=spans),
                          reps=reps)
    out = {"metric": "burst makespan (µs), items/s and achieved GB/s: one persistent batch vs per-item "
                     "launches vs captured hipGraph",
           "unit": "items/s", "higher_is_better": True, "n_gpus": 1, "dtype": "int32 / f32",
           "data": "synthetic (seeded: bursts seed 5, tuning seed 50)", "steps": reps, "warmup": 1,
           "scaling": "weak", "vs_baseline": None,
           "config": {"workload": "bursts of uneven items, log-uniform 256..2^20 elements, int32 affine and "
                                  "fp32 SAXPY 50/50, one persistent batch per burst", "bursts": sizes,
                      "worker_sizes_tuned": list(worker_sizes), "spans_tuned": list(spans)},
           "tuning": {str(k): {"tile": v["tile"], "poll_sleep": v["poll_sleep"], "threads": v["threads"],
                               "span": v["span"]} for k, v in table.items()},
           "bursts": {}}
    # The persistent bursts first, then every context closed, then the per-launch and graph
    # baselines on a GPU with no persistent workers resident (workers of 1024 threads fill
    # their CUs' register files, and a launched item could not be scheduled beside them).
    ms_of = {}
    for size in sizes:
        tune_row = table[size]
        d, nt, part = staged_tiles((size, 5), tune_row["tile"])
        ctx = ctx_for((tune_row["poll_sleep"], tune_row["threads"], tune_row["span"]))
        ctx.run_batch(0, d, nt, part, reps=1)
        ms_of[size] = (ctx.run_batch(0, d, nt, part, reps=reps), nt)
    for old in list(ctxs):
        ctxs.pop(old).close()
    for size in sizes:
        key = (size, 5)
        ms_p, nt = ms_of[size]
        items = items_of(plans[key])
        lk.launch_burst(items, graph=False, reps=1)
        ms_l = lk.launch_burst(items, graph=False, reps=reps)
        ms_g = lk.launch_burst(items, graph=True, reps=reps)
        b = item_bytes(plans[key])
        row = {}
        for name, ms in (("persistent", ms_p), ("launch", ms_l), ("graph", ms_g)):
            med = float(np.median(ms))
            row[name] = {"makespan_us": round(med, 2), "items_per_s": round(size / (med * 1e-6), 1),
                         "gbps": round(b / (med * 1e-6) / 1e9, 1)}
        row["tiles"] = int(nt)
        row["bytes"] = int(b)
        out["bursts"][str(size)] = row
        log(f"burst {size}: persistent {row['persistent']['makespan_us']} us, launch {row['launch']['makespan_us']} us, "
            f"graph {row['graph']['makespan_us']} us")
    big = out["bursts"][str(max(sizes))]
    out["value"] = big["persistent"]["items_per_s"]
    out["ms_per_step"] = round(big["persistent"]["makespan_us"] / 1e3, 4)
    out["roofline"] = {"bound": "hbm", "achieved": big["persistent"]["gbps"], "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                       "frac": round(big["persistent"]["gbps"] / HBM_PEAK_GBPS, 4), "traffic": None,
                       "kernel": "lk_worker (one batch)"}
    return out


def bench_serving(args):
    """Serving with continuous batching: Poisson arrivals of mixed requests (40% int32
    affine + sum, 30% int64 sum, 30% fp32 SAXPY written out of place), log-uniform
    256 .. 2^22 elements, inputs resident in device pools, outputs admitted against a
    device-memory budget; latency is arrival to completion observed."""
    import torch
    from paper_2310_01212_amd import lk, workloads

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    lk.lib()
    dev = torch.device("cuda:0")
    rates = [float(v) for v in args.rates.split(",")]
    pool_elems = 1 << 26
    log(f"serving: pools of {pool_elems} elements, budget {args.budget_gib} GiB")
    xi, xf = workloads.device_arena(pool_elems, seed=7, device=dev)
    yf = workloads.device_arena(pool_elems, seed=8, device=dev)[1]
    budget = int(args.budget_gib * (1 << 30)) // 256 * 256
    arena = torch.empty(budget // 4, dtype=torch.int32, device=dev)
    torch.cuda.synchronize()
    xi_host = xi.cpu().numpy()
    out = {"metric": "request latency p50/p99/p99.9/max (µs) and items/s under Poisson arrivals",
           "unit": "items/s", "higher_is_better": True, "n_gpus": 1, "dtype": "int32/int64/f32",
           "data": "synthetic (seeded, seed 7)", "steps": len(rates), "warmup": 0, "scaling": "weak",
           "vs_baseline": None,
           "config": {"workload": "serving with continuous batching: mixed requests (40% affine+sum, 30% sum, 30% "
                                  "SAXPY), log-uniform 256..2^22 elements, Poisson arrivals, outputs admitted against "
                                  f"a {args.budget_gib} GiB device-memory budget", "seconds_per_rate": args.serve_seconds,
                      "tile_elems": args.tile, "host_threads": args.serve_schedulers,
                      "threads_per_worker": args.serve_threads},
           "rates": {}}
    with lk.Context(n_workers=0, depth=4, threads=args.serve_threads, idle_timeout_ms=600000) as ctx:
        for rate in rates:
            tr = workloads.serving(rate, args.serve_seconds, pool_elems, seed=7)
            kind = tr["kind"]
            req = np.zeros(kind.size, lk.REQUEST_DTYPE)
            req["arrival_us"] = tr["arrival_us"]
            req["op"] = np.choose(kind, [lk.OP_AFFINE_SUM_I32, lk.OP_SUM_I32_I64, lk.OP_AXPY_F32])
            req["a"], req["b"], req["alpha"], req["n"] = tr["ab"][:, 0], tr["ab"][:, 1], tr["alpha"], tr["n"]
            req["inp"] = np.where(kind == 2, xf.data_ptr(), xi.data_ptr()).astype(np.uint64) + tr["off_x"] * 4
            req["in2"] = np.where(kind == 2, yf.data_ptr() + tr["off_y"].astype(np.int64) * 4, 0).astype(np.uint64)
            log(f"serving: {rate:.0f} req/s, {kind.size} requests")
            outc, st = ctx.serve(req, arena, budget, tile_elems=args.tile, threads=args.serve_schedulers,
                                 timeout=30.0)
            lat = outc["done_us"] - tr["arrival_us"]
            n = tr["n"].astype(np.float64)
            nbytes = float(np.sum(np.where(kind == 0, 8 * n + 8, np.where(kind == 1, 4 * n + 8, 12 * n))))
            row = {"requests": int(kind.size), "latency_us": lat_summary(lat),
                   "queue_us": lat_summary(outc["admit_us"] - tr["arrival_us"]),
                   "items_per_s": round(kind.size / st["elapsed_s"], 1),
                   "achieved_gbps": round(nbytes / st["elapsed_s"] / 1e9, 1),
                   "offered_gbps": round(nbytes / (tr["arrival_us"][-1] * 1e-6) / 1e9, 1),
                   "tiles": int(st["tiles"]), "deferred": int(st["deferred"]),
                   "peak_output_bytes": int(st["peak_bytes"])}
            # where the tail sits in time: p99 per 100 ms window of arrivals
            win = (tr["arrival_us"] // 1e5).astype(np.int64)
            order = np.argsort(win, kind="stable")
            bounds = np.flatnonzero(np.diff(win[order])) + 1
            w99 = [(int(win[order][g[0]]), pct(lat[g], 0.99), g.size) for g in np.split(order, bounds)]
            worst = max(w99, key=lambda t: t[1])
            row["windows_100ms"] = {"count": len(w99), "p99_over_1ms": int(sum(t[1] > 1000 for t in w99)),
                                    "worst": {"start_s": worst[0] / 10, "p99_us": round(worst[1], 3),
                                              "requests": int(worst[2])}}
            # sanity check of sampled int64 results
            sample = np.flatnonzero(kind != 2)[:: max(1, int(np.sum(kind != 2)) // 40)][:40]
            bad = 0
            for i in sample:
                ox, nn = int(tr["off_x"][i]), int(tr["n"][i])
                xs = xi_host[ox:ox + nn]
                want = (int_sum_check(xs, int(tr["ab"][i, 0]), int(tr["ab"][i, 1])) if kind[i] == 0
                        else int_sum_check(xs))
                bad += int(outc["result"][i] != want)
            row["sampled_result_mismatches"] = bad
            out["rates"][str(int(rate))] = row
            log(f"  p50 {row['latency_us']['p50']} us p99 {row['latency_us']['p99']} us, "
                f"{row['items_per_s']:,.0f} items/s, {row['achieved_gbps']} GB/s")
    top = out["rates"][str(int(max(rates)))]
    out["value"] = top["items_per_s"]
    out["ms_per_step"] = None
    return out


def bench_replay(args):
    """The paper's evaluation protocol on one MI355X: per run, Init/Trigger/Wait/Dispose of
    the persistent path and Alloc/Spawn/Wait/Dispose of one ordinary launch, with the
    paper's compute-only loop item, on one CU and on every CU."""
    import torch
    from paper_2310_01212_amd import lk

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    lk.lib()
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    out = {"metric": "host time per phase, avg and worst over runs (µs and host TSC cycles)",
           "unit": "us", "higher_is_better": False, "n_gpus": 1, "dtype": "int32 (compute-only loop)",
           "data": "synthetic", "steps": args.runs, "warmup": 0, "scaling": "weak", "vs_baseline": None,
           "config": {"workload": f"paper protocol: SPIN item of {args.spin_iters} iterations per thread, "
                                  f"{args.runs} runs, single CU and all {cus} CUs"}}
    for scope, nw in (("single_cu", 1), ("full_gpu", cus)):
        log(f"replay: {scope} ({nw} workers), {args.runs} runs")
        lk_us, hip_us, lk_cy, hip_cy = lk.replay(nw, args.spin_iters, args.runs)
        res = {}
        for sys_name, us, cy, phases in (("LK", lk_us, lk_cy, lk.REPLAY_PHASES_LK),
                                         ("HIP", hip_us, hip_cy, lk.REPLAY_PHASES_HIP)):
            res[sys_name] = {ph: {"avg_us": round(float(us[:, i].mean()), 3), "worst_us": round(float(us[:, i].max()), 3),
                                  "avg_cycles": int(cy[:, i].astype(np.float64).mean()),
                                  "worst_cycles": int(cy[:, i].max())}
                             for i, ph in enumerate(phases)}
        out[scope] = res
    out["paper_cycles_gtx980_i7_3.6GHz"] = {f"{a}/{b}/{c}": v for (a, b, c), v in PAPER_CYCLES.items()}
    out["value"] = out["single_cu"]["LK"]["Trigger"]["avg_us"] + out["single_cu"]["LK"]["Wait"]["avg_us"]
    out["ms_per_step"] = None
    return out


def bench_isolation(args):
    """Cluster isolation: 8 clusters = 8 XCDs; cluster 0 gets a critical int32 affine +
    int64 sum item over 262,144 elements every period, released by a host busy-wait, while
    clusters 1-7 copy private fp32 buffers back-to-back (interference on), idle-poll
    (interference off) or do not exist (absent: a context whose workers are all on XCD 0).
    on_pinned: interference on, the critical item's x (the same every period) kept in its
    cluster's LDS, so the item reads nothing from memory and only writes y."""
    import torch
    from paper_2310_01212_amd import lk, workloads

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    lk.lib()
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
    crit_pinned = lk.make_items(lk.OP_AFFINE_SUM_I32, xh.size, x.data_ptr(), y.data_ptr(), AB[:, 0], AB[:, 1],
                                flags=lk.DF_PIN_INPUT)
    bg = lk.make_items(lk.OP_COPY_F32, elems, [s.data_ptr() for s in srcs], [d.data_ptr() for d in dsts])
    out = {"metric": "critical-item latency p50/p99/p99.9/max (µs) under cross-XCD interference",
           "unit": "us", "higher_is_better": False, "n_gpus": 1, "dtype": "int32/int64 (critical), f32 copy",
           "data": "synthetic (seeded)", "steps": P, "warmup": 0, "scaling": "weak", "vs_baseline": None,
           "config": {"workload": "cluster isolation: 8 clusters = 8 XCDs; cluster 0 critical affine+sum over "
                                  f"{xh.size} int32 every {args.period_us} us; clusters 1-7 copy private "
                                  f"{args.copy_mib} MiB fp32 buffers back-to-back", "periods": P,
                      "threads_per_worker": args.iso_threads}}
    with lk.Context(n_workers=0, clusters=lk.CLUSTERS_PER_XCD, threads=args.iso_threads,
                    idle_timeout_ms=600000) as ctx:
        ncl = ctx.info()["n_clusters"]
        assert ncl == 8, f"expected 8 XCD clusters, got {ncl}"
        ctx.run_isolation(0, crit[:200], args.period_us * 1e-6, [], bg[:0])  # warm-up, untimed
        wall = float(ctx.info()["wall_clock_hz"])
        # one XCD's copy ceiling: the same 256 MiB copy on cluster 1 with every other
        # cluster idle, timed on the device wall clock (first pickup to last completion)
        spans = []
        for rep in range(6):
            t = ctx.submit(1, lk.OP_COPY_F32, x=int(bg["inp"][0]), y=int(bg["out"][0]), n=elems)
            ci = ctx.wait_info(1, t, timeout=30.0)
            if rep:
                spans.append((ci["t_done_max"] - ci["t_pick_min"]) / wall)
        xcd_gbps = 2 * elems * 4 / float(np.median(spans)) / 1e9
        out["xcd_copy_gbps"] = round(xcd_gbps, 1)
        log(f"isolation: one XCD copies at {xcd_gbps:,.0f} GB/s")

        def summarize(r, bgc, pinned=False):
            span = (r["info"]["t_done_max"] - r["info"]["t_pick_min"]) / wall * 1e6
            v = {"latency_us": lat_summary(r["lat_us"]), "device_span_us": lat_summary(span),
                 "release_lateness_us": lat_summary(r["late_us"]),
                 "submit_to_done_us": lat_summary(r["lat_us"] - r["late_us"]), "elapsed_s": round(r["elapsed_s"], 3)}
            # the critical item's own memory bandwidth (8n + 8 bytes, 4n + 8 with x pinned,
            # over its device span) against one XCD's copy ceiling
            crit_bytes = (4 if pinned else 8) * xh.size + 8
            crit_gbps = crit_bytes / (float(np.median(span)) * 1e-6) / 1e9
            v["critical_gbps_p50"] = round(crit_gbps, 1)
            v["critical_frac_of_xcd_copy"] = round(crit_gbps / xcd_gbps, 3)
            if bgc:
                copied = float(r["bg_done"].sum()) * 2 * (elems * 4)
                v["interference_copy_gbps"] = round(copied / r["elapsed_s"] / 1e9, 1)
                v["interference_items"] = int(r["bg_done"].sum())
            # sanity check of the sums of 20 sampled periods
            idx = np.linspace(0, P - 1, 20).astype(int)
            v["sampled_sum_mismatches"] = sum(int(r["results"][k] != int_sum_check(xh, int(AB[k, 0]), int(AB[k, 1])))
                                              for k in idx)
            return v

        for name, bgc, items in (("off", [], crit), ("on", list(range(1, 8)), crit),
                                 ("on_pinned", list(range(1, 8)), crit_pinned)):
            log(f"isolation: interference {name}")
            r = ctx.run_isolation(0, items, args.period_us * 1e-6, bgc, bg[:len(bgc)])
            out[name] = summarize(r, bgc, pinned=items is crit_pinned)
    # absent: only XCD 0's workers exist (the context's XCD mask), nothing else runs
    log("isolation: other clusters absent")
    with lk.Context(n_workers=0, xcd_mask=0x1, clusters=lk.CLUSTERS_PER_XCD, threads=args.iso_threads,
                    idle_timeout_ms=600000) as ca:
        assert ca.info()["n_clusters"] == 1
        ca.run_isolation(0, crit[:200], args.period_us * 1e-6, [], bg[:0])  # warm-up, untimed
        out["absent"] = summarize(ca.run_isolation(0, crit, args.period_us * 1e-6, [], bg[:0]), [])
    out["value"] = out["on"]["latency_us"]["max"]
    out["ms_per_step"] = round(out["on"]["elapsed_s"] * 1e3 / P, 4)
    return out


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
    cold_pairs = args.cold if args.cold > 1 else 0
    if cold_pairs:
        if args.pin_input:
            sys.exit("--cold and --pin-input select different workloads; give one of them")
        g = torch.Generator(device=dev)
        g.manual_seed(2)
        cx = torch.randn((lanes, cold_pairs, n), generator=g, device=dev, dtype=torch.float32)
        cy = torch.randn((lanes, cold_pairs, n), generator=g, device=dev, dtype=torch.float32)
        torch.cuda.synchronize()

    def operands(s):
        if not cold_pairs:
            return x_addr, y_addr
        pair = ((s * per + np.arange(per)) % cold_pairs).astype(np.uint64)[None, :]
        off = (li * cold_pairs + pair) * n * 4
        return cx.data_ptr() + off, cy.data_ptr() + off

    # every step's descriptors are built before any timed region
    steps_items = [lk.make_items(lk.OP_SAXPY_F32, n, *operands(s), alpha=A[:, s * per:(s + 1) * per],
                                 flags=lk.DF_PIN_INPUT if args.pin_input else 0)
                   for s in range(args.warmup + args.steps)]

    def step_items(s):
        return steps_items[s]

    bytes_per_item = 12 * n  # SAXPY: 8n read + 4n write
    # with x pinned, memory carries y alone (4n read + 4n written); x is read once per worker
    hbm_bytes_per_item = 8 * n if args.pin_input else bytes_per_item

    # The timed steps run as one stream per mailbox: each lane's items of steps
    # warmup .. warmup + steps - 1 in order, back-to-back, in one call of the native runner
    # (its host threads start once, and no mailbox waits at a step boundary for the
    # slowest one).  The list and the runner's output arrays are prepared before the
    # context boots, so the persistent dispatch holds nothing but the warm-up and timed work.
    timed_items = np.concatenate([step_items(s) for s in range(args.warmup, args.warmup + args.steps)], axis=1)
    timed_out = lk.lanes_outputs(lanes, timed_items.shape[1], with_info=True)
    warm_items = (np.concatenate([step_items(s) for s in range(args.warmup)], axis=1) if args.warmup else None)
    warm_out = lk.lanes_outputs(lanes, warm_items.shape[1]) if args.warmup else None

    # ---------------- persistent path
    log("persistent path: boot")
    ctx = lk.Context(n_workers=lanes, depth=args.depth, threads=args.threads_per_worker,
                     poll_sleep=args.poll_sleep, idle_timeout_ms=60000)
    info0 = ctx.info()
    if args.warmup:
        ctx.run_lanes(np.arange(lanes), warm_items, in_flight=args.depth, threads=args.threads, out=warm_out)
    log("persistent path: timed steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, lat_all, runner_s, comp_all = ctx.run_lanes(np.arange(lanes), timed_items, in_flight=args.depth,
                                                   threads=args.threads, with_info=True, out=timed_out)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ctx.close()
    info = ctx.info()
    del timed_items, warm_items, warm_out
    lat_all = lat_all.ravel()
    comp_all = comp_all.ravel()
    timed_count = lanes * per * args.steps
    items_per_s = timed_count / elapsed
    # duration of the single worker dispatch, measured by the kernel itself on the device
    # wall clock (first worker boot to last worker exit); the packet processor's dispatch
    # timestamps are reported beside it (a tool intercepting the queue can hide them)
    kernel_ms, kernel_clock = info["device_span_ms"], "device wall clock, first boot to last exit"
    if kernel_ms <= 0:
        kernel_ms, kernel_clock = info["kernel_ms"], "dispatch timestamps"
    session_items = lanes * per * (args.warmup + args.steps)
    achieved_gbps = gb_per_s(session_items * hbm_bytes_per_item, kernel_ms)
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
        "config": {"workload": "all-CU SAXPY: one worker per CU, each mailbox fed items back-to-back" +
                               (", x pinned in each worker's LDS" if args.pin_input else "") +
                               (f", each mailbox rotating through {cold_pairs} (x, y) pairs" if cold_pairs else ""),
                   "workers": lanes, "items_per_mailbox": per * args.steps, "n": n,
                   "item_bytes": bytes_per_item, "queue_depth": args.depth, "pin_input": args.pin_input,
                   "cold_pairs": cold_pairs,
                   "host_threads": args.threads, "threads_per_worker": args.threads_per_worker,
                   "poll_sleep": args.poll_sleep},
        "latency_us": lat_summary(lat_all),
        # the native runner's own time (first submit to last completion) per step; the rest
        # of ms_per_step is starting and joining its host threads
        "runner_ms_per_step": round(runner_s * 1e3 / args.steps, 3),
        "init_ms": round(info0["init_ms"], 3),
        "dispose_ms": round(info["dispose_ms"], 3),
    }

    # ---------------- byte rate of the worker kernel (one launch = the session).  For the
    # hot workload this is not the binding bound: x and y of every mailbox stay in its XCD's
    # L2 and the Infinity Cache, and the item rate is bound by dispatch latency (below).
    # The cold form (--cold P) streams every operand from HBM and is bound by it.
    byte_rate = {"achieved": round(achieved_gbps, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                 "frac": round(achieved_gbps / HBM_PEAK_GBPS, 4), "traffic": None,
                 "kernel": "lk_worker", "kernel_ms": round(kernel_ms, 3), "kernel_clock": kernel_clock,
                 "dispatch_timestamps_ms": round(info["kernel_ms"], 3),
                 "items_per_launch": session_items, "algorithmic_bytes_per_item": hbm_bytes_per_item,
                 "algorithmic_bytes": session_items * hbm_bytes_per_item}
    tr = traffic_per_item(n, args.threads_per_worker, args.pin_input, args.depth, cold_pairs)
    if tr is not None:
        byte_rate["traffic"] = round(tr["bytes_per_item"] * session_items)
        byte_rate["traffic_source"] = tr["source"]

    # ---------------- streaming-copy probe (HBM roofline reference, known-size kernel): the
    # fastest form measured on this machine (one workgroup of 256 threads per CU, four
    # 16-byte vectors in flight per thread, non-temporal loads and stores), and beside it
    # the persistent worker's own shape and store policy (1024 threads per CU, stores
    # written through the L2)
    nbytes = args.copy_probe_mib << 20
    src = torch.empty(nbytes // 4, dtype=torch.int32, device=dev)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    ms, gbps = lk.copy_bandwidth(src, dst, nbytes, grid=lanes, reps=5, threads=256, unroll=4,
                                 policy=lk.COPY_NONTEMPORAL)
    wms, wgbps = lk.copy_bandwidth(src, dst, nbytes, grid=lanes, reps=5, threads=1024, unroll=4,
                                   policy=lk.COPY_SYSTEM)
    result["copy_probe"] = {"bytes": nbytes, "ms": round(ms, 4), "gbps": round(gbps, 1),
                            "frac_of_peak": round(gbps / HBM_PEAK_GBPS, 4),
                            "form": f"{lanes} workgroups x 256 threads, 4 vectors in flight, non-temporal",
                            "worker_shape_written_through": {
                                "ms": round(wms, 4), "gbps": round(wgbps, 1),
                                "form": f"{lanes} workgroups x 1024 threads, 4 vectors in flight, stores sc0 sc1"}}
    del src, dst

    def session(items_steps, depth=1, **ctx_kw):
        """One context over a list of per-step item arrays: the first step as an untimed
        warm-up, the others as one timed call of the native runner; the items and output
        arrays are prepared before the context boots, so its dispatch holds nothing but
        this work.  Returns (lat_us, runner_s, info after dispose)."""
        nm = items_steps[0].shape[0]
        warm, timed = items_steps[0], np.concatenate(items_steps[1:], axis=1)
        wout, tout = lk.lanes_outputs(nm, warm.shape[1]), lk.lanes_outputs(nm, timed.shape[1])
        kw = dict(n_workers=lanes, depth=depth, threads=args.threads_per_worker, poll_sleep=args.poll_sleep,
                  idle_timeout_ms=60000)
        kw.update(ctx_kw)
        with lk.Context(**kw) as cx:
            cx.run_lanes(np.arange(nm), warm, in_flight=depth, threads=args.threads, out=wout)
            _, lat, el = cx.run_lanes(np.arange(nm), timed, in_flight=depth, threads=args.threads, out=tout)
        return lat.ravel(), el, cx.info()

    # ---------------- baselines on the same workload
    if not args.skip_baselines:
        base = {}
        # launch: one hipLaunchKernelGGL per item; graph: a single-node graph relaunched per
        # item (its parameters updated); graph_chain: each lane's items captured once as a
        # chain of kernel nodes and launched as one graph (throughput only: the timed region
        # is the native runner's, excluding capture and instantiation)
        lane_forms = [("launch", 0), ("graph", lk.USE_GRAPH), ("graph_chain", lk.GRAPH_CHAIN)]
        if args.no_graph_relaunch:
            lane_forms = [f for f in lane_forms if f[1] != lk.USE_GRAPH]
        for name, mode in lane_forms:
            bl, el_native = [], 0.0
            t0 = time.perf_counter()
            for s in range(args.baseline_steps):
                _, lat, el = lk.launch_lanes(step_items(s), streams=args.streams, threads_host=args.threads,
                                             threads=args.threads_per_worker, mode=mode)
                bl.append(lat)
                el_native += el
            el = el_native if mode == lk.GRAPH_CHAIN else time.perf_counter() - t0
            bl = np.concatenate([b.ravel() for b in bl])
            base[name] = {"items_per_s": round(bl.size / el, 1),
                          "latency_us": None if mode == lk.GRAPH_CHAIN else lat_summary(bl),
                          "streams": args.streams, "threads_per_wg": args.threads_per_worker,
                          "items": int(bl.size)}
            log(f"{name}: {bl.size / el:,.0f} items/s" +
                ("" if mode == lk.GRAPH_CHAIN else f", p50 {pct(bl, .5):.2f} us"))
        result["baselines"] = base
        result["speedup_items_per_s"] = {k: round(items_per_s / v["items_per_s"], 2) for k, v in base.items()}

        # pipelined variant: the same mailboxes kept `depth` items ahead (latency then
        # includes the time an item waits behind the ones before it in its ring)
        if args.pipelined_depth > 1:
            d = args.pipelined_depth
            psteps = min(4, args.warmup + args.steps)
            pl, pt, pinf = session([step_items(s) for s in range(psteps)], depth=d)
            result["pipelined"] = {"queue_depth": d, "items_per_s": round(pl.size / pt, 1),
                                   "latency_us": lat_summary(pl), "items": int(pl.size)}
            # With the ring kept ahead the CUs never wait for the host, and the bound becomes
            # the memory side: y's reads and written-through stores miss the L2 on every
            # item (x stays in it), so the measured traffic of the committed counter summary
            # of this workload, over the dispatch, is set against the 8 TB/s peak and the
            # best streaming copy
            ptr = traffic_per_item(n, args.threads_per_worker, args.pin_input, d, cold_pairs)
            if ptr is not None and pinf["device_span_ms"] > 0:
                p_items = lanes * per * psteps
                p_traffic = round(ptr["bytes_per_item"] * p_items)
                result["pipelined"]["roofline"] = hbm_roofline(
                    p_traffic, pinf["device_span_ms"], result["copy_probe"]["gbps"], traffic=p_traffic,
                    traffic_source=ptr["source"], kernel="lk_worker", items_per_launch=p_items,
                    bytes="memory-side traffic measured by the counters (L2 misses to the Infinity Cache and "
                          "HBM), not algorithmic bytes")
            log(f"pipelined depth {d}: {pl.size / pt:,.0f} items/s")

        # several workers per CU: k mailboxes per CU, each fed back-to-back at depth 1, so
        # one worker's round trip to the host overlaps another's execution on the same CU
        if args.variant_per_cu > 1:
            k = args.variant_per_cu
            tv = min(args.threads_per_worker, 1024 // k)
            vl = lanes * k
            vsteps = min(4, args.warmup + args.steps)
            VX = np.empty((vl, n), np.float32)
            VY = np.empty((vl, n), np.float32)
            VA = np.empty((vl, vsteps * per), np.float32)
            for w in range(vl):
                VX[w], VY[w], VA[w] = workloads.allcu_lane(w, items=vsteps * per, n=n)
            vx, vy = torch.from_numpy(VX).to(dev), torch.from_numpy(VY).to(dev)
            torch.cuda.synchronize()
            vli = np.arange(vl, dtype=np.uint64)[:, None]
            vitems = [lk.make_items(lk.OP_SAXPY_F32, n, vx.data_ptr() + vli * n * 4, vy.data_ptr() + vli * n * 4,
                                    alpha=VA[:, s * per:(s + 1) * per]) for s in range(vsteps)]
            vlat, vt, _ = session(vitems, n_workers=0, workers_per_cu=k, threads=tv)
            del vx, vy
            result["workers_per_cu_variant"] = {"workers_per_cu": k, "threads_per_worker": tv, "mailboxes": vl,
                                                "queue_depth": 1, "items_per_s": round(vlat.size / vt, 1),
                                                "latency_us": lat_summary(vlat), "items": int(vlat.size)}
            log(f"{k} workers per CU: {vlat.size / vt:,.0f} items/s")

        # cold variant: every mailbox rotates through P (x, y) pairs (item k uses pair
        # k mod P), 512 MiB in aggregate at P = 16, more than the 256 MB Infinity Cache, so
        # the operands stream from HBM and algorithmic bytes are real traffic
        if args.cold_pairs > 1:
            P = args.cold_pairs
            g = torch.Generator(device=dev)
            g.manual_seed(2)
            cx = torch.randn((lanes, P, n), generator=g, device=dev, dtype=torch.float32)
            cy = torch.randn((lanes, P, n), generator=g, device=dev, dtype=torch.float32)
            torch.cuda.synchronize()
            csteps = min(4, args.warmup + args.steps)
            cit = []
            for s in range(csteps):
                pair = ((s * per + np.arange(per)) % P).astype(np.uint64)[None, :]
                off = (li * P + pair) * n * 4
                cit.append(lk.make_items(lk.OP_SAXPY_F32, n, cx.data_ptr() + off, cy.data_ptr() + off,
                                         alpha=A[:, s * per:(s + 1) * per]))
            cold = {}
            # depth 1 (the headline's form), then the ring kept args.pipelined_depth ahead:
            # with the look-ahead read the CUs stay busy and HBM becomes the bound
            for cd in sorted({1, max(1, args.pipelined_depth)}):
                clat, ct, cinfo = session(cit, depth=cd)
                c_items = lanes * per * csteps
                c_gbps = gb_per_s(c_items * bytes_per_item, cinfo["device_span_ms"])
                cold[cd] = {"queue_depth": cd, "items_per_s": round(clat.size / ct, 1), "latency_us": lat_summary(clat),
                            "kernel_ms": round(cinfo["device_span_ms"], 3), "items_per_launch": c_items,
                            "achieved_gbps": round(c_gbps, 1), "frac_of_peak": round(c_gbps / HBM_PEAK_GBPS, 4)}
                # measured memory bytes per item, from the committed counter summary of the
                # same workload (bench.py --cold P --depth d) when one matches
                ctr = traffic_per_item(n, args.threads_per_worker, False, cd, P)
                if ctr is not None:
                    cold[cd]["traffic_bytes_per_item"] = ctr["bytes_per_item"]
                    cold[cd]["traffic_source"] = ctr["source"]
                # every operand streams from HBM: the binding roofline is bandwidth, against
                # the 8 TB/s peak and, beside it, the best streaming copy measured here
                cold[cd]["roofline"] = hbm_roofline(
                    c_items * bytes_per_item, cinfo["device_span_ms"], result["copy_probe"]["gbps"],
                    traffic=round(ctr["bytes_per_item"] * c_items) if ctr else None, kernel="lk_worker")
                log(f"cold ({P} pairs per mailbox, depth {cd}): {clat.size / ct:,.0f} items/s, {c_gbps:,.0f} GB/s")
            del cx, cy
            result["cold_variant"] = {"pairs_per_mailbox": P, "footprint_bytes": lanes * P * n * 8, **cold[1]}
            if len(cold) > 1:
                result["cold_variant"]["pipelined"] = cold[max(cold)]

        # pinned-input variants: x kept in each worker's LDS across items (descriptor flag
        # DF_PIN_INPUT).  "hot" is the headline workload with the flag; "y_cold" keeps x per
        # mailbox and rotates y through P buffers (512 MiB at P = 32, past the Infinity Cache),
        # run without and with the flag.  Their byte rates are given both ways: algorithmic
        # (12n bytes per item) and HBM (8n: y read and written through; x stays in the XCD's
        # L2, or in LDS when pinned)
        if args.pinned and not args.pin_input:
            def timed(ctx_kw, items_of_step, nsteps, depth=1):
                return session([items_of_step(s) for s in range(nsteps)], depth=depth, **ctx_kw)

            psteps = min(4, args.warmup + args.steps)
            pin_items = []
            for s in range(psteps):
                it = step_items(s).copy()
                it["flags"] = lk.DF_PIN_INPUT
                pin_items.append(it)
            pl, pt, pinf = timed({}, lambda s: pin_items[s], psteps)
            pv = {"workload": "the headline workload with x pinned", "items_per_s": round(pl.size / pt, 1),
                  "latency_us": lat_summary(pl), "items": int(pl.size),
                  "pin_capacity_bytes": pinf["pin_capacity"]}
            log(f"pinned (hot): {pl.size / pt:,.0f} items/s")
            if args.pipelined_depth > 1:
                d = args.pipelined_depth
                ql, qt, _ = timed({}, lambda s: pin_items[s], psteps, depth=d)
                pv["pipelined"] = {"queue_depth": d, "items_per_s": round(ql.size / qt, 1),
                                   "latency_us": lat_summary(ql), "items": int(ql.size)}
                log(f"pinned (hot), depth {d}: {ql.size / qt:,.0f} items/s")
            P = 32
            g = torch.Generator(device=dev)
            g.manual_seed(3)
            ycold = torch.randn((lanes, P, n), generator=g, device=dev, dtype=torch.float32)
            torch.cuda.synchronize()
            ycit = {0: [], lk.DF_PIN_INPUT: []}
            for s in range(psteps):
                pair = ((s * per + np.arange(per)) % P).astype(np.uint64)[None, :]
                yo = ycold.data_ptr() + (li * P + pair) * n * 4
                for fl in ycit:
                    ycit[fl].append(lk.make_items(lk.OP_SAXPY_F32, n, x_addr, yo, alpha=A[:, s * per:(s + 1) * per],
                                                  flags=fl))
            for fl, key in ((0, "y_cold_unpinned"), (lk.DF_PIN_INPUT, "y_cold_pinned")):
                yl, yt, yinf = timed({}, lambda s, fl=fl: ycit[fl][s], psteps)
                y_items = lanes * per * psteps
                gbps = gb_per_s(y_items * bytes_per_item, yinf["device_span_ms"])
                hbm_gbps = gb_per_s(y_items * 8 * n, yinf["device_span_ms"])
                pv[key] = {"y_buffers_per_mailbox": P, "y_footprint_bytes": lanes * P * n * 4,
                           "items_per_s": round(yl.size / yt, 1), "latency_us": lat_summary(yl),
                           "kernel_ms": round(yinf["device_span_ms"], 3), "items_per_launch": y_items,
                           "algorithmic_bytes_per_item": bytes_per_item, "algorithmic_gbps": round(gbps, 1),
                           "hbm_bytes_per_item": 8 * n, "hbm_gbps": round(hbm_gbps, 1),
                           "hbm_frac_of_peak": round(hbm_gbps / HBM_PEAK_GBPS, 4)}
                log(f"{key}: {yl.size / yt:,.0f} items/s, {hbm_gbps:,.0f} GB/s of y from HBM")
            del ycold
            result["pinned_variant"] = pv

    if args.skip_floors:
        result["roofline"] = ({"bound": "hbm", **byte_rate} if cold_pairs else
                              {"bound": "latency", "achieved": round(items_per_s, 1), "peak": None, "unit": "items/s",
                               "frac": None, "traffic": byte_rate["traffic"], "kernel": "lk_worker",
                               "kernel_ms": byte_rate["kernel_ms"], "items_per_launch": session_items})
        if not cold_pairs:
            result["byte_rate"] = byte_rate
    else:
        # ---------------- dispatch latency floors (measured in every run)
        # the bare host<->device echo, one wave alone and with every CU's wave polling its own
        # word (the host pings them in turn)
        rtt = lk.pingpong(workers=1, iters=5000)[:, 500:]
        rtt_all = lk.pingpong(workers=lanes, iters=200)[:, 20:]
        # one headline item on one worker alone: device pickup to status record, from the log
        with lk.Context(n_workers=1, threads=args.threads_per_worker, log_capacity=512,
                        idle_timeout_ms=30000) as c1:
            c1.run_lanes(np.arange(1), step_items(0)[:1, :500], in_flight=1, threads=1)
        hz = float(c1.info()["wall_clock_hz"])
        e1 = c1.log(0)[100:]
        item_alone_us = float(np.median((e1["t_done"] - e1["t_pick"]) / hz * 1e6))
        echo_all_us = pct(rtt_all, 0.5)
        # At depth 1 every item of a mailbox costs at least one host round trip (status record
        # seen, next command posted and seen) plus the item itself; with the ring kept ahead the
        # round trip can hide behind the item, which then bounds alone.
        floor_all, bound = latency_bound(lanes, echo_all_us, item_alone_us, args.depth)
        result["latency_roofline_all_cus"] = {
            "floor": ("all-CU ping-pong RTT p50 + the headline item's device span on one worker alone"
                      if args.depth == 1 else "the headline item's device span on one worker alone"),
            "echo_us": round(echo_all_us, 3), "item_alone_us": round(item_alone_us, 3), "floor_us": round(floor_all, 3),
            "items_per_s_bound": round(bound, 1), "achieved_items_per_s": round(items_per_s, 1),
            "frac": round(items_per_s / bound, 3)}
        log(f"all-CU latency bound: {bound:,.0f} items/s (echo {echo_all_us:.3f} us + item {item_alone_us:.2f} us)")
        if cold_pairs:
            result["roofline"] = {"bound": "hbm", **byte_rate}
        else:
            result["roofline"] = {"bound": "latency", "achieved": round(items_per_s, 1), "peak": round(bound, 1),
                                  "unit": "items/s", "frac": round(items_per_s / bound, 4), "traffic": byte_rate["traffic"],
                                  "floor": result["latency_roofline_all_cus"]["floor"], "floor_us": round(floor_all, 3),
                                  "kernel": "lk_worker", "kernel_ms": byte_rate["kernel_ms"],
                                  "items_per_launch": session_items}
            result["byte_rate"] = byte_rate

        # where an item's time goes (host steady clock and device wall clock): Trigger is
        # inside the latency; the device span runs from the first member's pickup to the last
        # member's status record; the rest is the two host-link crossings and the polls
        span_all = (comp_all["t_done_max"] - comp_all["t_pick_min"]) / hz * 1e6
        result["latency_split_us"] = {"latency": lat_summary(lat_all), "device_span": lat_summary(span_all),
                                      "host_link_and_polls": lat_summary(lat_all - span_all),
                                      "echo_floor_p50": round(echo_all_us, 3)}

        # ---------------- the plain single-worker workload (1 CU, 1000 affine+sum items of 4096 int32)
        Xs, ABs = workloads.plain()
        xs = torch.from_numpy(Xs).to(dev)
        ys = torch.zeros_like(xs)
        torch.cuda.synchronize()
        rows = np.arange(Xs.shape[0], dtype=np.uint64)
        items = lk.make_items(lk.OP_AFFINE_SUM_I32, Xs.shape[1], xs.data_ptr() + rows * Xs.shape[1] * 4,
                              ys.data_ptr() + rows * Xs.shape[1] * 4, ABs[:, 0], ABs[:, 1])
        with lk.Context(n_workers=1, idle_timeout_ms=30000) as c1:
            c1.run_serial(0, items[:100])
            _, lat_p, trig_p, comp_p = c1.run_serial(0, items)
        span_p = (comp_p["t_done_max"] - comp_p["t_pick_min"]) / hz * 1e6
        serial = {"persistent": lat_summary(lat_p), "persistent_trigger": lat_summary(trig_p),
                  "persistent_device_span": lat_summary(span_p),
                  "persistent_host_link_and_polls": lat_summary(lat_p - trig_p - span_p)}
        if not args.skip_baselines:
            for name, mode in (("launch_sync", lk.COMPLETE_SYNC), ("launch_flag", lk.COMPLETE_FLAG),
                               ("graph_sync", lk.COMPLETE_SYNC | lk.USE_GRAPH),
                               ("graph_flag", lk.COMPLETE_FLAG | lk.USE_GRAPH)):
                if args.no_graph_relaunch and mode & lk.USE_GRAPH:
                    continue
                lk.launch_serial(items[:100], mode=mode)
                _, lat_b, lau_b = lk.launch_serial(items, mode=mode)
                serial[name] = lat_summary(lat_b)
                serial[name + "_launch_call"] = lat_summary(lau_b)
        serial["pingpong_rtt"] = lat_summary(rtt)
        serial["pingpong_rtt_all_cus"] = lat_summary(rtt_all)
        # one-CU streaming copy: the bandwidth one worker can reach on its own
        cb = 32 << 20
        csrc = torch.empty(cb // 4, dtype=torch.int32, device=dev)
        cdst = torch.empty_like(csrc)
        torch.cuda.synchronize()
        _, bw1 = lk.copy_bandwidth(csrc, cdst, cb, grid=1, reps=3)
        del csrc, cdst
        item_bytes = 8 * Xs.shape[1] + 8
        serial["copy_1cu_gbps"] = round(bw1, 2)
        result["serial_1cu"] = {"workload": "1 worker on 1 CU, 1000 submit-then-wait items: int32 affine "
                                            "+ int64 sum over 4096 elements", **serial}
        result["latency_roofline"] = {"floor": "host<->device coherent ping-pong RTT p50",
                                      "floor_us": serial["pingpong_rtt"]["p50"],
                                      "floor_us_all_cus_polling": serial["pingpong_rtt_all_cus"]["p50"],
                                      "dispatch_p50_us": serial["persistent"]["p50"],
                                      "frac": round(serial["pingpong_rtt"]["p50"] / serial["persistent"]["p50"], 3),
                                      "item_bytes": item_bytes,
                                      "bytes_frac_of_1cu_copy": round(
                                          item_bytes / (serial["persistent"]["p50"] * 1e-6) / 1e9 / bw1, 3)}
        log(f"serial: persistent p50 {serial['persistent']['p50']} us")

        # one dispatch at a time at the headline's item size: lane 0's SAXPY items of 16,384
        # on one worker of the headline's width, submit-then-wait, against one launch of
        # one workgroup of the same width per item (the all-CU baseline latencies above
        # include waiting behind the other lanes of a stream; these do not)
        sx = step_items(0)[0, :1000].copy()
        with lk.Context(n_workers=1, threads=args.threads_per_worker, idle_timeout_ms=30000) as c1:
            c1.run_serial(0, sx[:100])
            _, lat_s, trig_s, comp_s = c1.run_serial(0, sx)
        span_s = (comp_s["t_done_max"] - comp_s["t_pick_min"]) / hz * 1e6
        one = {"workload": f"1 worker of {args.threads_per_worker} threads on 1 CU, 1000 submit-then-wait SAXPY "
                           f"items of {n} fp32 (mailbox 0's items)",
               "persistent": lat_summary(lat_s), "persistent_trigger": lat_summary(trig_s),
               "persistent_device_span": lat_summary(span_s)}
        if not args.skip_baselines:
            for name, mode in (("launch_sync", lk.COMPLETE_SYNC), ("launch_flag", lk.COMPLETE_FLAG),
                               ("graph_sync", lk.COMPLETE_SYNC | lk.USE_GRAPH),
                               ("graph_flag", lk.COMPLETE_FLAG | lk.USE_GRAPH)):
                if args.no_graph_relaunch and mode & lk.USE_GRAPH:
                    continue
                lk.launch_serial(sx[:100], threads=args.threads_per_worker, mode=mode)
                _, lat_b, _ = lk.launch_serial(sx, threads=args.threads_per_worker, mode=mode)
                one[name] = lat_summary(lat_b)
        result["serial_1cu_headline_item"] = one
        log(f"one dispatch at a time, headline item: persistent p50 {one['persistent']['p50']} us")

    # ---------------- the other workloads, shortened: cluster isolation, serving, batching
    # and the paper's phase protocol (each also runs at full length with --workload)
    if not args.skip_legs:
        for name, fn, over in (("isolation", bench_isolation, {"periods": args.leg_periods}),
                               ("serving", bench_serving, {"serve_seconds": args.leg_serve_seconds}),
                               ("batching", bench_batching, {}),
                               ("replay", bench_replay, {"runs": args.leg_runs})):
            t0 = time.perf_counter()
            leg = fn(argparse.Namespace(**{**vars(args), **over}))
            for k in ("n_gpus", "scaling", "vs_baseline", "higher_is_better"):
                leg.pop(k, None)
            leg["wall_s"] = round(time.perf_counter() - t0, 2)
            result[name] = leg

    # ---------------- CPU oracle on a bounded sample of the same workload
    if not args.skip_cpu:
        import oracle
        oracle.build(force=False)
        host_cpus = len(os.sched_getaffinity(0))
        cores = min(16, host_cpus)
        per_cpu = min(args.cpu_items, A.shape[1])
        # The item lists are marshalled before the clock starts; the timed region is the
        # oracle's own FIFO executor, one mailbox after another on each thread.
        ys_cpu = [Y0[w].copy() for w in range(lanes)]
        packed = [oracle.pack_chain(oracle.SAXPY_F32, X[w], ys_cpu[w], A[w, :per_cpu]) for w in range(lanes)]

        def lane_job(w):
            oracle.run_packed(packed[w])

        t0 = time.perf_counter()
        with cf.ThreadPoolExecutor(max_workers=cores) as ex:
            list(ex.map(lane_job, range(lanes)))
        el = time.perf_counter() - t0
        # the plain workload on one host thread: each item executed as soon as it is
        # "submitted", one after another
        Xs, ABs = workloads.plain()
        lat_c = np.empty(Xs.shape[0])
        yc = np.empty(Xs.shape[1], np.int32)
        t1 = time.perf_counter()
        for i in range(Xs.shape[0]):
            ti = time.perf_counter()
            oracle.affine_sum_i32(Xs[i], int(ABs[i, 0]), int(ABs[i, 1]), y=yc)
            lat_c[i] = (time.perf_counter() - ti) * 1e6
        el1 = time.perf_counter() - t1
        result["cpu_baseline"] = {"value": round(lanes * per_cpu / el, 1), "unit": "items/s", "cores": cores,
                                  "kind": "oracle", "host_cpus": host_cpus, "cpu_model": host_cpu_model(),
                                  "sample": f"{lanes} mailboxes x {per_cpu} SAXPY items of {n} fp32 "
                                            f"({lanes * per_cpu} items), lanes spread over {cores} threads",
                                  "seconds": round(el, 3),
                                  "plain_single_thread": {
                                      "items_per_s": round(Xs.shape[0] / el1, 1), "cores": 1,
                                      "latency_us": lat_summary(lat_c),
                                      "sample": f"{Xs.shape[0]} affine+sum items of {Xs.shape[1]} int32, one "
                                                "after another on one host thread"}}
        log(f"cpu oracle: {lanes * per_cpu / el:,.0f} items/s on {cores} threads; plain workload "
            f"{Xs.shape[0] / el1:,.0f} items/s on 1 thread")

    return result


if __name__ == "__main__":
    main()
