"""Autotuner of the batched persistent dispatch: per burst size, the tile size (elements
per claimed tile) and the context the burst runs on -- the workers' polling interval,
their size (threads per workgroup) and how many CUs the burst spreads over (every CU,
half of them (four XCDs), or one XCD's) -- that minimise the median makespan.

Tuning runs on training bursts (their own seed) and the chosen table is then used on the
evaluation bursts.  Larger tiles cost fewer counter claims and less per-tile overhead;
smaller tiles balance uneven items better over the workers; the polling interval trades
PCIe read traffic of idle workers against pickup latency; larger workers keep more loads
in flight per CU (long bursts) but take longer over the reductions and barriers of short
tiles; fewer workers take a short burst with fewer command posts (one XCD's 32 workers
also keep the tile claims within one L2), while long bursts need every CU.
"""
import json
import os

import numpy as np

TILE_CANDIDATES = (4096, 16384, 65536, 262144)
SLEEP_CANDIDATES = (0, 8)
THREAD_CANDIDATES = (256, 1024)
SPAN_CANDIDATES = ("all", "half", "xcd")


def contexts(sleeps=SLEEP_CANDIDATES, threads=THREAD_CANDIDATES, spans=SPAN_CANDIDATES):
    """Every context setting (poll_sleep, threads, span) of the candidates."""
    return tuple((s, t, sp) for sp in spans for t in threads for s in sleeps)


def pick_best(timings):
    """timings: {(tile, (poll_sleep, threads, span)): [makespan_us, ...]} -> the key with
    the smallest median; ties go to the larger tile, then to the longer polling interval,
    then to the smaller worker (which leaves more of its CU to other kernels), then to the
    wider span."""
    best = None
    for (tile, (sleep, threads, span)), v in timings.items():
        key = (float(np.median(v)), -tile, -sleep, threads, SPAN_CANDIDATES.index(span))
        if best is None or key < best[0]:
            best = (key, (tile, (sleep, threads, span)))
    return best[1]


def tune(run_burst, sizes, tiles=TILE_CANDIDATES, ctx_settings=None, reps=5):
    """run_burst(size, tile, (poll_sleep, threads, span), reps) -> list of makespans (us) of a
    training burst.  A context setting belongs to a running context, so it is the outer
    loop (one context per setting).  Returns {size: {"tile", "poll_sleep", "threads",
    "span", "median_us", "grid"}}."""
    ctx_settings = contexts() if ctx_settings is None else tuple(ctx_settings)
    timings = {size: {} for size in sizes}
    for cs in ctx_settings:
        for size in sizes:
            for tile in tiles:
                timings[size][(tile, cs)] = list(run_burst(size, tile, cs, reps))
    table = {}
    for size in sizes:
        tile, (sleep, thr, span) = pick_best(timings[size])
        table[int(size)] = {"tile": int(tile), "poll_sleep": int(sleep), "threads": int(thr), "span": span,
                            "median_us": float(np.median(timings[size][(tile, (sleep, thr, span))])),
                            "grid": {f"{t}/{s}/{w}/{sp}": float(np.median(v))
                                     for (t, (s, w, sp)), v in timings[size].items()}}
    return table


def save(table, path, device_name):
    with open(path, "w") as f:
        json.dump({"device": device_name, "table": table}, f, indent=1, sort_keys=True)


def load(path, device_name):
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("device") != device_name:
        return None
    # tables written before the worker size and span were tuned: 256-thread workers on every CU
    return {int(k): {"threads": 256, "span": "all", **v} for k, v in d["table"].items()}
