"""Autotuner of the batched persistent dispatch: per burst size, the tile size (elements
per claimed tile), the workers' polling interval and the workers' size (threads per
workgroup) that minimise the median makespan.

Tuning runs on training bursts (their own seed) and the chosen table is then used on the
evaluation bursts.  Larger tiles cost fewer counter claims and less per-tile overhead;
smaller tiles balance uneven items better over the 256 workers; the polling interval
trades PCIe read traffic of idle workers against pickup latency; larger workers keep more
loads in flight per CU (long bursts) but take longer over the reductions and barriers of
short tiles.
"""
import json
import os

import numpy as np

TILE_CANDIDATES = (4096, 16384, 65536, 262144)
SLEEP_CANDIDATES = (0, 8)
THREAD_CANDIDATES = (256, 1024)


def pick_best(timings):
    """timings: {(tile, sleep, threads): [makespan_us, ...]} -> the key with the smallest
    median; ties go to the larger tile, then to the longer polling interval, then to the
    smaller worker (which leaves more of its CU to other kernels)."""
    best = None
    for (tile, sleep, threads), v in timings.items():
        key = (float(np.median(v)), -tile, -sleep, threads)
        if best is None or key < best[0]:
            best = (key, (tile, sleep, threads))
    return best[1]


def tune(run_burst, sizes, tiles=TILE_CANDIDATES, sleeps=SLEEP_CANDIDATES, threads=THREAD_CANDIDATES, reps=5):
    """run_burst(size, tile, sleep, threads, reps) -> list of makespans (us) of a training
    burst.  The polling interval and the worker size are properties of a running context,
    so they are the outer loops (one context per pair).  Returns {size: {"tile": t,
    "poll_sleep": s, "threads": w, "median_us": m, "grid": {...}}}."""
    timings = {size: {} for size in sizes}
    for thr in threads:
        for sleep in sleeps:
            for size in sizes:
                for tile in tiles:
                    timings[size][(tile, sleep, thr)] = list(run_burst(size, tile, sleep, thr, reps))
    table = {}
    for size in sizes:
        tile, sleep, thr = pick_best(timings[size])
        table[int(size)] = {"tile": int(tile), "poll_sleep": int(sleep), "threads": int(thr),
                            "median_us": float(np.median(timings[size][(tile, sleep, thr)])),
                            "grid": {f"{t}/{s}/{w}": float(np.median(v)) for (t, s, w), v in timings[size].items()}}
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
    # tables written before the worker size was tuned hold 256-thread workers
    return {int(k): {"threads": 256, **v} for k, v in d["table"].items()}
