"""Autotuner of the batched persistent dispatch: per burst size, the tile size (elements
per claimed tile) and the workers' polling interval that minimise the median makespan.

Tuning runs on training bursts (their own seed) and the chosen table is then used on the
evaluation bursts.  Larger tiles cost fewer counter claims and less per-tile overhead;
smaller tiles balance uneven items better over the 256 workers; the polling interval
trades PCIe read traffic of idle workers against pickup latency.
"""
import json
import os

import numpy as np

TILE_CANDIDATES = (4096, 16384, 65536, 262144)
SLEEP_CANDIDATES = (0, 8)


def pick_best(timings):
    """timings: {(tile, sleep): [makespan_us, ...]} -> (tile, sleep) with the smallest
    median; ties go to the larger tile, then to the longer polling interval."""
    best = None
    for (tile, sleep), v in timings.items():
        key = (float(np.median(v)), -tile, -sleep)
        if best is None or key < best[0]:
            best = (key, (tile, sleep))
    return best[1]


def tune(run_burst, sizes, tiles=TILE_CANDIDATES, sleeps=SLEEP_CANDIDATES, reps=5):
    """run_burst(size, tile, sleep, reps) -> list of makespans (us) of a training burst.
    The polling interval is a property of a running context, so it is the outermost loop
    (one context per interval).  Returns {size: {"tile": t, "poll_sleep": s,
    "median_us": m, "grid": {...}}}."""
    timings = {size: {} for size in sizes}
    for sleep in sleeps:
        for size in sizes:
            for tile in tiles:
                timings[size][(tile, sleep)] = list(run_burst(size, tile, sleep, reps))
    table = {}
    for size in sizes:
        tile, sleep = pick_best(timings[size])
        table[int(size)] = {"tile": int(tile), "poll_sleep": int(sleep),
                            "median_us": float(np.median(timings[size][(tile, sleep)])),
                            "grid": {f"{t}/{s}": float(np.median(v)) for (t, s), v in timings[size].items()}}
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
    return {int(k): v for k, v in d["table"].items()}
