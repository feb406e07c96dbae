"""Seeded synthetic inputs for the dispatch workloads.

This module only draws random numbers; it holds none of the method's arithmetic.  Both
the CPU oracle (in the tests and the CPU baseline) and the GPU path are fed from here.
The paper's own work item is a compute-only loop (Sec. 3) and it uses no dataset; the
items below are synthetic, with the shapes and distributions of the evaluation
workloads.
"""
import numpy as np

# plain: 1 worker, 1000 sequential items, int32 affine + int64 sum over 4096 elements
PLAIN_ITEMS, PLAIN_N = 1000, 4096
# all CUs: one worker per CU, 10,000 SAXPY items per mailbox over 16,384 fp32
ALLCU_ITEMS, ALLCU_N = 10000, 16384
# ... fed as the benchmark does: workers of 1024 threads (four wave64 per SIMD), ring
# depth 1 (4 in the pipelined form), and in the cold form each mailbox rotating through
# 16 (x, y) pairs (512 MiB in all, more than the 256 MB Infinity Cache)
ALLCU_THREADS, ALLCU_PIPELINED_DEPTH, ALLCU_COLD_PAIRS = 1024, 4, 16

# batching: bursts of uneven items, log-uniform 256 .. 2^20 elements, affine / SAXPY 50/50
BATCH_SIZES = (1, 4, 16, 64, 256, 1024, 4096)
BATCH_LOG2_RANGE = (8, 20)
# serving: Poisson arrivals, op mix 40% affine / 30% sum / 30% SAXPY, log-uniform
# 256 .. 2^22 elements
SERVE_RATES = (10_000, 100_000, 1_000_000)
SERVE_LOG2_RANGE = (8, 22)
# cluster isolation: critical int32 affine+sum over 262,144 elements, 1 ms period;
# interference: 256 MiB fp32 copies on the other clusters
ISO_N, ISO_PERIOD_S, ISO_COPY_ELEMS = 262144, 1e-3, (256 << 20) // 4


def feeder_threads(cpus=None):
    """Host threads feeding the all-CU mailboxes: every host CPU but two, at most 14."""
    import os
    cpus = os.cpu_count() if cpus is None else cpus
    return max(1, min(14, (cpus or 2) - 2))


def uniform_i32(rng, shape):
    return rng.integers(0, 2 ** 32, shape, dtype=np.uint32).view(np.int32)


def plain(seed=0, items=PLAIN_ITEMS, n=PLAIN_N):
    """X[items, n] int32 ~ uniform over all int32, AB[items, 2] int32 ~ uniform."""
    rng = np.random.default_rng(seed)
    X = uniform_i32(rng, (items, n))
    AB = uniform_i32(rng, (items, 2))
    return X, AB


def allcu_lane(w, items=ALLCU_ITEMS, n=ALLCU_N, seed=2):
    """Lane w (dense worker index): x, y ~ N(0,1) fp32, alpha[items] ~ U(-2, 2) fp32."""
    rng = np.random.default_rng([seed, w])
    x = rng.standard_normal(n, dtype=np.float32)
    y = rng.standard_normal(n, dtype=np.float32)
    alpha = rng.uniform(-2, 2, items).astype(np.float32)
    return x, y, alpha


def isolation(seed=3, periods=100000, n=ISO_N):
    """Critical item input x[n] (fixed) and per-period (a, b) pairs."""
    rng = np.random.default_rng(seed)
    x = uniform_i32(rng, n)
    AB = uniform_i32(rng, (periods, 2))
    return x, AB


def isolation_copy_source(cluster, elems=ISO_COPY_ELEMS, seed=3):
    """Private fp32 ~ N(0,1) source buffer of one interfering cluster."""
    rng = np.random.default_rng([seed, 100 + cluster])
    return rng.standard_normal(elems, dtype=np.float32)


def isolation_copy_source_device(cluster, elems=ISO_COPY_ELEMS, device="cuda", seed=3):
    """The same kind of private source as isolation_copy_source, drawn on the device with
    torch's seeded generator (fp32 ~ N(0,1)) so that 256 MiB buffers need no host copy."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed * 1000 + 100 + cluster)
    return torch.randn(elems, generator=g, device=device, dtype=torch.float32)


def batching(count, seed=5, log2_range=BATCH_LOG2_RANGE):
    """A burst of `count` uneven items: ops (1 = int32 affine + sum, 3 = fp32 SAXPY, each
    with probability 1/2), element counts round(2**U(lo, hi)), per-item a, b (int32) and
    alpha ~ U(-2, 2)."""
    rng = np.random.default_rng(seed)
    ops = np.where(rng.random(count) < 0.5, 1, 3).astype(np.uint32)
    n = np.rint(2.0 ** rng.uniform(log2_range[0], log2_range[1], count)).astype(np.uint64)
    ab = uniform_i32(rng, (count, 2))
    alpha = rng.uniform(-2, 2, count).astype(np.float32)
    return ops, n, ab, alpha


def device_arena(elems, seed, device="cuda"):
    """Seeded device buffers for burst inputs: x as random 32-bit words, y ~ N(0,1) fp32."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed * 7919 + 1)
    x = torch.randint(-2 ** 31, 2 ** 31 - 1, (elems,), generator=g, device=device, dtype=torch.int32)
    y = torch.randn(elems, generator=g, device=device, dtype=torch.float32)
    return x, y


def serving(rate, seconds, pool_elems, seed=7, log2_range=SERVE_LOG2_RANGE, max_requests=None):
    """Poisson request trace: arrival times (us) with exponential inter-arrival 1/rate,
    op choice [affine + sum, sum, SAXPY] with p = [.4, .3, .3], n = round(2**U(lo, hi)),
    input windows at uniform 256-aligned offsets inside a resident pool of pool_elems
    elements (x and, for SAXPY, y), per-request a, b (int32) and alpha ~ U(-2, 2)."""
    rng = np.random.default_rng(seed)
    count = int(rate * seconds) if max_requests is None else int(max_requests)
    gaps = rng.exponential(1.0 / rate, count)
    arrival_us = np.cumsum(gaps) * 1e6
    kind = rng.choice(3, size=count, p=[0.4, 0.3, 0.3])
    n = np.rint(2.0 ** rng.uniform(log2_range[0], log2_range[1], count)).astype(np.uint64)
    n = np.minimum(n, pool_elems)
    slots = (pool_elems - n) // 256
    off_x = (rng.random(count) * (slots + 1)).astype(np.uint64) * 256
    off_y = (rng.random(count) * (slots + 1)).astype(np.uint64) * 256
    ab = uniform_i32(rng, (count, 2))
    alpha = rng.uniform(-2, 2, count).astype(np.float32)
    return dict(arrival_us=arrival_us, kind=kind, n=n, off_x=off_x, off_y=off_y, ab=ab, alpha=alpha)
