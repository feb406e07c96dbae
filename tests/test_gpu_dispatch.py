"""GPU parity of the persistent dispatch path against the CPU oracle, through the C ABI.

Each test prints the case it runs (seed, shape, entry point) before touching the GPU.
While a context is open nothing here calls a device-wide synchronisation: results are
read after close(), or through an independent stream (the visibility test).
"""
import os
import time

import numpy as np
import pytest

import oracle
from paper_2310_01212_amd import lk, workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SENT_I32 = 0x7FBADBAD
SENT_F32_BITS = 0x7FA0DEAD  # a signalling-NaN payload


def say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def gpu():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    lk.lib()
    oracle.build(force=False)
    torch.cuda.synchronize()
    yield
    torch.cuda.synchronize()


def to_dev(a):
    t = torch.from_numpy(np.ascontiguousarray(a)).to("cuda")
    torch.cuda.current_stream().synchronize()
    return t


def _shape(shape):
    return (shape,) if isinstance(shape, int) else tuple(shape)


def sentinel_i32(shape):
    return torch.full(_shape(shape), SENT_I32, dtype=torch.int32, device="cuda")


def sentinel_f32(shape):
    return torch.full(_shape(shape), SENT_F32_BITS, dtype=torch.int32, device="cuda").view(torch.float32)


def addr(t, elem_offset=0):
    return t.data_ptr() + elem_offset * t.element_size()


def same_f32(got, want):
    """Bitwise equality, except that a NaN result only has to be a NaN: IEEE 754 leaves
    the sign and payload of a NaN produced by an operation to the implementation."""
    got = np.asarray(got, np.float32)
    want = np.asarray(want, np.float32)
    nan = np.isnan(want)
    return bool(np.array_equal(np.isnan(got), nan) and
                np.array_equal(got[~nan].view(np.uint32), want[~nan].view(np.uint32)))


def check_log(entries, n_items, code, allowed_xcc=None):
    """I1 exactly once and I2 FIFO per mailbox; I3 placement on allowed XCDs."""
    assert entries.size == n_items
    assert np.array_equal(entries["seq"], np.arange(1, n_items + 1, dtype=np.uint32))
    if code is not None:
        assert np.all(entries["code"] == code)
    assert np.all(entries["t_done"] >= entries["t_pick"])
    if allowed_xcc is not None:
        assert set(np.unique(entries["xcc"]).tolist()) <= set(allowed_xcc)
    cu_bits = entries["hwid"] & 0x7F00  # CU_ID, SH_ID, SE_ID fields: the physical CU
    assert np.unique(cu_bits).size == 1, "a worker moved between CUs"


# ------------------------------------------------------------------ plain: 1 worker, 1000 items
def test_plain_1000_items_bit_exact_with_log_invariants():
    say("plain: 1 worker x 1000 affine+sum items of 4096 int32, seed 0")
    X, AB = workloads.plain()
    x = to_dev(X)
    y = sentinel_i32(X.shape)
    torch.cuda.current_stream().synchronize()
    rows = np.arange(X.shape[0], dtype=np.uint64)
    items = lk.make_items(lk.OP_AFFINE_SUM_I32, X.shape[1], addr(x) + rows * X.shape[1] * 4,
                          addr(y) + rows * X.shape[1] * 4, AB[:, 0], AB[:, 1])
    ctx = lk.Context(n_workers=1, log_capacity=2048)
    try:
        res, lat, trig, comp = ctx.run_serial(0, items)
    finally:
        ctx.close()
    Y = y.cpu().numpy()
    for i in range(X.shape[0]):
        yr, sr = oracle.affine_sum_i32(X[i], int(AB[i, 0]), int(AB[i, 1]))
        assert res[i] == sr, i
        assert np.array_equal(Y[i], yr), i
    check_log(ctx.log(0), X.shape[0], lk.CODE_WORK + lk.OP_AFFINE_SUM_I32)
    assert np.all(lat > 0) and np.all(trig <= lat)
    info = ctx.info()
    assert info["state"] == 1 and info["kernel_ms"] > 0


@pytest.mark.parametrize("delay", [0, 40, lk.POLL_DELAY_ADAPTIVE])
def test_first_poll_delay_settings_keep_results_and_order(delay):
    say(f"first poll delay {delay}: 1 worker x 300 affine+sum items of 4096 int32")
    X, AB = workloads.plain(items=300)
    x = to_dev(X)
    y = sentinel_i32(X.shape)
    rows = np.arange(X.shape[0], dtype=np.uint64)
    items = lk.make_items(lk.OP_AFFINE_SUM_I32, X.shape[1], addr(x) + rows * X.shape[1] * 4,
                          addr(y) + rows * X.shape[1] * 4, AB[:, 0], AB[:, 1])
    with lk.Context(n_workers=1, first_poll_delay=delay, log_capacity=512) as ctx:
        res, _, _, _ = ctx.run_serial(0, items)
    Y = y.cpu().numpy()
    for i in range(X.shape[0]):
        yr, sr = oracle.affine_sum_i32(X[i], int(AB[i, 0]), int(AB[i, 1]))
        assert res[i] == sr and np.array_equal(Y[i], yr), i
    check_log(ctx.log(0), X.shape[0], lk.CODE_WORK + lk.OP_AFFINE_SUM_I32)


# ------------------------------------------------------------------ edge cases on one worker
EDGE_N = [0, 1, 3, 4, 5, 255, 256, 257, 1023, 4097, 65537, 1000003]


def _edge_items(rng, sizes=EDGE_N):
    """(op, n, x_off, y_off) with ragged sizes and misalignments."""
    cases = []
    for n in sizes:
        for xo, yo in [(0, 0), (1, 1), (3, 3), (1, 2)]:
            cases.append((lk.OP_AFFINE_SUM_I32, n, xo, yo))
            cases.append((lk.OP_SAXPY_F32, n, xo, yo))
        cases.append((lk.OP_SUM_I32_I64, n, 2, 0))
        cases.append((lk.OP_COPY_F32, n, 1, 3))
    return cases


def test_edge_cases_ragged_misaligned_and_special_values():
    _run_edge_cases(256, EDGE_N, seed=42)


@pytest.mark.parametrize("threads", [64, 512, 1024])
def test_other_worker_sizes_match_oracle(threads):
    """Workgroups of 1, 8 and 16 waves run the same bodies (strides, wave reduction)."""
    _run_edge_cases(threads, [0, 1, 255, 257, 4097, 65537, 300001], seed=43 + threads)


def _run_edge_cases(threads, sizes, seed):
    rng = np.random.default_rng(seed)
    cases = _edge_items(rng, sizes)
    say(f"edge: {len(cases)} items, ragged n up to {max(sizes)}, misaligned in/out, {threads} threads/worker")
    span = max(sizes) + 8
    xs_i = rng.integers(-2 ** 31, 2 ** 31, (len(cases), span), dtype=np.int64).astype(np.int32)
    # float inputs with specials: subnormals, +-0, inf, nan payloads, near-overflow
    xs_f = rng.standard_normal((len(cases), span)).astype(np.float32)
    ys_f = rng.standard_normal((len(cases), span)).astype(np.float32)
    special = np.array([0.0, -0.0, np.inf, -np.inf, np.nan, 1e-45, -1e-40, 3e38, -3e38], np.float32)
    xs_f[:, :special.size] = special
    ys_f[:, 1:special.size + 1] = special[::-1]
    xs_f.view(np.uint32)[:, 20] = 0x7FC01234  # quiet NaN with payload
    x_i = to_dev(xs_i)
    x_f = to_dev(xs_f)
    y_f = to_dev(ys_f.copy())
    y_i = sentinel_i32((len(cases), span))
    torch.cuda.current_stream().synchronize()
    AB = rng.integers(-2 ** 31, 2 ** 31, (len(cases), 2), dtype=np.int64)
    alphas = rng.uniform(-2, 2, len(cases)).astype(np.float32)
    alphas[::7] = np.float32(0.0)
    rows = []
    for r, (op, n, xo, yo) in enumerate(cases):
        if op in (lk.OP_AFFINE_SUM_I32, lk.OP_SUM_I32_I64):
            inp, out = addr(x_i, r * span + xo), addr(y_i, r * span + yo)
        elif op == lk.OP_SAXPY_F32:
            inp, out = addr(x_f, r * span + xo), addr(y_f, r * span + yo)
        else:
            inp, out = addr(x_f, r * span + xo), addr(y_i, r * span + yo)
        rows.append((op, n, inp, out, AB[r, 0], AB[r, 1], alphas[r]))
    cols = list(zip(*rows))
    items = lk.make_items(np.array(cols[0]), np.array(cols[1], np.uint64), np.array(cols[2], np.uint64),
                          np.array(cols[3], np.uint64), np.array(cols[4]), np.array(cols[5]),
                          np.array(cols[6], np.float32))
    # NOP and SPIN ride along (no memory effect, result 0)
    extra = lk.make_items(np.array([lk.OP_NOP, lk.OP_SPIN]), 0, 0, 0, a=np.array([0, 2000]), b=0)
    items = np.concatenate([items, extra])
    with lk.Context(n_workers=1, threads=threads, log_capacity=4096) as ctx:
        assert ctx.info()["threads_per_worker"] == threads
        res, _, _, _ = ctx.run_serial(0, items)
    YI = y_i.cpu().numpy()
    YF = y_f.cpu().numpy()
    for r, (op, n, xo, yo) in enumerate(cases):
        if op == lk.OP_AFFINE_SUM_I32:
            yr, sr = oracle.affine_sum_i32(xs_i[r, xo:xo + n].copy(), int(AB[r, 0]), int(AB[r, 1]))
            assert res[r] == sr, (r, op, n)
            assert np.array_equal(YI[r, yo:yo + n], yr), (r, n, xo, yo)
            assert np.all(YI[r, :yo] == SENT_I32) and np.all(YI[r, yo + n:] == SENT_I32)
        elif op == lk.OP_SUM_I32_I64:
            assert res[r] == oracle.sum_i32_i64(xs_i[r, xo:xo + n].copy()), (r, n)
        elif op == lk.OP_SAXPY_F32:
            yr = ys_f[r].copy()
            seg = yr[yo:yo + n].copy()
            oracle.saxpy_f32(alphas[r], xs_f[r, xo:xo + n].copy(), seg)
            yr[yo:yo + n] = seg
            assert same_f32(YF[r], yr), (r, n, xo, yo)
        else:
            got = YI[r, yo:yo + n].view(np.uint32)
            want = oracle.copy_f32(xs_f[r, xo:xo + n].copy()).view(np.uint32)
            assert np.array_equal(got, want), (r, n)
            assert np.all(YI[r, yo + n:] == SENT_I32)
    assert res[-1] == 0 and res[-2] == 0


# ------------------------------------------------------------------ all CUs: small, full compare
def _allcu_setup(ctx, items_per_lane, n_of_lane):
    lanes = ctx.info()["n_workers"]
    span = max(n_of_lane(w) for w in range(lanes)) + 4
    X = np.zeros((lanes, span), np.float32)
    Y0 = np.zeros((lanes, span), np.float32)
    A = np.zeros((lanes, items_per_lane), np.float32)
    for w in range(lanes):
        x, y, a = workloads.allcu_lane(w, items=items_per_lane, n=n_of_lane(w))
        X[w, :x.size], Y0[w, :y.size], A[w] = x, y, a
    return X, Y0, A, span


def test_all_cus_small_fifo_chains_bit_exact():
    with lk.Context(n_workers=0, log_capacity=128) as ctx:
        lanes = ctx.info()["n_workers"]
        assert lanes == ctx.info()["cu_count"]
        say(f"all CUs small: {lanes} lanes x 60 SAXPY items, ragged n")
        nl = lambda w: 1000 + 37 * (w % 11)
        X, Y0, A, span = _allcu_setup(ctx, 60, nl)
        x, y = to_dev(X), to_dev(Y0)
        torch.cuda.current_stream().synchronize()
        lanes_idx = np.arange(lanes, dtype=np.uint64)[:, None]
        n = np.array([nl(w) for w in range(lanes)], np.uint64)[:, None]
        items = lk.make_items(lk.OP_SAXPY_F32, n, addr(x) + lanes_idx * span * 4,
                              addr(y) + lanes_idx * span * 4, alpha=A)
        res, lat, el = ctx.run_lanes(np.arange(lanes), items, in_flight=1, threads=8)
    Y = y.cpu().numpy()
    for w in range(lanes):
        yr = Y0[w, :nl(w)].copy()
        oracle.run_fifo([dict(op=oracle.SAXPY_F32, inp=X[w, :nl(w)].copy(), out=yr, alpha=a) for a in A[w]])
        assert np.array_equal(Y[w, :nl(w)].view(np.uint32), yr.view(np.uint32)), w
        check_log(ctx.log(w), 60, lk.CODE_WORK + lk.OP_SAXPY_F32)
    # workers are in physical order and each sits on its own CU, every XCD holding the same
    # number of them (32 on each of the 8 XCDs of an MI355X)
    topo = [ctx.topology(w) for w in range(lanes)]
    assert topo == sorted(topo) and len(set(topo)) == lanes
    per_xcd = np.unique(np.array([t[0] for t in topo]), return_counts=True)[1]
    assert np.all(per_xcd == lanes // per_xcd.size), per_xcd


def test_rotating_buffer_pairs_chains_bit_exact():
    """The cold pattern: each mailbox's items rotate through P (x, y) pairs (item k uses
    pair k mod P); every pair's final y is the oracle's chain of its own alphas."""
    P, items, n = 4, 40, 2048
    with lk.Context(n_workers=0, threads=1024, idle_timeout_ms=20000) as ctx:
        lanes = ctx.info()["n_workers"]
        say(f"rotating pairs: {lanes} lanes x {P} pairs x {items} SAXPY items of {n}")
        rng = np.random.default_rng(61)
        X = rng.standard_normal((lanes, P, n)).astype(np.float32)
        Y0 = rng.standard_normal((lanes, P, n)).astype(np.float32)
        A = rng.uniform(-2, 2, (lanes, items)).astype(np.float32)
        x, y = to_dev(X), to_dev(Y0)
        torch.cuda.current_stream().synchronize()
        li = np.arange(lanes, dtype=np.uint64)[:, None]
        pair = (np.arange(items) % P).astype(np.uint64)[None, :]
        off = (li * P + pair) * n * 4
        ctx.run_lanes(np.arange(lanes), lk.make_items(lk.OP_SAXPY_F32, n, addr(x) + off, addr(y) + off, alpha=A),
                      in_flight=1, threads=8)
    Y = y.cpu().numpy()
    for w in range(lanes):
        for p in range(P):
            xr, yr = X[w, p].copy(), Y0[w, p].copy()  # the packed list points into both
            oracle.run_packed(oracle.pack_chain(oracle.SAXPY_F32, xr, yr, A[w, p::P]))
            assert np.array_equal(Y[w, p].view(np.uint32), yr.view(np.uint32)), (w, p)


@pytest.mark.parametrize("per_cu,threads", [(2, 256), (4, 256), (2, 512)])
def test_several_workers_per_cu_fifo_chains_bit_exact(per_cu, threads):
    """k persistent workgroups on every CU, each with its own mailbox: FIFO chains exact,
    exactly k workers on each physical CU, log invariants per worker."""
    with lk.Context(n_workers=0, workers_per_cu=per_cu, threads=threads, log_capacity=64) as ctx:
        info = ctx.info()
        lanes = info["n_workers"]
        say(f"{per_cu} workers per CU x {threads} threads: {lanes} lanes x 20 SAXPY items, ragged n")
        assert lanes == info["cu_count"] * per_cu and info["max_workers_on_a_cu"] == per_cu
        nl = lambda w: 600 + 37 * (w % 11)
        X, Y0, A, span = _allcu_setup(ctx, 20, nl)
        x, y = to_dev(X), to_dev(Y0)
        torch.cuda.current_stream().synchronize()
        li = np.arange(lanes, dtype=np.uint64)[:, None]
        n = np.array([nl(w) for w in range(lanes)], np.uint64)[:, None]
        items = lk.make_items(lk.OP_SAXPY_F32, n, addr(x) + li * span * 4, addr(y) + li * span * 4, alpha=A)
        ctx.run_lanes(np.arange(lanes), items, in_flight=1, threads=8)
        topo = [ctx.topology(w) for w in range(lanes)]
    Y = y.cpu().numpy()
    for w in range(lanes):
        yr = Y0[w, :nl(w)].copy()
        oracle.run_fifo([dict(op=oracle.SAXPY_F32, inp=X[w, :nl(w)].copy(), out=yr, alpha=a) for a in A[w]])
        assert np.array_equal(Y[w, :nl(w)].view(np.uint32), yr.view(np.uint32)), w
        check_log(ctx.log(w), 20, lk.CODE_WORK + lk.OP_SAXPY_F32)
    assert topo == sorted(topo)
    _, counts = np.unique(np.array(topo), axis=0, return_counts=True)
    assert counts.size == lanes // per_cu and np.all(counts == per_cu)


def _oracle_lane_chains(X, Y0, A, pair_of_item=None):
    """Final y of every lane (and pair) under the oracle's FIFO executor, lanes spread over
    host threads (the executor is plain C and releases the interpreter while it runs)."""
    import concurrent.futures as cf
    lanes = X.shape[0]

    def lane(w):
        if pair_of_item is None:
            yr = Y0[w].copy()
            oracle.run_packed(oracle.pack_chain(oracle.SAXPY_F32, X[w], yr, A[w]))
            return yr
        out = Y0[w].copy()
        for p in range(X.shape[1]):
            oracle.run_packed(oracle.pack_chain(oracle.SAXPY_F32, X[w, p], out[p], A[w][pair_of_item == p]))
        return out

    with cf.ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        return list(ex.map(lane, range(lanes)))


@pytest.mark.parametrize("depth,items", [(1, workloads.ALLCU_ITEMS), (workloads.ALLCU_PIPELINED_DEPTH, 3000)])
def test_all_cus_full_size_every_element_in_the_bench_launch_configuration(depth, items):
    """The all-CU workload exactly as the benchmark launches it: one worker of 1024
    threads per CU, ring depth 1 (and the pipelined depth 4), 16,384-element SAXPY items
    fed back-to-back by the same native runner and host thread count, operands laid out
    contiguously per lane.  Every element of every lane's final y against the oracle's
    FIFO chain of that lane's alphas (the chain is order-sensitive, so this also checks
    that each mailbox ran its items once each, in order)."""
    n, threads, feeders = workloads.ALLCU_N, workloads.ALLCU_THREADS, workloads.feeder_threads()
    lanes = torch.cuda.get_device_properties(0).multi_processor_count
    say(f"all CUs full size, bench launch configuration: {lanes} workers x {threads} threads, depth {depth}, "
        f"{items} SAXPY items of {n} per mailbox, {feeders} feeder threads")
    X = np.empty((lanes, n), np.float32)
    Y0 = np.empty((lanes, n), np.float32)
    A = np.empty((lanes, items), np.float32)
    for w in range(lanes):
        X[w], Y0[w], A[w] = workloads.allcu_lane(w, items=items, n=n)
    x, y = to_dev(X), to_dev(Y0)
    li = np.arange(lanes, dtype=np.uint64)[:, None]
    its = lk.make_items(lk.OP_SAXPY_F32, n, addr(x) + li * n * 4, addr(y) + li * n * 4, alpha=A)
    out = lk.lanes_outputs(lanes, items, with_info=True)  # as the benchmark passes them
    with lk.Context(n_workers=lanes, depth=depth, threads=threads, poll_sleep=0, idle_timeout_ms=60000) as ctx:
        t0 = time.time()
        res, lat, el, info = ctx.run_lanes(np.arange(lanes), its, in_flight=depth, threads=feeders, timeout=30.0,
                                           with_info=True, out=out)
        say(f"  {lanes * items / el:.0f} items/s, p50 {np.percentile(lat, 50):.2f} us, wall {time.time() - t0:.2f} s")
    assert not res.any()
    assert res is out[0] and lat is out[1] and info is out[2]
    assert np.all(lat > 0) and np.all(info["t_done_max"] >= info["t_pick_min"]) and np.all(info["t_pick_min"] > 0)
    Y = y.cpu().numpy()
    want = _oracle_lane_chains(X, Y0, A)
    for w in range(lanes):
        assert np.array_equal(Y[w].view(np.uint32), want[w].view(np.uint32)), w


@pytest.mark.parametrize("depth", [1, workloads.ALLCU_PIPELINED_DEPTH])
def test_all_cus_cold_form_full_size_every_element(depth):
    """The cold form of the all-CU workload as the benchmark runs it: every mailbox rotates
    through 16 (x, y) pairs of 16,384 fp32 (512 MiB in all, drawn on the device by the same
    seeded generator), item k using pair k mod 16, 48 items per lane; every element of
    every pair's final y against the oracle's chain of that pair's alphas."""
    n, P, items = workloads.ALLCU_N, workloads.ALLCU_COLD_PAIRS, 48
    threads, feeders = workloads.ALLCU_THREADS, workloads.feeder_threads()
    lanes = torch.cuda.get_device_properties(0).multi_processor_count
    say(f"all CUs cold form: {lanes} workers x {threads} threads, depth {depth}, {P} pairs x {n} per mailbox, "
        f"{items} items per mailbox")
    g = torch.Generator(device="cuda")
    g.manual_seed(2)
    cx = torch.randn((lanes, P, n), generator=g, device="cuda", dtype=torch.float32)
    cy = torch.randn((lanes, P, n), generator=g, device="cuda", dtype=torch.float32)
    X, Y0 = cx.cpu().numpy(), cy.cpu().numpy()
    A = np.stack([workloads.allcu_lane(w, items=items, n=n)[2] for w in range(lanes)])
    pair = (np.arange(items) % P).astype(np.uint64)
    li = np.arange(lanes, dtype=np.uint64)[:, None]
    off = (li * P + pair[None, :]) * n * 4
    its = lk.make_items(lk.OP_SAXPY_F32, n, addr(cx) + off, addr(cy) + off, alpha=A)
    torch.cuda.synchronize()
    with lk.Context(n_workers=lanes, depth=depth, threads=threads, poll_sleep=0, idle_timeout_ms=60000) as ctx:
        ctx.run_lanes(np.arange(lanes), its, in_flight=depth, threads=feeders, timeout=30.0)
    Y = cy.cpu().numpy()
    want = _oracle_lane_chains(X, Y0, A, pair_of_item=pair)
    for w in range(lanes):
        for p in range(P):
            assert np.array_equal(Y[w, p].view(np.uint32), want[w][p].view(np.uint32)), (w, p)


# ------------------------------------------------------------------ the paper's compute-only item
def test_spin_and_nop_items_leave_memory_untouched_and_match_the_oracle():
    """SPIN (the paper's compute-only item, Sec. 3) and NOP given sentinel-filled buffers
    as in/out: on one worker, on an XCD cluster of 32 members, inside a batch and as
    per-launch kernels, the buffers keep every sentinel word and the results equal the
    oracle's; in a FIFO with SAXPY items on one y, the final y equals the oracle's run of
    the same list, SPIN and NOP included."""
    n = 4096 + 37
    say(f"SPIN/NOP with sentinel buffers of {n}: 1 worker, XCD cluster, batch, per-launch")
    sx, sy = sentinel_f32(n), sentinel_i32(n)
    torch.cuda.synchronize()
    spin_it = lk.make_items([lk.OP_SPIN, lk.OP_NOP, lk.OP_SPIN], n, addr(sx), addr(sy), a=[20000, 0, 0])
    want = [oracle.exec_item(oracle.SPIN, n=n, a=20000), oracle.exec_item(oracle.NOP, n=n),
            oracle.exec_item(oracle.SPIN, n=n, a=0)]
    rng = np.random.default_rng(43)
    xf = rng.standard_normal(n).astype(np.float32)
    y0 = rng.standard_normal(n).astype(np.float32)
    al = rng.uniform(-2, 2, 6).astype(np.float32)
    dx, dy = to_dev(xf), to_dev(y0)
    ops = [lk.OP_SAXPY_F32, lk.OP_SPIN, lk.OP_SAXPY_F32, lk.OP_NOP, lk.OP_SAXPY_F32, lk.OP_SPIN]
    mix = lk.make_items(ops, n, addr(dx), addr(dy), a=[0, 5000, 0, 0, 0, 1], alpha=al)
    with lk.Context(n_workers=1, log_capacity=64) as ctx:
        res, _, _, _ = ctx.run_serial(0, spin_it)
        assert res.tolist() == want
        mres, _, _, _ = ctx.run_serial(0, mix)
    yr = y0.copy()
    ores = oracle.run_fifo([dict(op=int(o), inp=xf, out=yr, alpha=a, a=int(k), n=n)
                            for o, a, k in zip(ops, al, mix["a"])])
    assert mres.tolist() == ores.tolist()
    assert same_f32(dy.cpu().numpy(), yr)
    codes = [lk.CODE_WORK + lk.OP_SPIN, lk.CODE_WORK + lk.OP_NOP, lk.CODE_WORK + lk.OP_SPIN]
    assert ctx.log(0)["code"][:3].tolist() == codes
    with lk.Context(n_workers=0, clusters=lk.CLUSTERS_PER_XCD) as ctx:
        k = len(ctx.members(0))
        for it, w in zip(spin_it, want):
            t = ctx.submit(0, int(it["op"]), x=addr(sx), y=addr(sy), a=int(it["a"]), n=n)
            assert ctx.wait(0, t) == oracle.exec_cluster(int(it["op"]), k, n=n, a=int(it["a"])) == w
        tiles, _ = lk.batch_plan(spin_it, 1024)
        d = torch.from_numpy(tiles.view(np.uint8)).to("cuda")
        part = torch.full((tiles.size,), -7, dtype=torch.int64, device="cuda")
        torch.cuda.synchronize()
        ctx.run_batch(0, d, tiles.size, part, reps=1)
    assert not part.cpu().numpy().any()
    for mode in (lk.COMPLETE_SYNC, lk.COMPLETE_FLAG):
        lres, _, _ = lk.launch_serial(spin_it, k=4, mode=mode)
        assert lres.tolist() == want
    torch.cuda.synchronize()
    assert torch.all(sx.view(torch.int32) == SENT_F32_BITS) and torch.all(sy == SENT_I32)


# ------------------------------------------------------------------ pinned input (x in LDS)
def _pinned_sequence(ctx, cluster, n, seed):
    """Flagged, changed-x, unflagged, reload and new-address items on one cluster; returns
    (device y, expected y).  After x changes in memory, PIN_INPUT items must still see the
    pinned copy (the LDS copy is really what they read) until PIN_RELOAD replaces it."""
    rng = np.random.default_rng(seed)
    x0 = rng.standard_normal(n).astype(np.float32)
    x0[:4] = [np.inf, -0.0, 1e-40, 3e38]
    x2 = rng.standard_normal(n).astype(np.float32)
    y0 = rng.standard_normal(n).astype(np.float32)
    al = rng.uniform(-2, 2, 8).astype(np.float32)
    dx, dx2, dy = to_dev(x0), to_dev(x2), to_dev(y0)
    P, R = lk.DF_PIN_INPUT, lk.DF_PIN_RELOAD

    def run(xd, alpha, flags):
        t = ctx.submit(cluster, lk.OP_SAXPY_F32, x=addr(xd), y=addr(dy), alpha=alpha, n=n, flags=flags)
        ctx.wait(cluster, t)

    run(dx, al[0], P)                   # pins x0
    dx.add_(1.0)                        # x changes in memory: x1
    torch.cuda.synchronize()
    x1 = x0 + np.float32(1.0)
    run(dx, al[1], P)                   # pinned copy: x0
    run(dx, al[2], 0)                   # memory: x1
    run(dx, al[3], P)                   # still x0
    run(dx, al[4], R)                   # reload: x1
    run(dx, al[5], P)                   # x1
    run(dx2, al[6], P)                  # another address: x2
    run(dx, al[7], P)                   # back: x1 (its slice is still held)
    want = y0.copy()
    oracle.run_fifo([dict(op=oracle.SAXPY_F32, inp=xs, out=want, alpha=a)
                     for xs, a in zip([x0, x0, x1, x0, x1, x1, x2, x1], al)])
    torch.cuda.synchronize()
    return dy.cpu().numpy(), want


@pytest.mark.parametrize("n", [4, 260, 4096, 16384, 16388, 24576])
def test_pinned_input_reads_the_lds_copy_until_reload(n):
    with lk.Context(n_workers=1, idle_timeout_ms=20000) as ctx:
        cap = ctx.info()["pin_capacity"]
        assert cap == 96 * 1024 and n * 4 <= cap
        say(f"pinned input: one worker, n={n}")
        got, want = _pinned_sequence(ctx, 0, n, seed=n)
    assert same_f32(got, want)


def _pinned_slices_expected(cap_bytes, slots=4):
    """Which x a flagged item computes with, under the worker's table of pinned slices: a
    match (same address and length) is served from its copy unless RELOAD; a new slice is
    placed after the others while fewer than `slots` are held and all fit in cap_bytes,
    else the table is cleared first.  Returns see(addr, n, flags, memory) -> x."""
    table = []  # [addr, n, offset in elements, copy]

    def see(a, n, flags, mem):
        e = next((t for t in table if t[0] == a and t[1] == n), None)
        if e is not None and not flags & lk.DF_PIN_RELOAD:
            return e[3]
        if e is None:
            used = table[-1][2] + table[-1][1] if table else 0
            if len(table) == slots or (used + n) * 4 > cap_bytes:
                table.clear()
                used = 0
            e = [a, n, used, None]
            table.append(e)
        e[3] = mem.copy()
        return e[3]
    return see


@pytest.mark.parametrize("per_cu,n", [(1, 4096), (2, 6144)])
def test_pinned_input_keeps_several_slices_per_worker(per_cu, n):
    """Five x buffers through one worker's table of pinned slices: four 16 KiB slices stay
    pinned together at one worker per CU; at two per CU (78 KiB) 24 KiB slices overflow
    the capacity at the fourth.  Every x is changed in memory after it is pinned, so each
    flagged item shows which copy it read; the y chain is exact against the oracle's over
    the x each item should see."""
    rng = np.random.default_rng(500 + n)
    X = rng.standard_normal((5, n)).astype(np.float32)
    y0 = rng.standard_normal(n).astype(np.float32)
    dX, dy = to_dev(X), to_dev(y0)
    P, R = lk.DF_PIN_INPUT, lk.DF_PIN_RELOAD
    mem = X.copy()
    seq = []
    with lk.Context(n_workers=1, workers_per_cu=per_cu, threads=1024 // per_cu, idle_timeout_ms=20000) as ctx:
        cap = ctx.info()["pin_capacity"]
        see = _pinned_slices_expected(cap)
        say(f"pinned slices: {per_cu} per CU, capacity {cap}, n={n}")

        def run(k, flags, alpha):
            t = ctx.submit(0, lk.OP_SAXPY_F32, x=addr(dX[k]), y=addr(dy), alpha=alpha, n=n, flags=flags)
            ctx.wait(0, t)
            xs = see(addr(dX[k]), n, flags, mem[k]) if flags else mem[k].copy()
            seq.append((xs, np.float32(alpha)))

        def change(k, v):
            dX[k].add_(v)
            torch.cuda.synchronize()
            mem[k] = mem[k] + np.float32(v)

        for k in range(4):
            run(k, P, 0.5 + k)
        for k in range(5):
            change(k, 1.0 + k)
        for k in (3, 1, 0, 2):
            run(k, P, -0.75)
        run(1, 0, 1.25)                 # unflagged: memory
        run(4, P, 0.25)                 # a fifth slice
        run(0, P, -1.5)
        run(4, P, 2.0)
        change(4, -3.0)
        run(4, R, 0.5)                  # reload in place
        run(4, P, -0.5)
    want = y0.copy()
    oracle.run_fifo([dict(op=oracle.SAXPY_F32, inp=xs, out=want, alpha=a) for xs, a in seq])
    torch.cuda.synchronize()
    assert same_f32(dy.cpu().numpy(), want)


def test_pinned_input_refuses_shapes_the_buffer_cannot_take():
    with lk.Context(n_workers=1, idle_timeout_ms=20000) as ctx:
        cap = ctx.info()["pin_capacity"]
        big = torch.zeros(cap // 4 + 64, dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        say("pinned input: refused shapes")
        for kw in (dict(n=cap // 4 + 4), dict(n=1022), dict(n=64, x=addr(big, 1), y=addr(big, 1)),
                   dict(n=64, flags=4)):
            a = dict(x=addr(big), y=addr(big), flags=lk.DF_PIN_INPUT)
            a.update(kw)
            with pytest.raises(lk.LKError) as e:
                ctx.submit(0, lk.OP_SAXPY_F32, alpha=1.0, **a)
            assert e.value.code == lk.EINVAL
        with pytest.raises(lk.LKError):
            ctx.submit(0, lk.OP_COPY_F32, x=addr(big), y=addr(big), n=64, flags=lk.DF_PIN_INPUT)
        t = ctx.submit(0, lk.OP_SAXPY_F32, x=addr(big), y=addr(big), alpha=1.0, n=cap // 4, flags=lk.DF_PIN_INPUT)
        ctx.wait(0, t)  # the largest slice the buffer holds is accepted


def test_pinned_input_on_xcd_clusters_pins_each_members_slice():
    """An item sliced over the 32 members of an XCD: every member pins its own slice."""
    n = 131084  # slices of 4352 elements, a ragged 524-element one, and an empty one
    with lk.Context(n_workers=0, clusters=lk.CLUSTERS_PER_XCD, idle_timeout_ms=20000) as ctx:
        say(f"pinned input: XCD clusters, n={n}")
        res = [_pinned_sequence(ctx, c, n, seed=100 + c) for c in (0, ctx.info()["n_clusters"] - 1)]
    for got, want in res:
        assert same_f32(got, want)


@pytest.mark.parametrize("per_cu", [1, 2])
def test_pinned_input_all_cus_chains_bit_exact(per_cu):
    """The all-CU SAXPY shape (n = 16,384) with x pinned on every worker, k workers per
    CU each with its own copy: every lane's chain equals the oracle's."""
    items, n = 200, workloads.ALLCU_N
    with lk.Context(n_workers=0, workers_per_cu=per_cu, threads=1024 // per_cu, idle_timeout_ms=20000) as ctx:
        lanes = ctx.info()["n_workers"]
        say(f"pinned input all CUs: {per_cu} per CU, {lanes} lanes x {items} items of {n}")
        X, Y0, A, span = _allcu_setup(ctx, items, lambda w: n)
        assert span % 4 == 0
        x, y = to_dev(X), to_dev(Y0)
        torch.cuda.current_stream().synchronize()
        li = np.arange(lanes, dtype=np.uint64)[:, None]
        it = lk.make_items(lk.OP_SAXPY_F32, n, addr(x) + li * span * 4, addr(y) + li * span * 4, alpha=A,
                           flags=lk.DF_PIN_INPUT)
        ctx.run_lanes(np.arange(lanes), it, in_flight=1, threads=8)
    Y = y.cpu().numpy()
    for w in range(lanes):
        xr, yr = X[w, :n].copy(), Y0[w, :n].copy()
        oracle.run_packed(oracle.pack_chain(oracle.SAXPY_F32, xr, yr, A[w]))
        assert np.array_equal(Y[w, :n].view(np.uint32), yr.view(np.uint32)), w


def test_pinned_input_axpy_out_of_place():
    rng = np.random.default_rng(23)
    n = 8192
    x = rng.standard_normal(n).astype(np.float32)
    yv = rng.standard_normal(n).astype(np.float32)
    dx, dy = to_dev(x), to_dev(yv)
    outs = [sentinel_f32((n,)) for _ in range(3)]
    torch.cuda.synchronize()
    al = np.float32([0.75, -3.0, 1.5])
    say("pinned input: out-of-place AXPY")
    with lk.Context(n_workers=1, idle_timeout_ms=20000) as ctx:
        for o, a in zip(outs, al):
            t = ctx.submit(0, lk.OP_AXPY_F32, x=addr(dx), y=addr(o), alpha=a, n=n, aux=addr(dy),
                           flags=lk.DF_PIN_INPUT)
            ctx.wait(0, t)
    for o, a in zip(outs, al):
        assert same_f32(o.cpu().numpy(), oracle.axpy_f32(a, x.copy(), yv.copy()))


def _pinned_int_sequence(ctx, cluster, n, seed):
    """AFFINE_SUM_I32 and SUM_I32_I64 with x pinned: after x changes in memory, flagged
    items keep summing (and writing y from) the pinned copy until PIN_RELOAD.  Returns the
    (got, want) results and the final y pair."""
    rng = np.random.default_rng(seed)
    x0 = rng.integers(-2**31, 2**31, n, dtype=np.int64).astype(np.int32)
    x0[:2] = [np.iinfo(np.int32).min, np.iinfo(np.int32).max]
    dx = to_dev(x0)
    dy = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    P, R = lk.DF_PIN_INPUT, lk.DF_PIN_RELOAD
    x1 = x0 ^ np.int32(0x5A5A5A5)
    got, want, last_y = [], [], [None]

    def aff(a, b, flags, xs):
        got.append(ctx.wait(cluster, ctx.submit(cluster, lk.OP_AFFINE_SUM_I32, x=addr(dx), y=addr(dy), a=a, b=b,
                                                 n=n, flags=flags)))
        last_y[0], s = oracle.affine_sum_i32(xs.copy(), a, b)
        want.append(s)

    def isum(flags, xs):
        got.append(ctx.wait(cluster, ctx.submit(cluster, lk.OP_SUM_I32_I64, x=addr(dx), n=n, flags=flags)))
        want.append(oracle.sum_i32_i64(xs.copy()))

    aff(-3, 7, P, x0)                   # pins x0
    dx.bitwise_xor_(0x5A5A5A5)          # x changes in memory: x1
    torch.cuda.synchronize()
    aff(5, -11, P, x0)                  # pinned copy
    isum(P, x0)                         # same address and length: the copy again
    isum(0, x1)                         # memory
    aff(-1, 0, R, x1)                   # reload
    isum(P, x1)
    return got, want, dy.cpu().numpy(), last_y[0]


@pytest.mark.parametrize("n", [4, 4100, 24576])
def test_pinned_input_integer_ops_read_the_lds_copy_until_reload(n):
    with lk.Context(n_workers=1, idle_timeout_ms=20000) as ctx:
        say(f"pinned input, integer ops: one worker, n={n}")
        got, want, gy, wy = _pinned_int_sequence(ctx, 0, n, seed=300 + n)
    assert got == want
    assert np.array_equal(gy, wy)


def test_pinned_input_integer_ops_on_xcd_clusters():
    n = 131084
    with lk.Context(n_workers=0, clusters=lk.CLUSTERS_PER_XCD, idle_timeout_ms=20000) as ctx:
        say(f"pinned input, integer ops: XCD clusters, n={n}")
        res = [_pinned_int_sequence(ctx, c, n, seed=400 + c) for c in (0, ctx.info()["n_clusters"] - 1)]
    for got, want, gy, wy in res:
        assert got == want
        assert np.array_equal(gy, wy)


# ------------------------------------------------------------------ clusters = XCDs
def test_clusters_per_xcd_split_items_and_placement():
    rng = np.random.default_rng(3)
    with lk.Context(n_workers=0, clusters=lk.CLUSTERS_PER_XCD, log_capacity=64) as ctx:
        info = ctx.info()
        ncl = info["n_clusters"]
        say(f"clusters per XCD: {ncl} clusters; affine+sum over 262144(+ragged), tiny and empty items")
        assert ncl == info["xcd_count"]
        members = [ctx.members(c) for c in range(ncl)]
        xccs = [{ctx.topology(w)[0] for w in m} for m in members]
        assert all(len(s) == 1 for s in xccs)
        sizes = [262144, 262144 + 1000, 100, 0]
        N = max(sizes)
        X = rng.integers(-2 ** 31, 2 ** 31, (ncl, len(sizes), N), dtype=np.int64).astype(np.int32)
        AB = rng.integers(-2 ** 31, 2 ** 31, (ncl, len(sizes), 2), dtype=np.int64)
        x = to_dev(X)
        y = sentinel_i32(X.shape)
        aux = torch.zeros((ncl, len(sizes), 64), dtype=torch.int64, device="cuda")
        torch.cuda.current_stream().synchronize()
        results = {}
        for c in range(ncl):
            for s, n in enumerate(sizes):
                off = (c * len(sizes) + s) * N
                t = ctx.submit(c, lk.OP_AFFINE_SUM_I32, x=addr(x, off), y=addr(y, off), a=int(AB[c, s, 0]),
                               b=int(AB[c, s, 1]), n=n, aux=addr(aux, (c * len(sizes) + s) * 64))
                results[(c, s)] = ctx.wait(c, t)
    Y = y.cpu().numpy()
    AUX = aux.cpu().numpy()
    for c in range(ncl):
        k = len(members[c])
        for s, n in enumerate(sizes):
            yr, sr = oracle.affine_sum_i32(X[c, s, :n].copy(), int(AB[c, s, 0]), int(AB[c, s, 1]))
            assert results[(c, s)] == sr
            assert oracle.exec_cluster(oracle.AFFINE_SUM_I32, k, X[c, s, :n].copy(), np.empty(n, np.int32),
                                       a=int(AB[c, s, 0]), b=int(AB[c, s, 1])) == sr
            assert np.array_equal(Y[c, s, :n], yr) and np.all(Y[c, s, n:] == SENT_I32)
            assert AUX[c, s, :k].sum() == sr   # per-member partials
        for w in members[c]:
            check_log(ctx.log(w), len(sizes), lk.CODE_WORK + lk.OP_AFFINE_SUM_I32, allowed_xcc=xccs[c])


# ------------------------------------------------------------------ I4 visibility and coexistence
def test_xcd_mask_places_workers_only_on_the_named_xcds():
    """Workers restricted to XCD 0, then to XCDs 5 and 7: worker counts, placement from the
    hardware ids (at boot and in every log entry), XCD clusters computing exactly; masks
    beyond the device and too many workers for the masked CUs are refused."""
    rng = np.random.default_rng(29)
    n = 262144 + 1000
    X = rng.integers(-2 ** 31, 2 ** 31, n, dtype=np.int64).astype(np.int32)
    AB = rng.integers(-2 ** 31, 2 ** 31, (4, 2), dtype=np.int64).astype(np.int32)
    x = to_dev(X)
    for mask, xcds, per_cu in ((0x1, [0], 1), (0xA0, [5, 7], 1), (0x2, [1], 2)):
        say(f"xcd_mask {mask:#x}: workers on XCDs {xcds}, {per_cu} per CU")
        with lk.Context(n_workers=0, xcd_mask=mask, clusters=lk.CLUSTERS_PER_XCD, log_capacity=16,
                        idle_timeout_ms=20000, workers_per_cu=per_cu, threads=256) as ctx:
            info = ctx.info()
            per_xcd = info["cu_count"] // 8
            assert info["n_workers"] == per_xcd * len(xcds) * per_cu and info["xcd_mask"] == mask
            assert info["max_workers_on_a_cu"] == per_cu
            assert info["n_clusters"] == len(xcds) and info["xcd_count"] == len(xcds)
            for cl, xcd in enumerate(xcds):
                assert {ctx.topology(w)[0] for w in ctx.members(cl)} == {xcd}
            outs = []
            for cl in range(len(xcds)):
                y = sentinel_i32((n,))
                torch.cuda.synchronize()
                t = ctx.submit(cl, lk.OP_AFFINE_SUM_I32, x=x, y=y, a=int(AB[cl, 0]), b=int(AB[cl, 1]))
                outs.append((cl, y, ctx.wait(cl, t)))
        for cl, y, s_got in outs:
            yr, sr = oracle.affine_sum_i32(X, int(AB[cl, 0]), int(AB[cl, 1]))
            assert s_got == sr and np.array_equal(y.cpu().numpy(), yr), (mask, cl)
        for w in range(info["n_workers"]):
            assert set(np.unique(ctx.log(w)["xcc"]).tolist()) <= set(xcds)
    for kw in (dict(xcd_mask=0x100), dict(xcd_mask=0x1, n_workers=33)):
        with pytest.raises(lk.LKError) as e:
            lk.Context(**kw)
        assert e.value.code == lk.EINVAL


def test_completion_implies_visibility_on_an_independent_stream():
    rng = np.random.default_rng(11)
    n = 1 << 20
    X = rng.integers(-2 ** 31, 2 ** 31, n, dtype=np.int64).astype(np.int32)
    say("visibility: 1 worker, affine over 1 Mi int32, read back on an independent stream")
    x = to_dev(X)
    y = sentinel_i32((n,))
    torch.cuda.current_stream().synchronize()
    side = torch.cuda.Stream()
    with lk.Context(n_workers=4, idle_timeout_ms=4000) as ctx:
        for trial in range(3):
            a, b = int(rng.integers(-2 ** 31, 2 ** 31)), int(rng.integers(-2 ** 31, 2 ** 31))
            t = ctx.submit(trial % 4, lk.OP_AFFINE_SUM_I32, x=x, y=y, a=a, b=b)
            s = ctx.wait(trial % 4, t)
            t0 = time.time()
            with torch.cuda.stream(side):
                host = y.to("cpu", non_blocking=False)
                side.synchronize()
                z = (x.float() * 2).sum()  # torch compute while the workers spin
                side.synchronize()
            dt = time.time() - t0
            yr, sr = oracle.affine_sum_i32(X, a, b)
            assert s == sr
            assert np.array_equal(host.numpy(), yr)
            assert dt < 2.0, f"side stream took {dt:.2f} s: queued behind the persistent kernel?"
            # the legacy default stream and a device-wide synchronisation do not wait for
            # the persistent dispatch either: it lives on a queue of its own
            t0 = time.time()
            host2 = y.cpu()
            torch.cuda.synchronize()
            dt = time.time() - t0
            assert np.array_equal(host2.numpy(), yr)
            assert dt < 2.0, f"default stream took {dt:.2f} s"
            del z


@pytest.mark.parametrize("threads", [256, 1024])
def test_torch_work_progresses_beside_workers_on_every_cu(threads):
    """Torch kernels on a stream of their own run while a worker sits on every CU, also
    with the benchmark's 1024-thread workers (four worker waves per SIMD, 416 of its 512
    VGPRs held): elementwise work and a reduction finish within seconds, and afterwards
    every worker still serves items (none left on its idle watchdog meanwhile)."""
    say(f"coexistence: torch ops on a side stream beside 256 workers of {threads} threads")
    n = 1 << 20
    x = torch.randn(n, device="cuda")
    want = float((x.double() * 3 + 1).sum())
    y = torch.zeros(256, 1024, device="cuda")
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    with lk.Context(n_workers=0, threads=threads, idle_timeout_ms=6000) as ctx:
        nw = ctx.info()["n_workers"]
        for w in range(nw):
            ctx.wait(w, ctx.submit(w, lk.OP_SAXPY_F32, x=x[:1024], y=y[w], alpha=1.0))
        t0 = time.time()
        with torch.cuda.stream(side):
            z = float((x.double() * 3 + 1).sum())
            side.synchronize()
        dt = time.time() - t0
        assert dt < 2.0, f"torch work on a side stream took {dt:.2f} s beside the workers"
        assert abs(z - want) <= 1e-9 * max(1.0, abs(want))
        for w in range(nw):
            ctx.wait(w, ctx.submit(w, lk.OP_SAXPY_F32, x=x[:1024], y=y[w], alpha=1.0))
    got = y.cpu().numpy()
    xs = x[:1024].cpu().numpy()
    want_y = np.zeros(1024, np.float32)
    for _ in range(2):
        oracle.saxpy_f32(np.float32(1.0), xs.copy(), want_y)
    for w in range(nw):
        assert same_f32(got[w], want_y), w


# ------------------------------------------------------------------ error paths
def test_ring_full_timeout_and_disposed_state():
    say("errors: EAGAIN at depth 1, ETIMEDOUT on a long SPIN item, ESTATE after close")
    with lk.Context(n_workers=1, depth=1, idle_timeout_ms=5000) as ctx:
        t1 = ctx.submit(0, lk.OP_SPIN, a=2_000_000)
        with pytest.raises(lk.LKError) as e:
            ctx.submit(0, lk.OP_NOP)
        assert e.value.code == lk.EAGAIN
        with pytest.raises(lk.LKError) as e:
            ctx.wait(0, t1, timeout=0.0)
        assert e.value.code == lk.ETIMEDOUT
        assert ctx.try_wait(0, t1) is None  # not finished: nothing released
        assert ctx.wait(0, t1, timeout=10.0) == 0
        with pytest.raises(lk.LKError) as e:
            ctx.wait(0, t1)
        assert e.value.code == lk.EINVAL   # already released
        t2 = ctx.submit(0, lk.OP_NOP)
        ctx.prefetch(0, t2)  # a hint: no effect on the result
        assert ctx.wait(0, t2) == 0
        xs = torch.arange(1000, dtype=torch.int32, device="cuda")
        torch.cuda.synchronize()
        t3 = ctx.submit(0, lk.OP_SUM_I32_I64, x=xs)
        done = None
        while done is None:
            done = ctx.try_wait(0, t3)
        assert done["result"] == 999 * 1000 // 2
        with pytest.raises(lk.LKError) as e:
            ctx.try_wait(0, t3)
        assert e.value.code == lk.EINVAL  # already released
        ctx.prefetch(0, t2)  # released ticket: only the next command slot
        with pytest.raises(lk.LKError) as e:
            ctx.prefetch(1, 0)
        assert e.value.code == lk.EINVAL
    with pytest.raises(lk.LKError) as e:
        ctx.submit(0, lk.OP_NOP)
    assert e.value.code == lk.ESTATE
    with pytest.raises(lk.LKError) as e:
        ctx.prefetch(0, 0)
    assert e.value.code == lk.ESTATE
    ctx.close()  # idempotent


@pytest.mark.parametrize("in_flight,flags,threads,n", [(8, 0, 256, 4096), (8, lk.F_NO_LOOKAHEAD, 256, 4096),
                                                        (1, 0, 256, 4096), (3, 0, 256, 4096),
                                                        (8, 0, 64, 65536), (8, 0, 1024, 65536)])
def test_deeper_ring_keeps_fifo(in_flight, flags, threads, n):
    """Depth 8 with the ring kept full (the look-ahead read finds the next command), with
    the look-ahead switched off, with fewer items in flight than slots (it finds an old
    sequence number in the next slot and falls back to polling), and with items long
    enough for the look-ahead on workers of one wave and of sixteen."""
    rng = np.random.default_rng(5)
    x0 = rng.standard_normal(n).astype(np.float32)
    y0 = rng.standard_normal(n).astype(np.float32)
    alphas = rng.uniform(-2, 2, 200).astype(np.float32)
    say(f"depth 8: 200 SAXPY items of {n} on one mailbox, {in_flight} in flight, flags {flags}, {threads} threads")
    x, y = to_dev(x0), to_dev(y0)
    with lk.Context(n_workers=1, depth=8, log_capacity=256, flags=flags, threads=threads) as ctx:
        items = lk.make_items(lk.OP_SAXPY_F32, n, addr(x), addr(y), alpha=alphas)[None, :]
        res, lat, el = ctx.run_lanes([0], items, in_flight=in_flight, threads=1)
    want = y0.copy()
    oracle.run_fifo([dict(op=oracle.SAXPY_F32, inp=x0, out=want, alpha=a) for a in alphas])
    assert np.array_equal(y.cpu().numpy().view(np.uint32), want.view(np.uint32))
    check_log(ctx.log(0), 200, lk.CODE_WORK + lk.OP_SAXPY_F32)


def _mixed_depth4(flags, items_per_lane=64, n=65532):
    """All CUs at depth 4, each mailbox fed a FIFO mix of affine + sum, SAXPY, NOP and sum
    items four ahead; checks every result, the final outputs and the log order against
    the oracle and returns the median device-side gap from a completion to the next
    pickup (us)."""
    with lk.Context(n_workers=0, depth=4, log_capacity=128, idle_timeout_ms=20000, flags=flags) as ctx:
        lanes = ctx.info()["n_workers"]
        say(f"look-ahead flags {flags}: {lanes} lanes x {items_per_lane} mixed items at depth 4")
        rng = np.random.default_rng(71)
        span = n + 4
        XI = rng.integers(-2 ** 31, 2 ** 31, (lanes, span), dtype=np.int64).astype(np.int32)
        XF = rng.standard_normal((lanes, span)).astype(np.float32)
        YF0 = rng.standard_normal((lanes, span)).astype(np.float32)
        AB = rng.integers(-2 ** 31, 2 ** 31, (lanes, items_per_lane, 2), dtype=np.int64).astype(np.int32)
        AL = rng.uniform(-2, 2, (lanes, items_per_lane)).astype(np.float32)
        xi, xf, yf = to_dev(XI), to_dev(XF), to_dev(YF0)
        yi = sentinel_i32((lanes, span))
        torch.cuda.synchronize()
        li = np.arange(lanes, dtype=np.uint64)[:, None]
        kinds = np.array([lk.OP_AFFINE_SUM_I32, lk.OP_SAXPY_F32, lk.OP_NOP, lk.OP_SUM_I32_I64])
        op = np.broadcast_to(kinds[np.arange(items_per_lane) % 4], (lanes, items_per_lane))
        is_f = op == lk.OP_SAXPY_F32
        inp = np.where(is_f, addr(xf) + li * span * 4, addr(xi) + li * span * 4)
        out = np.where(is_f, addr(yf) + li * span * 4, addr(yi) + li * span * 4)
        nn = np.where(op == lk.OP_NOP, 0, n)
        it = lk.make_items(op, nn, inp, out, a=AB[..., 0], b=AB[..., 1], alpha=AL)
        res, lat, el = ctx.run_lanes(np.arange(lanes), it, in_flight=4, threads=8)
    YI, YF = yi.cpu().numpy(), yf.cpu().numpy()
    hz = ctx.info()["wall_clock_hz"]
    gaps = []
    for w in range(lanes):
        x = XI[w, :n].copy()
        s_sum = oracle.sum_i32_i64(x)
        y_last = None
        for k in range(items_per_lane):
            if op[w, k] == lk.OP_AFFINE_SUM_I32:
                y_last, sr = oracle.affine_sum_i32(x, int(AB[w, k, 0]), int(AB[w, k, 1]))
                assert res[w, k] == sr, (w, k)
            elif op[w, k] == lk.OP_SUM_I32_I64:
                assert res[w, k] == s_sum, (w, k)
        assert np.array_equal(YI[w, :n], y_last), w
        want = YF0[w, :n].copy()
        oracle.run_packed(oracle.pack_chain(oracle.SAXPY_F32, XF[w, :n].copy(), want, AL[w, is_f[w]]))
        assert np.array_equal(YF[w, :n].view(np.uint32), want.view(np.uint32)), w
        e = ctx.log(w)
        assert np.array_equal(e["seq"], np.arange(1, items_per_lane + 1, dtype=np.uint32))
        assert np.array_equal(e["code"], lk.CODE_WORK + op[w])
        gaps.append(np.median((e["t_pick"][1:] - e["t_done"][:-1]) * 1e6 / hz))
    say(f"  median gap completion -> next pickup {np.median(gaps):.2f} us")
    return float(np.median(gaps))


def test_lookahead_mixed_ops_all_cus_depth4_exact():
    """The mixed depth-4 workload with the look-ahead read and without it: exact both ways.
    Its items are long enough (65,532 elements) for the worker to read the next slot while
    each one runs, so with the look-ahead the device-side gap from a completion to the
    next pickup loses most of a host round trip."""
    gap_off = _mixed_depth4(lk.F_NO_LOOKAHEAD)
    gap_on = _mixed_depth4(0)
    assert gap_on < gap_off - 0.5, (gap_on, gap_off)


def test_idle_watchdog_ends_workers():
    say("watchdog: idle timeout 300 ms, then submit sees the exited workers")
    ctx = lk.Context(n_workers=2, idle_timeout_ms=300)
    time.sleep(1.0)
    assert ctx.info()["workers_exited"] == 2
    with pytest.raises(lk.LKError) as e:
        ctx.submit(0, lk.OP_NOP)
    assert e.value.code == lk.ESTATE
    ctx.close()
    assert ctx.info()["state"] == 1


# ------------------------------------------------------------------ per-launch baselines
@pytest.mark.parametrize("mode", [lk.COMPLETE_SYNC, lk.COMPLETE_FLAG, lk.COMPLETE_SYNC | lk.USE_GRAPH])
def test_per_launch_baseline_matches_oracle(mode):
    say(f"baseline launch mode {mode}: 50 plain items, then one 32-slice item")
    X, AB = workloads.plain(items=50)
    x = to_dev(X)
    y = sentinel_i32(X.shape)
    torch.cuda.current_stream().synchronize()
    rows = np.arange(50, dtype=np.uint64)
    items = lk.make_items(lk.OP_AFFINE_SUM_I32, 4096, addr(x) + rows * 4096 * 4, addr(y) + rows * 4096 * 4,
                          AB[:, 0], AB[:, 1])
    res, lat, lau = lk.launch_serial(items, k=1, mode=mode)
    Y = y.cpu().numpy()
    for i in range(50):
        yr, sr = oracle.affine_sum_i32(X[i], int(AB[i, 0]), int(AB[i, 1]))
        assert res[i] == sr and np.array_equal(Y[i], yr)
    big = np.random.default_rng(8).integers(-2 ** 31, 2 ** 31, 262144 + 5, dtype=np.int64).astype(np.int32)
    xb = to_dev(big)
    yb = sentinel_i32(big.shape)
    torch.cuda.current_stream().synchronize()
    it = lk.make_items(lk.OP_AFFINE_SUM_I32, big.size, addr(xb), addr(yb), 7, -3)[None]
    r2, _, _ = lk.launch_serial(it, k=32, mode=mode)
    yr, sr = oracle.affine_sum_i32(big, 7, -3)
    assert r2[0] == sr and np.array_equal(yb.cpu().numpy(), yr)


def test_launch_lanes_baseline_matches_oracle():
    say("baseline launch lanes: 16 lanes x 20 SAXPY items, 4 streams, plain, graph and graph chain")
    rng = np.random.default_rng(6)
    lanes, per, n = 16, 20, 3000
    X = rng.standard_normal((lanes, n)).astype(np.float32)
    Y0 = rng.standard_normal((lanes, n)).astype(np.float32)
    A = rng.uniform(-2, 2, (lanes, per)).astype(np.float32)
    for mode in (0, lk.USE_GRAPH, lk.GRAPH_CHAIN):
        x, y = to_dev(X), to_dev(Y0)
        li = np.arange(lanes, dtype=np.uint64)[:, None]
        items = lk.make_items(lk.OP_SAXPY_F32, n, addr(x) + li * n * 4, addr(y) + li * n * 4, alpha=A)
        lk.launch_lanes(items, streams=4, threads_host=4, mode=mode)
        Y = y.cpu().numpy()
        for w in range(lanes):
            want = Y0[w].copy()
            oracle.run_fifo([dict(op=oracle.SAXPY_F32, inp=X[w], out=want, alpha=a) for a in A[w]])
            assert np.array_equal(Y[w].view(np.uint32), want.view(np.uint32)), (mode, w)


# ------------------------------------------------------------------ probes
def test_pingpong_and_copy_probes_run():
    say("probes: pingpong 1 and 8 workers, copy 64 MiB")
    rtt = lk.pingpong(workers=1, iters=2000)
    assert rtt.shape == (1, 2000) and np.all(rtt > 0) and np.median(rtt) < 50
    rtt8 = lk.pingpong(workers=8, iters=200)
    assert np.all(rtt8 > 0)
    nbytes = 64 << 20
    src = torch.randint(-2 ** 31, 2 ** 31 - 1, (nbytes // 4,), dtype=torch.int32, device="cuda")
    dst = torch.zeros_like(src)
    torch.cuda.current_stream().synchronize()
    ms, gbps = lk.copy_bandwidth(src, dst, nbytes, grid=2048, reps=5)
    assert gbps > 100
    assert torch.equal(src.cpu(), dst.cpu())


@pytest.mark.parametrize("policy", [lk.COPY_PLAIN, lk.COPY_NONTEMPORAL, lk.COPY_SYSTEM])
def test_copy_probe_forms_copy_every_byte(policy):
    """Every launch shape and store policy of the bandwidth probe copies the buffer exactly,
    including a ragged tail of vectors beyond the unrolled loop; bytes after it untouched."""
    vec = (5 << 20) // 16 + 37
    src = torch.randint(-2 ** 31, 2 ** 31 - 1, (vec * 4,), dtype=torch.int32, device="cuda")
    for threads, unroll, grid in ((256, 4, 512), (1024, 8, 256), (64, 16, 1000), (1024, 16, 4096)):
        say(f"copy probe: policy {policy}, {threads} threads, unroll {unroll}, grid {grid}, {vec} vectors")
        dst = torch.full((vec * 4 + 64,), SENT_I32, dtype=torch.int32, device="cuda")
        torch.cuda.current_stream().synchronize()
        lk.copy_bandwidth(src, dst, vec * 16, grid=grid, reps=1, threads=threads, unroll=unroll, policy=policy)
        d = dst.cpu()
        assert torch.equal(d[:vec * 4], src.cpu()) and torch.all(d[vec * 4:] == SENT_I32)


# ------------------------------------------------------------------ cluster isolation runner
def test_isolation_runner_critical_items_and_copies_exact():
    say("isolation: 200 periods of 0.5 ms on XCD 0, copies of 16 MiB on XCDs 1-2")
    xh, AB = workloads.isolation(periods=200)
    x = to_dev(xh)
    y = sentinel_i32(xh.shape)
    elems = (16 << 20) // 4
    srcs = [workloads.isolation_copy_source_device(c, elems, "cuda") for c in (1, 2)]
    dsts = [torch.zeros_like(s) for s in srcs]
    torch.cuda.synchronize()
    crit = lk.make_items(lk.OP_AFFINE_SUM_I32, xh.size, addr(x), addr(y), AB[:, 0], AB[:, 1])
    bg = lk.make_items(lk.OP_COPY_F32, elems, [addr(s) for s in srcs], [addr(d) for d in dsts])
    with lk.Context(n_workers=0, clusters=lk.CLUSTERS_PER_XCD, idle_timeout_ms=20000) as ctx:
        r = ctx.run_isolation(0, crit, 0.5e-3, [1, 2], bg)
    for k in range(200):
        assert r["results"][k] == oracle.affine_sum_i32(xh, int(AB[k, 0]), int(AB[k, 1]))[1], k
    yr, _ = oracle.affine_sum_i32(xh, int(AB[-1, 0]), int(AB[-1, 1]))
    assert np.array_equal(y.cpu().numpy(), yr)
    for s, d in zip(srcs, dsts):
        assert np.array_equal(s.cpu().numpy().view(np.uint32), d.cpu().numpy().view(np.uint32))
    assert np.all(r["bg_done"] > 0)
    assert np.all(r["lat_us"] > 0) and np.all(r["late_us"] < r["lat_us"])


@pytest.mark.parametrize("pinned", [False, True])
def test_isolation_full_size_critical_items_and_256mib_copies_exact(pinned):
    """The isolation workload at its full sizes: a 262,144-element critical item every
    1 ms on XCD 0 (32 slices) while XCDs 1-7 copy private 256 MiB buffers; pinned: the
    critical item's x kept in its members' LDS (each pins its 8,192-element slice)."""
    periods = 100
    say(f"isolation full size: {periods} periods of 1 ms, 7 x 256 MiB copies, pinned={pinned}")
    xh, AB = workloads.isolation(periods=periods)
    x = to_dev(xh)
    y = sentinel_i32(xh.shape)
    elems = workloads.ISO_COPY_ELEMS
    srcs = [workloads.isolation_copy_source_device(c, elems, "cuda") for c in range(1, 8)]
    dsts = [torch.zeros_like(t) for t in srcs]
    torch.cuda.synchronize()
    crit = lk.make_items(lk.OP_AFFINE_SUM_I32, xh.size, addr(x), addr(y), AB[:, 0], AB[:, 1],
                         flags=lk.DF_PIN_INPUT if pinned else 0)
    bg = lk.make_items(lk.OP_COPY_F32, elems, [addr(t) for t in srcs], [addr(d) for d in dsts])
    with lk.Context(n_workers=0, clusters=lk.CLUSTERS_PER_XCD, idle_timeout_ms=30000) as ctx:
        assert ctx.info()["n_clusters"] == 8
        r = ctx.run_isolation(0, crit, 1e-3, list(range(1, 8)), bg)
    for k in range(periods):
        assert r["results"][k] == oracle.affine_sum_i32(xh, int(AB[k, 0]), int(AB[k, 1]))[1], k
    yr, _ = oracle.affine_sum_i32(xh, int(AB[-1, 0]), int(AB[-1, 1]))
    assert np.array_equal(y.cpu().numpy(), yr)
    for t, d in zip(srcs, dsts):
        assert torch.equal(t.view(torch.int32), d.view(torch.int32))
    assert np.all(r["bg_done"] > 0)


# ------------------------------------------------------------------ paper replay protocol
def test_replay_protocol_runs_on_one_cu_and_all_cus():
    say("replay: 3 runs of Init/Trigger/Wait/Dispose vs Alloc/Spawn/Wait/Dispose, SPIN 20000")
    for nw in (1, torch.cuda.get_device_properties(0).multi_processor_count):
        lk_us, hip_us, lk_cy, hip_cy, res = lk.replay(nw, 20000, 3, with_results=True)
        assert np.all(lk_us > 0) and np.all(hip_us > 0)
        assert np.all(lk_cy > 0) and np.all(hip_cy > 0)
        # the loop dominates Wait; Trigger is a few host stores
        assert np.all(lk_us[:, 1] < lk_us[:, 2])
        # the item's result on both paths, summed over the nw workers, is the oracle's
        want = oracle.exec_cluster(oracle.SPIN, nw, n=0, a=20000)
        assert np.all(res == want), res


# ------------------------------------------------------------------ batches
def _burst(count, seed, log2_range=(8, 16)):
    ops, n, ab, alpha = workloads.batching(count, seed=seed, log2_range=log2_range)
    off = np.concatenate([[0], np.cumsum((n + 255) // 256 * 256)])
    rng = np.random.default_rng(seed + 1000)
    total = int(off[-1])
    xi = rng.integers(-2 ** 31, 2 ** 31, total, dtype=np.int64).astype(np.int32)
    xf = rng.standard_normal(total).astype(np.float32)
    yf = rng.standard_normal(total).astype(np.float32)
    return ops, n, ab, alpha, off, xi, xf, yf


def test_batches_of_uneven_items_bit_exact_over_all_cus_and_one_xcd():
    ops, n, ab, alpha, off, xi, xf, yf = _burst(64, 11)
    say(f"batch: 64 uneven items ({int(n.sum())} elements), tiles of 4096, cluster ONE, XCD 0 and "
        "the first half of the workers, 3 reps")
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    half = (np.arange(n_cu) >= n_cu // 2).astype(np.uint32)
    for policy, cluster in ((lk.CLUSTERS_ONE, 0), (lk.CLUSTERS_PER_XCD, 0), (lk.CLUSTERS_EXPLICIT, 0),
                            (lk.CLUSTERS_EXPLICIT, 1)):
        d_xi, d_xf, d_yf = to_dev(xi), to_dev(xf), to_dev(yf.copy())
        d_z = sentinel_i32(xi.shape)
        ins = np.where(ops == lk.OP_AFFINE_SUM_I32, addr(d_xi), addr(d_xf)) + off[:-1].astype(np.uint64) * 4
        outs = np.where(ops == lk.OP_AFFINE_SUM_I32, addr(d_z), addr(d_yf)) + off[:-1].astype(np.uint64) * 4
        items = lk.make_items(ops, n, ins.astype(np.uint64), outs.astype(np.uint64), ab[:, 0], ab[:, 1], alpha)
        tiles, owner = lk.batch_plan(items, 4096)
        d_tiles = torch.from_numpy(tiles.view(np.uint8)).to("cuda")
        partials = torch.zeros(tiles.size, dtype=torch.int64, device="cuda")
        torch.cuda.synchronize()
        kw = dict(n_workers=n_cu, cluster_of_worker=half) if policy == lk.CLUSTERS_EXPLICIT else dict(n_workers=0)
        with lk.Context(clusters=policy, idle_timeout_ms=20000, **kw) as ctx:
            if policy == lk.CLUSTERS_EXPLICIT:
                assert sorted(ctx.members(cluster)) == list(range(cluster * n_cu // 2, (cluster + 1) * n_cu // 2))
            ms = ctx.run_batch(cluster, d_tiles, tiles.size, partials, reps=3)
        assert ms.size == 3 and np.all(ms > 0)
        P = partials.cpu().numpy()
        Z, YF = d_z.cpu().numpy(), d_yf.cpu().numpy()
        for i in range(64):
            lo, hi = int(off[i]), int(off[i]) + int(n[i])
            if ops[i] == lk.OP_AFFINE_SUM_I32:
                yr, sr = oracle.affine_sum_i32(xi[lo:hi].copy(), int(ab[i, 0]), int(ab[i, 1]))
                assert int(P[owner == i].sum()) == sr, (policy, i)
                assert np.array_equal(Z[lo:hi], yr), (policy, i)
            else:
                want = yf[lo:hi].copy()
                for _ in range(3):
                    oracle.saxpy_f32(alpha[i], xf[lo:hi].copy(), want)
                assert np.array_equal(YF[lo:hi].view(np.uint32), want.view(np.uint32)), (policy, i)


def test_batches_in_flight_two_deep_keep_their_own_counters():
    ops, n, ab, alpha, off, xi, xf, yf = _burst(16, 12)
    ops[:] = lk.OP_AFFINE_SUM_I32
    say("batch: two different batches in flight on one cluster (depth 2), 5 rounds")
    d_xi = to_dev(xi)
    d_z1, d_z2 = sentinel_i32(xi.shape), sentinel_i32(xi.shape)
    plans = []
    for d_z, shift in ((d_z1, 0), (d_z2, 1)):
        items = lk.make_items(ops, n, addr(d_xi) + off[:-1].astype(np.uint64) * 4,
                              addr(d_z) + off[:-1].astype(np.uint64) * 4, ab[:, 0].astype(np.int64) + shift, ab[:, 1])
        tiles, owner = lk.batch_plan(items, 1024)
        plans.append((torch.from_numpy(tiles.view(np.uint8)).to("cuda"), tiles.size, owner,
                      torch.zeros(tiles.size, dtype=torch.int64, device="cuda")))
    torch.cuda.synchronize()
    with lk.Context(n_workers=0, clusters=lk.CLUSTERS_ONE, depth=2, idle_timeout_ms=20000) as ctx:
        for _ in range(5):
            t1 = ctx.submit_batch(0, plans[0][0], plans[0][1], plans[0][3])
            t2 = ctx.submit_batch(0, plans[1][0], plans[1][1], plans[1][3])
            assert ctx.wait(0, t1) == plans[0][1]
            assert ctx.wait(0, t2) == plans[1][1]
    for (dt, nt, owner, part), d_z, shift in zip(plans, (d_z1, d_z2), (0, 1)):
        P, Z = part.cpu().numpy(), d_z.cpu().numpy()
        for i in range(16):
            lo, hi = int(off[i]), int(off[i]) + int(n[i])
            yr, sr = oracle.affine_sum_i32(xi[lo:hi].copy(), lk._i32(int(ab[i, 0]) + shift), int(ab[i, 1]))
            assert int(P[owner == i].sum()) == sr and np.array_equal(Z[lo:hi], yr)


@pytest.mark.parametrize("threads", [256, 1024])
def test_batch_full_size_burst_of_4096_exact(threads):
    """The batching workload's largest evaluation burst at its full sizes (4096 items,
    log-uniform 256 .. 2^20 elements, seed 5), one persistent batch over all CUs with
    16,384-element tiles, on workers of both sizes the autotuner chooses from; every item
    checked."""
    ops, n, ab, alpha = workloads.batching(4096, seed=5)
    off = np.concatenate([[0], np.cumsum((n + 255) // 256 * 256)]).astype(np.uint64)
    total = int(off[-1])
    say(f"batch full size: 4096 items, {int(n.sum())} elements, tiles of 16384, {threads}-thread workers")
    rng = np.random.default_rng(1005)
    xi = rng.integers(0, 2 ** 32, total, dtype=np.uint32).view(np.int32)
    xf = rng.standard_normal(total, dtype=np.float32)
    yf = rng.standard_normal(total, dtype=np.float32)
    d_xi, d_xf, d_yf = to_dev(xi), to_dev(xf), to_dev(yf)
    d_z = sentinel_i32((total,))
    ins = np.where(ops == lk.OP_AFFINE_SUM_I32, addr(d_xi), addr(d_xf)).astype(np.uint64) + off[:-1] * 4
    outs = np.where(ops == lk.OP_AFFINE_SUM_I32, addr(d_z), addr(d_yf)).astype(np.uint64) + off[:-1] * 4
    items = lk.make_items(ops, n, ins, outs, ab[:, 0], ab[:, 1], alpha)
    tiles, owner = lk.batch_plan(items, 16384)
    d_tiles = torch.from_numpy(tiles.view(np.uint8)).to("cuda")
    partials = torch.zeros(tiles.size, dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    with lk.Context(n_workers=0, clusters=lk.CLUSTERS_ONE, poll_sleep=8, threads=threads,
                    idle_timeout_ms=30000) as ctx:
        ctx.run_batch(0, d_tiles, tiles.size, partials, reps=1)
    P = partials.cpu().numpy()
    sums = np.bincount(owner, weights=None, minlength=4096)  # tiles per item
    assert int(sums.sum()) == tiles.size
    part_sum = np.zeros(4096, np.int64)
    np.add.at(part_sum, owner, P)
    Z, YF = d_z.cpu().numpy(), d_yf.cpu().numpy()
    for i in range(4096):
        lo, hi = int(off[i]), int(off[i]) + int(n[i])
        if ops[i] == lk.OP_AFFINE_SUM_I32:
            yr, sr = oracle.affine_sum_i32(xi[lo:hi].copy(), int(ab[i, 0]), int(ab[i, 1]))
            assert int(part_sum[i]) == sr, i
            assert np.array_equal(Z[lo:hi], yr), i
        else:
            want = yf[lo:hi].copy()
            oracle.saxpy_f32(alpha[i], xf[lo:hi].copy(), want)
            assert same_f32(YF[lo:hi], want), i


def test_launch_burst_baseline_matches_oracle():
    ops, n, ab, alpha, off, xi, xf, yf = _burst(32, 13)
    say("launch burst: 32 uneven items as per-item launches and as a captured graph")
    for graph in (False, True):
        d_xi, d_xf, d_yf = to_dev(xi), to_dev(xf), to_dev(yf.copy())
        d_z = sentinel_i32(xi.shape)
        ins = np.where(ops == lk.OP_AFFINE_SUM_I32, addr(d_xi), addr(d_xf)) + off[:-1].astype(np.uint64) * 4
        outs = np.where(ops == lk.OP_AFFINE_SUM_I32, addr(d_z), addr(d_yf)) + off[:-1].astype(np.uint64) * 4
        items = lk.make_items(ops, n, ins.astype(np.uint64), outs.astype(np.uint64), ab[:, 0], ab[:, 1], alpha)
        ms = lk.launch_burst(items, elems_per_wg=4096, graph=graph, reps=2)
        assert np.all(ms > 0)
        Z, YF = d_z.cpu().numpy(), d_yf.cpu().numpy()
        for i in range(32):
            lo, hi = int(off[i]), int(off[i]) + int(n[i])
            if ops[i] == lk.OP_AFFINE_SUM_I32:
                assert np.array_equal(Z[lo:hi], oracle.affine_sum_i32(xi[lo:hi].copy(), int(ab[i, 0]), int(ab[i, 1]))[0])
            else:
                want = yf[lo:hi].copy()
                for _ in range(2):
                    oracle.saxpy_f32(alpha[i], xf[lo:hi].copy(), want)
                assert np.array_equal(YF[lo:hi].view(np.uint32), want.view(np.uint32)), (graph, i)


def test_out_of_place_axpy_single_cluster_and_batch():
    rng = np.random.default_rng(17)
    n = 70001
    x = rng.standard_normal(n + 8).astype(np.float32)
    yv = rng.standard_normal(n + 8).astype(np.float32)
    x[:5] = [np.inf, -0.0, 1e-40, np.nan, 3e38]
    say("axpy: out-of-place fma on one worker, on an XCD cluster and inside a batch")
    d_x, d_y = to_dev(x), to_dev(yv)
    outs = [sentinel_f32((n + 8,)) for _ in range(3)]
    torch.cuda.synchronize()
    alpha = np.float32(-1.75)
    with lk.Context(n_workers=0, clusters=lk.CLUSTERS_PER_XCD, idle_timeout_ms=20000) as ctx:
        t = ctx.submit(0, lk.OP_AXPY_F32, x=addr(d_x, 1), y=addr(outs[0], 1), alpha=alpha, n=n, aux=addr(d_y, 1))
        ctx.wait(0, t)
        it = lk.make_items(lk.OP_AXPY_F32, n, addr(d_x, 1), addr(outs[2], 1), alpha=alpha, in2=addr(d_y, 1))[None]
        tiles, owner = lk.batch_plan(it, 4096)
        d_t = torch.from_numpy(tiles.view(np.uint8)).to("cuda")
        part = torch.zeros(tiles.size, dtype=torch.int64, device="cuda")
        torch.cuda.synchronize()
        ctx.run_batch(1, d_t, tiles.size, part, reps=1)
    with lk.Context(n_workers=1, idle_timeout_ms=20000) as ctx:
        t = ctx.submit(0, lk.OP_AXPY_F32, x=addr(d_x, 1), y=addr(outs[1], 1), alpha=alpha, n=n, aux=addr(d_y, 1))
        ctx.wait(0, t)
    want = oracle.axpy_f32(alpha, x[1:n + 1].copy(), yv[1:n + 1].copy())
    for o in outs:
        got = o.cpu().numpy()
        assert same_f32(got[1:n + 1], want)
        assert got[0].view(np.uint32) == SENT_F32_BITS and np.all(got[n + 1:].view(np.uint32) == SENT_F32_BITS)
    assert np.array_equal(d_y.cpu().numpy().view(np.uint32), yv.view(np.uint32))  # y only read


# ------------------------------------------------------------------ serving (continuous batching)
def _serve_setup(count, seed, pool_elems=1 << 20, log2=(8, 16)):
    tr = workloads.serving(1e5, None, pool_elems, seed=seed, log2_range=log2, max_requests=count)
    rng = np.random.default_rng(seed + 1)
    xi = rng.integers(-2 ** 31, 2 ** 31, pool_elems, dtype=np.int64).astype(np.int32)
    xf = rng.standard_normal(pool_elems).astype(np.float32)
    yf = rng.standard_normal(pool_elems).astype(np.float32)
    return tr, xi, xf, yf


def _requests(tr, d_xi, d_xf, d_yf, arrival_us):
    req = np.zeros(tr["n"].size, lk.REQUEST_DTYPE)
    kind = tr["kind"]
    req["arrival_us"] = arrival_us
    req["op"] = np.choose(kind, [lk.OP_AFFINE_SUM_I32, lk.OP_SUM_I32_I64, lk.OP_AXPY_F32])
    req["a"], req["b"], req["alpha"], req["n"] = tr["ab"][:, 0], tr["ab"][:, 1], tr["alpha"], tr["n"]
    req["inp"] = np.where(kind == 2, addr(d_xf), addr(d_xi)).astype(np.uint64) + tr["off_x"] * 4
    req["in2"] = np.where(kind == 2, addr(d_yf) + tr["off_y"].astype(np.int64) * 4, 0).astype(np.uint64)
    return req


def _oracle_request(tr, i, xi, xf, yf):
    n, ox, oy = int(tr["n"][i]), int(tr["off_x"][i]), int(tr["off_y"][i])
    k = int(tr["kind"][i])
    if k == 0:
        return oracle.affine_sum_i32(xi[ox:ox + n].copy(), int(tr["ab"][i, 0]), int(tr["ab"][i, 1]))
    if k == 1:
        return None, oracle.sum_i32_i64(xi[ox:ox + n].copy())
    return oracle.axpy_f32(tr["alpha"][i], xf[ox:ox + n].copy(), yf[oy:oy + n].copy()), 0


def _read_output(arena, outc, i, n, kind):
    base = arena.data_ptr()
    off = (int(outc["out"][i]) - base) // 4
    v = arena[off:off + n].cpu().numpy()
    return v.view(np.float32) if kind == 2 else v


def test_serving_results_identical_alone_and_in_the_mix():
    count = 240
    tr, xi, xf, yf = _serve_setup(count, 21)
    say(f"serving: {count} requests all at once (mix) vs one at a time (alone), retained outputs")
    d_xi, d_xf, d_yf = to_dev(xi), to_dev(xf), to_dev(yf)
    # retained outputs: every shard's slice (arena / threads) must hold all of its requests
    per_req = (tr["n"].astype(np.int64) * 4 + 255) // 256 * 256
    per_shard = max(int(per_req[s::8].sum()) for s in range(8))
    need = 8 * (per_shard + (1 << 16))
    arenas = [torch.zeros(need // 4, dtype=torch.int32, device="cuda") for _ in range(2)]
    torch.cuda.synchronize()
    with lk.Context(n_workers=0, depth=4, idle_timeout_ms=30000) as ctx:
        mix, st_mix = ctx.serve(_requests(tr, d_xi, d_xf, d_yf, np.zeros(count)), arenas[0], need,
                                tile_elems=4096, threads=8, retain=True)
        alone, st_alone = ctx.serve(_requests(tr, d_xi, d_xf, d_yf, np.arange(count) * 400.0), arenas[1], need,
                                    tile_elems=4096, threads=1, retain=True)
    assert np.all(mix["status"] == 0) and np.all(alone["status"] == 0)
    # alone really was alone: requests finished before the next arrived (a host thread
    # preempted for a scheduler timeslice may let one overlap its successor, which does
    # not weaken the comparison below; the bulk must not)
    assert np.mean(alone["done_us"][:-1] < np.arange(1, count) * 400.0) >= 0.9
    assert np.array_equal(mix["result"], alone["result"])
    for i in range(count):
        k, n = int(tr["kind"][i]), int(tr["n"][i])
        yr, sr = _oracle_request(tr, i, xi, xf, yf)
        if k in (0, 1):
            assert mix["result"][i] == sr, i
        if k != 1:
            a = _read_output(arenas[0], mix, i, n, k)
            b = _read_output(arenas[1], alone, i, n, k)
            assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), i
            if k == 0:
                assert np.array_equal(a, yr), i
            else:
                assert same_f32(a, yr), i
    assert st_mix["tiles"] == st_alone["tiles"] == int(mix["tiles"].sum())


def test_serving_admission_waits_for_memory_budget():
    count = 400
    tr, xi, xf, yf = _serve_setup(count, 22)
    say(f"serving: {count} requests through a 2 MiB output budget (admission waits for memory)")
    d_xi, d_xf, d_yf = to_dev(xi), to_dev(xf), to_dev(yf)
    budget = 2 << 20
    arena = torch.zeros(budget // 4, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    with lk.Context(n_workers=0, depth=2, idle_timeout_ms=30000) as ctx:
        outc, st = ctx.serve(_requests(tr, d_xi, d_xf, d_yf, np.zeros(count)), arena, budget,
                             tile_elems=8192, threads=2, retain=False)
    assert np.all(outc["status"] == 0)
    assert st["deferred"] > 0 and st["peak_bytes"] <= budget
    assert np.all(outc["admit_us"] <= outc["done_us"])
    for i in range(count):
        if int(tr["kind"][i]) in (0, 1):
            assert outc["result"][i] == _oracle_request(tr, i, xi, xf, yf)[1], i


@pytest.mark.parametrize("threads,schedulers", [(256, 8), (1024, 4)])
def test_serving_full_size_requests_exact(threads, schedulers):
    """Serving with the workload's full request sizes (log-uniform 256 .. 2^22 elements,
    windows in resident pools of 2^26 elements), Poisson arrivals, tiles of 65,536, depth
    4, with the bench's workers and schedulers (1024 threads, 4 schedulers) and a second
    shape; every result and every retained output checked."""
    count = 300
    tr, xi, xf, yf = _serve_setup(count, 23, pool_elems=1 << 26, log2=(8, 22))
    say(f"serving full size: {count} requests, n up to 2^22, {int(tr['n'].sum())} elements, "
        f"{threads}-thread workers, {schedulers} schedulers")
    d_xi, d_xf, d_yf = to_dev(xi), to_dev(xf), to_dev(yf)
    per_req = (tr["n"].astype(np.int64) * 4 + 255) // 256 * 256
    per_shard = max(int(per_req[s::schedulers].sum()) for s in range(schedulers))
    need = schedulers * (per_shard + (1 << 16))
    arena = torch.zeros(need // 4, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    with lk.Context(n_workers=0, depth=4, threads=threads, idle_timeout_ms=30000) as ctx:
        outc, st = ctx.serve(_requests(tr, d_xi, d_xf, d_yf, tr["arrival_us"]), arena, need,
                             tile_elems=65536, threads=schedulers, retain=True)
    assert np.all(outc["status"] == 0) and st["tiles"] == int(outc["tiles"].sum())
    for i in range(count):
        k, n = int(tr["kind"][i]), int(tr["n"][i])
        yr, sr = _oracle_request(tr, i, xi, xf, yf)
        if k in (0, 1):
            assert outc["result"][i] == sr, i
        if k == 0:
            assert np.array_equal(_read_output(arena, outc, i, n, k), yr), i
        elif k == 2:
            assert same_f32(_read_output(arena, outc, i, n, k), yr), i


def test_second_context_that_cannot_fit_is_refused_at_once():
    say("two contexts: the second one asking for every CU is refused without booting")
    with lk.Context(n_workers=0, idle_timeout_ms=10000) as ctx:
        t0 = time.time()
        with pytest.raises(lk.LKError) as e:
            lk.Context(n_workers=0)
        assert e.value.code == lk.ENODEV and time.time() - t0 < 1.0
        t = ctx.submit(0, lk.OP_NOP)
        ctx.wait(0, t)
    with lk.Context(n_workers=8) as a, lk.Context(n_workers=8) as b:   # room for both
        for c in (a, b):
            c.wait(0, c.submit(0, lk.OP_NOP))
