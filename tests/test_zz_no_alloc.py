"""GPU test of the allocation-free per-launch entry point (lkb_launch_serial_static).

Its outputs are compared with those of the entry point it is a form of
(lkb_launch_serial, stream-synchronised completion) and with the oracle, on two calls in
a row, the second with a smaller input (fewer items, shorter items and fewer workgroups,
so that entries of the static partial-result array left by the first call are not
re-read by the second).
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2310_01212_amd import lk

pytestmark = pytest.mark.gpu

SENT_I32 = 0x7FBADBAD


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


def _case(seed, count, n, ops):
    """count items of n elements, op per item from `ops` in turn, over one int32 x per
    item (affine / sum) and one fp32 (x, y) pair shared by the SAXPY items (a FIFO chain)."""
    rng = np.random.default_rng(seed)
    xi = rng.integers(0, 2**32, (count, n), dtype=np.uint32).view(np.int32)
    ab = rng.integers(0, 2**32, (count, 2), dtype=np.uint32).view(np.int32)
    xf = rng.standard_normal(n).astype(np.float32)
    yf = rng.standard_normal(n).astype(np.float32)
    alpha = rng.uniform(-2, 2, count).astype(np.float32)
    op = np.array([ops[i % len(ops)] for i in range(count)], np.uint32)
    return xi, ab, xf, yf, alpha, op


def _run(entry, case, k, threads):
    xi, ab, xf, yf, alpha, op = case
    count, n = xi.shape
    dxi = torch.from_numpy(xi).cuda()
    dyi = torch.full((count, n), SENT_I32, dtype=torch.int32, device="cuda")
    dxf = torch.from_numpy(xf).cuda()
    dyf = torch.from_numpy(yf.copy()).cuda()
    torch.cuda.synchronize()
    rows = np.arange(count, dtype=np.uint64)
    saxpy = op == lk.OP_SAXPY_F32
    ins = np.where(saxpy, dxf.data_ptr(), dxi.data_ptr() + rows * n * 4).astype(np.uint64)
    outs = np.where(saxpy, dyf.data_ptr(), dyi.data_ptr() + rows * n * 4).astype(np.uint64)
    items = lk.make_items(op, n, ins, outs, ab[:, 0], ab[:, 1], alpha)
    if entry == "static":
        res, lat, _ = lk.launch_serial_static(items, k=k, threads=threads)
    else:
        res, lat, _ = lk.launch_serial(items, k=k, threads=threads, mode=lk.COMPLETE_SYNC)
    torch.cuda.synchronize()
    assert np.all(lat > 0)
    return res, dyi.cpu().numpy(), dyf.cpu().numpy()


def _oracle(case, k):
    xi, ab, xf, yf, alpha, op = case
    count, n = xi.shape
    yi = np.full((count, n), SENT_I32, np.int32)
    yr = yf.copy()
    res = np.zeros(count, np.int64)
    for i in range(count):
        o = int(op[i])
        if o == lk.OP_SAXPY_F32:
            res[i] = oracle.exec_cluster(oracle.SAXPY_F32, k, inp=xf, out=yr, alpha=alpha[i])
        elif o == lk.OP_AFFINE_SUM_I32:
            res[i] = oracle.exec_cluster(oracle.AFFINE_SUM_I32, k, inp=xi[i], out=yi[i], a=int(ab[i, 0]),
                                         b=int(ab[i, 1]))
        else:
            res[i] = oracle.exec_cluster(oracle.SUM_I32_I64, k, inp=xi[i], n=n)
    return res, yi, yr


@pytest.mark.parametrize("first,second", [
    # (seed, items, n, k, threads): the second call is smaller in every dimension
    ((11, 12, 70001, 64, 256), (12, 5, 4099, 3, 256)),
    ((13, 8, 1 << 20, 4096, 64), (14, 3, 513, 1, 1024)),
])
def test_static_entry_point_matches_the_allocating_one_on_two_calls(first, second):
    ops = [lk.OP_AFFINE_SUM_I32, lk.OP_SAXPY_F32, lk.OP_SUM_I32_I64]
    for seed, count, n, k, threads in (first, second):
        say(f"lkb_launch_serial_static vs lkb_launch_serial: seed {seed}, {count} items of {n}, k {k}, "
            f"{threads} threads")
        case = _case(seed, count, n, ops)
        rs, yis, yfs = _run("static", case, k, threads)
        ra, yia, yfa = _run("alloc", case, k, threads)
        assert rs.tolist() == ra.tolist()
        assert np.array_equal(yis, yia)
        assert np.array_equal(yfs.view(np.uint32), yfa.view(np.uint32))
        ro, yio, yfo = _oracle(case, k)
        assert rs.tolist() == ro.tolist()
        assert np.array_equal(yis, yio)
        assert np.array_equal(yfs.view(np.uint32), yfo.view(np.uint32))


def test_static_entry_point_rejects_sizes_beyond_its_array():
    say("lkb_launch_serial_static: k = 0 and k = 4097 refused before any launch")
    x = torch.zeros(16, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    items = lk.make_items(lk.OP_SUM_I32_I64, 16, x.data_ptr(), 0)
    for k in (0, 4097):
        with pytest.raises(lk.LKError) as ei:
            lk.launch_serial_static(items, k=k)
        assert ei.value.code == lk.EINVAL
        assert "4096" in str(ei.value)
