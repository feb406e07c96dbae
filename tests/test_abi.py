"""Host-side checks of the C-ABI library that need no GPU: it loads, it exports every
symbol include/*.h declares, the Python structs match the C layouts, the wire codes are
the paper's Table 1 values, argument validation happens before any device call, and the
host slicing rule agrees with the oracle's."""
import ctypes
import json
import os
import re
import subprocess

import numpy as np
import pytest

import oracle
from paper_2310_01212_amd import lk

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
INCLUDE = os.path.join(ROOT, "include")
WIRE = os.path.join(ROOT, "paper_2310_01212_amd", "csrc", "lk_wire.h")


def _declared():
    names = []
    for h in sorted(os.listdir(INCLUDE)):
        if h.endswith(".h"):
            text = open(os.path.join(INCLUDE, h)).read()
            names += re.findall(r"^LK_API\s+[\w\s\*]+?\b(lk[bs]?_\w+)\s*\(", text, re.M)
    return names


def test_library_exports_every_declared_symbol():
    L = lk.lib()
    declared = _declared()
    assert len(declared) >= 20
    for name in declared:
        assert hasattr(L, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", lk.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (lk[bs]?_\w+)", out))
    assert set(declared) == exported
    assert set(lk.EXPORTED) == exported


def test_struct_layouts_match_the_c_headers(tmp_path):
    src = tmp_path / "sizes.c"
    src.write_text('#include "lk.h"\n#include "lk_bench.h"\n#include <stdio.h>\n#include <stddef.h>\n'
                   'int main(void){printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(lk_desc),'
                   ' sizeof(lk_config), sizeof(lk_completion), sizeof(lk_info), sizeof(lk_log_entry), sizeof(lkb_item),'
                   ' offsetof(lk_config, init_timeout_ns), offsetof(lk_desc, aux), sizeof(lk_tile),'
                   ' offsetof(lk_config, workers_per_cu), offsetof(lk_info, workers_per_cu),'
                   ' offsetof(lk_config, first_poll_delay), offsetof(lk_config, xcd_mask),'
                   ' offsetof(lk_info, xcd_mask)); return 0;}\n')
    exe = tmp_path / "sizes"
    subprocess.check_call(["gcc", "-std=c11", "-I", INCLUDE, "-o", str(exe), str(src)])
    got = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    want = [ctypes.sizeof(lk.Desc), ctypes.sizeof(lk.Config), ctypes.sizeof(lk.Completion),
            ctypes.sizeof(lk.Info), ctypes.sizeof(lk.LogEntry), lk.ITEM_DTYPE.itemsize,
            lk.Config.init_timeout_ns.offset, lk.Desc.aux.offset, lk.TILE_DTYPE.itemsize,
            lk.Config.workers_per_cu.offset, lk.Info.workers_per_cu.offset, lk.Config.first_poll_delay.offset,
            lk.Config.xcd_mask.offset, lk.Info.xcd_mask.offset]
    assert got == want
    assert lk.LOG_DTYPE.itemsize == ctypes.sizeof(lk.LogEntry)
    assert lk.COMPLETION_DTYPE.itemsize == ctypes.sizeof(lk.Completion)
    # the serving structures (lk_serve.h)
    src2 = tmp_path / "serve_sizes.c"
    src2.write_text('#include "lk_serve.h"\n#include <stdio.h>\n#include <stddef.h>\n'
                    'int main(void){printf("%zu %zu %zu %zu %zu %zu\\n", sizeof(lks_request), sizeof(lks_config),'
                    ' sizeof(lks_outcome), sizeof(lks_stats), offsetof(lks_stats, posted), offsetof(lks_stats, drained));'
                    ' return 0;}\n')
    exe2 = tmp_path / "serve_sizes"
    subprocess.check_call(["gcc", "-std=c11", "-I", INCLUDE, "-o", str(exe2), str(src2)])
    got2 = [int(v) for v in subprocess.check_output([str(exe2)]).split()]
    assert got2 == [lk.REQUEST_DTYPE.itemsize, ctypes.sizeof(lk.ServeConfig), lk.OUTCOME_DTYPE.itemsize,
                    ctypes.sizeof(lk.ServeStats), lk.ServeStats.posted.offset, lk.ServeStats.drained.offset]


def _wire_defines():
    d = {}
    for m in re.finditer(r"#define\s+(LKW_\w+)\s+(\d+)u", open(WIRE).read()):
        d[m.group(1)] = int(m.group(2))
    return d


def test_wire_codes_are_table1():
    golden = {}
    for line in open(os.path.join(ROOT, "tests", "golden", "table1_mailbox_codes.txt")):
        if line.strip() and not line.startswith("#"):
            direction, name, v = line.split()
            golden[(direction, name)] = int(v)
    d = _wire_defines()
    assert d["LKW_FROM_INIT"] == golden[("from_GPU", "THREAD_INIT")]
    assert d["LKW_FROM_FINISHED"] == golden[("from_GPU", "THREAD_FINISHED")]
    assert d["LKW_FROM_WORKING"] == golden[("from_GPU", "THREAD_WORKING")]
    assert d["LKW_FROM_NOP"] == golden[("from_GPU", "THREAD_NOP")]
    assert d["LKW_TO_NOP"] == golden[("to_GPU", "THREAD_NOP")]
    assert d["LKW_TO_EXIT"] == golden[("to_GPU", "THREAD_EXIT")]
    assert d["LKW_TO_WORK"] == golden[("to_GPU", "THREAD_WORK")]
    # extension codes use values Table 1 leaves free
    ext = {d["LKW_FROM_ERROR"], d["LKW_FROM_EXITED"], d["LKW_FROM_TIMEDOUT"]}
    assert not ext & {0, 1, 2, 4} and len(ext) == 3
    assert lk.CODE_NOP == d["LKW_TO_NOP"] and lk.CODE_EXIT == d["LKW_TO_EXIT"] and lk.CODE_WORK == d["LKW_TO_WORK"]


def test_host_slicing_agrees_with_oracle():
    oracle.build(force=False)
    for n in [0, 1, 255, 256, 257, 4096, 8191, 262144, 262144 + 77, 16384, 10 ** 6 + 3]:
        for k in [1, 2, 3, 7, 8, 32, 256]:
            for j in range(k):
                assert lk.slice_bounds(n, k, j) == oracle.slice_bounds(n, k, j), (n, k, j)
    with pytest.raises(lk.LKError):
        lk.slice_bounds(10, 0, 0)


def test_strerror_names_every_code():
    names = {c: lk.strerror(c) for c in range(-7, 1)}
    assert len(set(names.values())) == 8
    assert lk.strerror(-99) == "unknown error"


def _cfg(**kw):
    cfg = lk.Config()
    lk.lib().lk_config_default(ctypes.byref(cfg))
    for k, v in kw.items():
        setattr(cfg, k, v)
    return cfg


@pytest.mark.parametrize("field,value", [
    ("threads_per_worker", 100), ("threads_per_worker", 2048), ("queue_depth", 65),
    ("cluster_policy", 9), ("poll_sleep", 200), ("idle_timeout_ms", 3600001),
    ("flags", 0x80), ("n_workers", 5000), ("init_timeout_ns", -1), ("workers_per_cu", 5),
    ("first_poll_delay", -2), ("first_poll_delay", 128),
])
def test_init_rejects_bad_config_before_touching_a_device(field, value):
    L = lk.lib()
    h = ctypes.c_void_p()
    rc = L.lk_init(ctypes.byref(_cfg(**{field: value})), ctypes.byref(h))
    assert rc == lk.EINVAL, (field, rc, lk.last_error())
    assert not h


def test_workers_per_cu_must_leave_every_worker_resident():
    L = lk.lib()
    h = ctypes.c_void_p()
    for wpc, t in ((2, 1024), (4, 512), (3, 384)):
        assert L.lk_init(ctypes.byref(_cfg(workers_per_cu=wpc, threads_per_worker=t)), ctypes.byref(h)) == lk.EINVAL
        assert "resident" in lk.last_error() and not h
    cfg = lk.Config()
    L.lk_config_default(ctypes.byref(cfg))
    assert cfg.workers_per_cu == 1 and cfg.first_poll_delay == lk.POLL_DELAY_ADAPTIVE


def test_explicit_clusters_are_validated():
    L = lk.lib()
    h = ctypes.c_void_p()
    cow = (ctypes.c_uint32 * 4)(0, 0, 2, 2)   # cluster 1 empty
    cfg = _cfg(cluster_policy=lk.CLUSTERS_EXPLICIT, n_clusters=3, n_workers=4,
               cluster_of_worker=ctypes.cast(cow, ctypes.POINTER(ctypes.c_uint32)))
    assert L.lk_init(ctypes.byref(cfg), ctypes.byref(h)) == lk.EINVAL
    assert "no worker" in lk.last_error()
    cow2 = (ctypes.c_uint32 * 2)(0, 3)
    cfg = _cfg(cluster_policy=lk.CLUSTERS_EXPLICIT, n_clusters=2, n_workers=2,
               cluster_of_worker=ctypes.cast(cow2, ctypes.POINTER(ctypes.c_uint32)))
    assert L.lk_init(ctypes.byref(cfg), ctypes.byref(h)) == lk.EINVAL


def test_calls_on_a_null_context_fail_cleanly():
    L = lk.lib()
    d = lk.Desc()
    t = ctypes.c_uint64()
    r = ctypes.c_int64()
    assert L.lk_submit(None, 0, ctypes.byref(d), None, None, ctypes.byref(t)) == lk.EINVAL
    assert L.lk_wait(None, 0, 1, 0, ctypes.byref(r)) == lk.EINVAL
    assert L.lk_dispose(None) == lk.EINVAL
    assert L.lk_prefetch(None, 0, 0) == lk.EINVAL
    assert L.lk_free(None) == lk.OK
    assert L.lk_init(None, None) == lk.EINVAL


def test_static_launch_entry_point_rejects_bad_sizes_before_touching_a_device():
    """The allocation-free per-launch entry point refuses k outside its static array
    (1..4096) and a misaligned item before any HIP call; the detail reaches lk_last_error
    (the runners share the library's per-thread error detail)."""
    it = lk.make_items(lk.OP_SUM_I32_I64, 16, 0x1000, 0)
    for k in (0, 4097):
        with pytest.raises(lk.LKError) as e:
            lk.launch_serial_static(it, k=k)
        assert e.value.code == lk.EINVAL
        assert "1..4096" in lk.last_error() and "1..4096" in str(e.value)
    bad = lk.make_items(lk.OP_SUM_I32_I64, 16, 0x1002, 0)
    with pytest.raises(lk.LKError) as e:
        lk.launch_serial_static(bad, k=1)
    assert e.value.code == lk.EINVAL and "invalid" in lk.last_error()


def test_init_without_a_gpu_reports_no_device():
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(lk.LKError) as e:
        lk.Context()
    assert e.value.code == lk.ENODEV


def test_make_items_marshals_int32_and_addresses():
    it = lk.make_items(lk.OP_AFFINE_SUM_I32, 4096, [0x1000, 0x2000], [0x3000, 0x4000],
                       a=np.array([2 ** 32 - 1, 5], dtype=np.uint32), b=-7, alpha=0.5)
    assert it.shape == (2,)
    assert it["a"].tolist() == [-1, 5] and it["b"].tolist() == [-7, -7]
    assert it["inp"].tolist() == [0x1000, 0x2000] and it["out"].tolist() == [0x3000, 0x4000]
    assert lk._i32(2 ** 31) == -2 ** 31 and lk._i32(-1) == -1


def test_submit_rejects_n_beyond_the_tensors_extent():
    """Context.submit passes bare addresses to lk_submit, which cannot see a buffer's end;
    the binding checks n against every tensor it was given before anything is posted."""
    torch = pytest.importorskip("torch")
    xi = torch.zeros(100, dtype=torch.int32)
    xf = torch.zeros(100, dtype=torch.float32)
    short_f = torch.zeros(60, dtype=torch.float32)
    # defaults and in-range counts
    assert lk.submit_extent(lk.OP_SAXPY_F32, None, xf, xf) == 100
    assert lk.submit_extent(lk.OP_SUM_I32_I64, None, xi) == 100
    assert lk.submit_extent(lk.OP_SAXPY_F32, 60, xf, short_f) == 60
    assert lk.submit_extent(lk.OP_AXPY_F32, 60, xf, short_f, aux=short_f) == 60
    assert lk.submit_extent(lk.OP_NOP, 0) == 0
    assert lk.submit_extent(lk.OP_SAXPY_F32, 10 ** 9, 0x1000, 0x2000) == 10 ** 9  # bare addresses
    # n past x, past y, past AXPY's y (aux)
    with pytest.raises(ValueError, match="x's"):
        lk.submit_extent(lk.OP_AFFINE_SUM_I32, 101, xi, torch.zeros(200, dtype=torch.int32))
    with pytest.raises(ValueError, match="y's"):
        lk.submit_extent(lk.OP_SAXPY_F32, 100, xf, short_f)
    with pytest.raises(ValueError, match="y's"):
        lk.submit_extent(lk.OP_COPY_F32, None, xf, short_f)
    with pytest.raises(ValueError, match="aux"):
        lk.submit_extent(lk.OP_AXPY_F32, 100, xf, xf, aux=short_f)
    with pytest.raises(ValueError, match="float32"):
        lk.submit_extent(lk.OP_AXPY_F32, 10, xf, xf, aux=xi)
    # per-member int64 results: one per member of the cluster
    res = torch.zeros(4, dtype=torch.int64)
    assert lk.submit_extent(lk.OP_AFFINE_SUM_I32, 100, xi, xi, aux=res, members=4) == 100
    with pytest.raises(ValueError, match="members"):
        lk.submit_extent(lk.OP_SUM_I32_I64, 100, xi, aux=res, members=8)
    with pytest.raises(ValueError, match="int64"):
        lk.submit_extent(lk.OP_SUM_I32_I64, 100, xi, aux=xi, members=1)
    with pytest.raises(ValueError):
        lk.submit_extent(lk.OP_SUM_I32_I64, -1, xi)


def test_bench_quotes_the_paper_tables_as_printed():
    import bench
    golden = {}
    for line in open(os.path.join(ROOT, "tests", "golden", "paper_phase_cycles.txt")):
        if line.strip() and not line.startswith("#"):
            table, scope, system, phase, cycles = line.split()
            golden[(table, scope, system, phase)] = float(cycles)
    seen = 0
    for (kind, scope, system), phases in bench.PAPER_CYCLES.items():
        table = "table2" if kind == "avg" else "table3"
        sc = "single_sm" if scope == "single" else "full_gpu"
        for phase, v in phases.items():
            assert golden[(table, sc, system, phase)] == v
            seen += 1
    assert seen == len(golden) == 24


def test_committed_traffic_profiles_are_used_only_while_they_match_the_worker():
    """bench.py quotes the memory traffic of a committed counter summary (FETCH_SIZE and
    WRITE_SIZE passes) only while the worker's sources hash to the digest recorded in it;
    a summary taken with another worker gives no traffic figure (null).  A current summary
    of the all-CU SAXPY workload (n = 16,384, 1024 threads) lies between the y-only bytes
    (8n) and the algorithmic 12n plus the mailbox records."""
    import json
    import bench
    digest = bench.worker_source_digest()
    seen = 0
    for path in bench.TRAFFIC_FILES:
        if not os.path.exists(path):
            continue
        m = re.search(r"```json\n(.*?)\n```", open(path).read(), re.S)
        assert m, f"{path}: no json block"
        d = json.loads(m.group(1))
        seen += 1
        tr = bench.traffic_per_item(d["n"], d.get("threads_per_worker", 256), d.get("pin_input", False),
                                    d.get("queue_depth", 1), d.get("cold_pairs", 0))
        if d.get("worker_source_digest") != digest:
            assert tr is None or tr["source"] != os.path.relpath(path, ROOT), path
            continue
        assert tr is not None and d["n"] == 16384
        hi = 12.1 if d.get("cold_pairs", 0) else 12.0
        assert 8 * 16384 <= tr["bytes_per_item"] <= hi * 16384, path
    assert seen > 0


def test_lanes_outputs_are_zeroed_contiguous_arrays_of_the_runner_layout():
    res, lat, info = lk.lanes_outputs(3, 5, with_info=True)
    assert res.shape == lat.shape == info.shape == (3, 5)
    assert res.dtype == np.int64 and lat.dtype == np.float64 and info.dtype == lk.COMPLETION_DTYPE
    assert all(a.flags.c_contiguous for a in (res, lat, info))
    assert not res.any() and not lat.any() and not info.view(np.uint8).any()
    assert lk.lanes_outputs(2, 2)[2] is None


def test_bench_roofline_arithmetic():
    """The bench's bound and roofline objects: GB/s from bytes and milliseconds, the
    depth-1 latency bound (round trip + item per mailbox) and its depth > 1 form (the item
    alone), and an HBM roofline against the 8 TB/s peak and a measured copy."""
    import bench
    assert bench.gb_per_s(8e9, 1000.0) == 8.0 and bench.gb_per_s(1e9, 0.0) == 0.0
    floor, bound = bench.latency_bound(256, 2.0, 3.0, 1)
    assert floor == 5.0 and abs(bound - 256 / 5e-6) < 1e-3
    floor4, bound4 = bench.latency_bound(256, 2.0, 3.0, 4)
    assert floor4 == 3.0 and abs(bound4 - 256 / 3e-6) < 1e-3
    r = bench.hbm_roofline(8e9, 1.0, copy_gbps=6000.0, traffic=123, kernel="k")
    assert (r["bound"], r["achieved"], r["peak"], r["unit"], r["frac"]) == ("hbm", 8000.0, 8000.0, "GB/s", 1.0)
    assert r["traffic"] == 123 and r["kernel"] == "k" and r["frac_of_copy_probe"] == round(8000 / 6000, 4)
    assert r["kernel_ms"] == 1.0
    assert "copy_probe_gbps" not in bench.hbm_roofline(1e9, 1.0)
    # the committed kernel trace of the benchmark command: the byte rate it states for the
    # headline dispatch follows from its 6,400,000 items of 196,608 bytes and the traced
    # duration, and that duration agrees with the same run's kernel_ms (device clock)
    text = open(os.path.join(ROOT, "profiles", "lk_worker_allcu_saxpy_kernel_trace.md")).read()
    m = re.search(r"took \*\*([0-9.]+) ms\*\* in the trace", text)
    rate = re.search(r"algorithmic bytes over ([0-9.]+) ms = ([0-9.]+) TB/s", text)
    kms = re.search(r"`kernel_ms` = ([0-9.]+) ms", text)
    assert m and rate and kms and float(rate.group(1)) == float(m.group(1))
    assert abs(bench.gb_per_s(6_400_000 * 196_608, float(m.group(1))) / 1000 - float(rate.group(2))) < 0.006
    assert abs(float(kms.group(1)) / float(m.group(1)) - 1) < 0.01


def test_bench_percentiles_are_nearest_rank():
    import bench
    v = np.arange(1, 101, dtype=np.float64)[::-1]  # order must not matter
    s = bench.lat_summary(v)
    assert (s["p50"], s["p99"], s["p999"], s["max"], s["jitter"]) == (50.0, 99.0, 100.0, 100.0, 99.0)
    w = np.arange(1, 1001, dtype=np.float64)
    assert bench.pct(w, 0.999) == 999.0 and bench.pct(w, 0.5) == 500.0 and bench.pct(w, 0.0) == 1.0
    assert bench.lat_summary([7.0]) == {"p50": 7.0, "p99": 7.0, "p999": 7.0, "max": 7.0, "jitter": 0.0, "mean": 7.0}
    assert s["mean"] == 50.5


def test_worker_digest_ignores_comments_but_not_code(tmp_path):
    import shutil
    import bench
    src = os.path.join(ROOT, "paper_2310_01212_amd", "csrc")
    for f in bench.WORKER_SOURCES:
        shutil.copy(os.path.join(src, f), tmp_path / f)
    base = bench.worker_source_digest(str(tmp_path))
    assert base == bench.worker_source_digest()
    w = tmp_path / "lk_worker.hip"
    text = w.read_text()
    w.write_text("// a new comment line\n/* and a block\n comment */\n" + text.replace("\n", "\n\n", 3))
    assert bench.worker_source_digest(str(tmp_path)) == base
    w.write_text(text.replace("uint32_t pre = 8;", "uint32_t pre = 9;"))
    assert bench.worker_source_digest(str(tmp_path)) != base


def test_make_items_carries_descriptor_flags():
    it = lk.make_items(lk.OP_SAXPY_F32, 64, [0x1000, 0x2000], 0x3000, alpha=1.0, flags=[lk.DF_PIN_INPUT, 0])
    assert it["flags"].tolist() == [lk.DF_PIN_INPUT, 0] and it["reserved"].tolist() == [0, 0]
    with pytest.raises(lk.LKError):
        lk.batch_plan(it, 4096)  # tiles take no descriptor flags


def test_batch_plan_cuts_items_into_tiles():
    items = lk.make_items(np.array([lk.OP_AFFINE_SUM_I32, lk.OP_SAXPY_F32, lk.OP_COPY_F32, lk.OP_NOP]),
                          np.array([1000, 256, 513, 0], np.uint64), np.array([0x1000, 0x8000, 0x20000, 0]),
                          np.array([0x4000, 0x9000, 0x40000, 0]), a=np.array([3, 0, 0, 0]),
                          b=np.array([-5, 0, 0, 0]), alpha=np.array([0, 1.5, 0, 0], np.float32))
    tiles, owner = lk.batch_plan(items, 256)
    assert owner.tolist() == [0, 0, 0, 0, 1, 2, 2, 2, 3]
    assert tiles["n"].tolist() == [256, 256, 256, 232, 256, 256, 256, 1, 0]
    assert tiles["inp"][:4].tolist() == [0x1000 + 256 * 4 * k for k in range(4)]
    assert tiles["out"][:4].tolist() == [0x4000 + 256 * 4 * k for k in range(4)]
    assert tiles["a"][0] == 3 and tiles["b"][0] == np.uint32(np.int32(-5).view(np.uint32))
    assert tiles["b"][4] == np.float32(1.5).view(np.uint32)
    for i, it in enumerate(items):
        assert tiles["n"][owner == i].sum() == it["n"]
    with pytest.raises(lk.LKError):
        lk.batch_plan(items, 100)   # not a multiple of 256
    assert lk.TILE_DTYPE.itemsize == 48
    ax = lk.make_items(lk.OP_AXPY_F32, 600, 0x1000, 0x2000, alpha=np.float32(2.0), in2=0x3000)[None]
    t2, o2 = lk.batch_plan(ax, 256)
    assert t2["in2"].tolist() == [0x3000, 0x3000 + 1024, 0x3000 + 2048] and t2["n"].tolist() == [256, 256, 88]
    assert t2["b"][0] == np.float32(2.0).view(np.uint32)


def test_autotuner_picks_the_fastest_median_with_stable_ties(tmp_path):
    from paper_2310_01212_amd import autotune
    A0, A8, B8, X0 = (0, 256, "all"), (8, 256, "all"), (8, 1024, "all"), (0, 256, "xcd")
    t = {(4096, A0): [10, 11, 50], (16384, A0): [9, 12, 12], (65536, A8): [11, 11, 11],
         (65536, A0): [30, 30, 30], (65536, B8): [11, 12, 12]}
    assert autotune.pick_best(t) == (65536, A8)   # medians 11 tie; larger tile wins
    t2 = {(4096, A0): [5.0], (16384, A0): [5.0], (16384, A8): [5.0], (16384, B8): [5.0], (16384, (8, 256, "xcd")): [5.0]}
    assert autotune.pick_best(t2) == (16384, A8)   # tie: larger tile, longer sleep, smaller worker, wider span
    assert autotune.pick_best({(4096, A0): [6.0], (4096, X0): [5.0]}) == (4096, X0)
    assert len(autotune.contexts()) == 12 and autotune.contexts()[0] == (0, 256, "all")
    assert autotune.pick_best({(4096, X0): [5.0], (4096, (0, 256, "half")): [5.0]})[1][2] == "half"
    calls = []

    def fake(size, tile, cs, reps):
        sleep, threads, span = cs
        calls.append((size, tile, cs))
        cost = abs(tile - 16384 * size) / 1e3 + sleep + 1
        cost += 0.5 if (threads == 1024) == (size == 1) else 0      # 1024 threads for size 4
        cost += 0.25 if (span == "xcd") != (size == 1) else 0       # one XCD for size 1
        return [cost] * reps
    table = autotune.tune(fake, [1, 4], tiles=(4096, 16384, 65536), reps=2)
    assert (table[1]["tile"], table[1]["poll_sleep"], table[1]["threads"], table[1]["span"]) == (16384, 0, 256, "xcd")
    assert (table[4]["tile"], table[4]["threads"], table[4]["span"]) == (65536, 1024, "all")
    assert len(calls) == 2 * 3 * 12
    # one context per setting: the outer loop changes least often
    settings = [c[2] for c in calls]
    assert all(settings[i] == settings[i // 6 * 6] for i in range(len(settings)))
    # a saved table reloads for the same device only; older tables: 256 threads, every CU
    path = str(tmp_path / "t.json")
    autotune.save(table, path, "gfx950")
    assert autotune.load(path, "other") is None
    assert autotune.load(path, "gfx950")[1]["span"] == "xcd" and autotune.load(path, "gfx950")[4]["threads"] == 1024
    json.dump({"device": "gfx950", "table": {"1": {"tile": 4096, "poll_sleep": 0}}}, open(path, "w"))
    assert autotune.load(path, "gfx950")[1] == {"threads": 256, "span": "all", "tile": 4096, "poll_sleep": 0}


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_serving_arena_best_fit_allocator(tmp_path, seed):
    """The serving loop's output allocator (csrc/lk_arena.hpp), driven by a randomised
    C++ check: no overlap, 256-byte alignment, exact accounting, full coalescing, best
    fit, and failure only when no free block is large enough."""
    exe = tmp_path / "arena_check"
    subprocess.run(["g++", "-O2", "-std=c++17", "-Wall", "-Werror",
                    "-I", os.path.join(ROOT, "paper_2310_01212_amd", "csrc"),
                    os.path.join(ROOT, "tests", "cpp", "arena_check.cpp"), "-o", str(exe)], check=True)
    r = subprocess.run([str(exe), str(seed)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip() == "OK", r.stderr
