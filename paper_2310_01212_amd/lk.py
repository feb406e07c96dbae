"""ctypes binding of liblk.so (include/lk.h, include/lk_bench.h).

Argument marshalling only: every step of the dispatch path runs in the native library and
its gfx950 kernels.  PyTorch tensors provide device memory (their data_ptr() is passed as
a plain device address).  If the library is missing this module raises; there is no
fallback path.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblk.so")

OK, EINVAL, EAGAIN, ETIMEDOUT, ESTATE, ENODEV, EHIP, EFAULT = 0, -1, -2, -3, -4, -5, -6, -7
OP_NOP, OP_AFFINE_SUM_I32, OP_SUM_I32_I64, OP_SAXPY_F32, OP_COPY_F32, OP_SPIN, OP_BATCH, OP_AXPY_F32 = range(8)
CLUSTERS_PER_WORKER, CLUSTERS_PER_XCD, CLUSTERS_ONE, CLUSTERS_EXPLICIT = range(4)
F_REPORT_WORKING, F_NO_ACQUIRE, F_ANY_PLACEMENT, F_NO_LOOKAHEAD = 1, 2, 4, 8
POLL_DELAY_ADAPTIVE = -1
DF_PIN_INPUT, DF_PIN_RELOAD = 1, 2
COMPLETE_SYNC, COMPLETE_FLAG, USE_GRAPH, GRAPH_CHAIN = 0, 1, 2, 4

# Table 1 values of the command codes recorded in the device log.
CODE_NOP, CODE_EXIT, CODE_WORK = 4, 8, 16

EXPORTED = [
    "lk_config_default", "lk_init", "lk_submit", "lk_submit_batch", "lk_batch_plan", "lk_wait", "lk_wait_info", "lk_poll",
    "lk_try_wait",
    "lk_prefetch", "lk_dispose", "lk_free", "lk_get_info", "lk_topology", "lk_cluster_members",
    "lk_read_log", "lk_slice", "lk_strerror", "lk_last_error",
    "lkb_serial", "lkb_lanes", "lkb_isolation", "lkb_replay", "lkb_batch", "lkb_launch_burst",
    "lkb_launch_serial", "lks_run", "lkb_launch_lanes", "lkb_pingpong",
    "lkb_copy", "lkb_launch_serial_static",
]


class LKError(RuntimeError):
    def __init__(self, code, where, detail=""):
        self.code = code
        super().__init__(f"{where}: {strerror(code)} ({code}) {detail}".strip())


class Config(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("n_workers", ctypes.c_uint32),
                ("threads_per_worker", ctypes.c_uint32), ("queue_depth", ctypes.c_uint32),
                ("cluster_policy", ctypes.c_uint32), ("n_clusters", ctypes.c_uint32),
                ("cluster_of_worker", ctypes.POINTER(ctypes.c_uint32)),
                ("poll_sleep", ctypes.c_uint32), ("flags", ctypes.c_uint32),
                ("log_capacity", ctypes.c_uint32), ("idle_timeout_ms", ctypes.c_uint32),
                ("workers_per_cu", ctypes.c_uint32), ("init_timeout_ns", ctypes.c_int64),
                ("first_poll_delay", ctypes.c_int32), ("xcd_mask", ctypes.c_uint32)]


class Desc(ctypes.Structure):
    _fields_ = [("op", ctypes.c_uint32), ("flags", ctypes.c_uint32), ("n", ctypes.c_uint64),
                ("a", ctypes.c_int32), ("b", ctypes.c_int32), ("alpha", ctypes.c_float),
                ("reserved", ctypes.c_uint32), ("aux", ctypes.c_uint64),
                ("user_tag", ctypes.c_uint64)]


class Completion(ctypes.Structure):
    _fields_ = [("result", ctypes.c_int64), ("t_pick_min", ctypes.c_uint64),
                ("t_pick_max", ctypes.c_uint64), ("t_done_min", ctypes.c_uint64),
                ("t_done_max", ctypes.c_uint64)]


class Info(ctypes.Structure):
    _fields_ = [("n_workers", ctypes.c_uint32), ("n_clusters", ctypes.c_uint32),
                ("queue_depth", ctypes.c_uint32), ("threads_per_worker", ctypes.c_uint32),
                ("cu_count", ctypes.c_uint32), ("xcd_count", ctypes.c_uint32),
                ("state", ctypes.c_uint32), ("workers_exited", ctypes.c_uint32),
                ("wall_clock_hz", ctypes.c_uint64), ("init_ms", ctypes.c_double),
                ("dispose_ms", ctypes.c_double), ("kernel_ms", ctypes.c_double),
                ("device_span_ms", ctypes.c_double), ("workers_per_cu", ctypes.c_uint32),
                ("max_workers_on_a_cu", ctypes.c_uint32), ("pin_capacity", ctypes.c_uint32),
                ("xcd_mask", ctypes.c_uint32)]


class LogEntry(ctypes.Structure):
    _fields_ = [("seq", ctypes.c_uint32), ("code", ctypes.c_uint16), ("worker", ctypes.c_uint16),
                ("xcc", ctypes.c_uint32), ("hwid", ctypes.c_uint32), ("t_pick", ctypes.c_uint64),
                ("t_done", ctypes.c_uint64)]


class ServeConfig(ctypes.Structure):
    _fields_ = [("arena", ctypes.c_uint64), ("arena_bytes", ctypes.c_uint64), ("tile_elems", ctypes.c_uint64),
                ("threads", ctypes.c_uint32), ("retain", ctypes.c_uint32), ("timeout_ns", ctypes.c_int64)]


class ServeStats(ctypes.Structure):
    _fields_ = [("elapsed_s", ctypes.c_double), ("tiles", ctypes.c_uint64), ("deferred", ctypes.c_uint64),
                ("peak_bytes", ctypes.c_uint64), ("posted", ctypes.c_uint64), ("drained", ctypes.c_uint64)]


REQUEST_DTYPE = np.dtype([("arrival_us", "<f8"), ("op", "<u4"), ("a", "<i4"), ("b", "<i4"), ("alpha", "<f4"),
                          ("n", "<u8"), ("inp", "<u8"), ("in2", "<u8")])
OUTCOME_DTYPE = np.dtype([("result", "<i8"), ("out", "<u8"), ("admit_us", "<f8"), ("done_us", "<f8"),
                          ("status", "<i4"), ("tiles", "<u4")])

# numpy view of lkb_item (56 bytes)
ITEM_DTYPE = np.dtype([("op", "<u4"), ("a", "<i4"), ("b", "<i4"), ("alpha", "<f4"),
                       ("n", "<u8"), ("inp", "<u8"), ("out", "<u8"), ("in2", "<u8"),
                       ("flags", "<u4"), ("reserved", "<u4")])
COMPLETION_DTYPE = np.dtype([("result", "<i8"), ("t_pick_min", "<u8"), ("t_pick_max", "<u8"),
                             ("t_done_min", "<u8"), ("t_done_max", "<u8")])
TILE_DTYPE = np.dtype([("inp", "<u8"), ("out", "<u8"), ("in2", "<u8"), ("n", "<u4"), ("op", "<u4"), ("a", "<i4"),
                       ("b", "<u4"), ("reserved", "<u8")])
LOG_DTYPE = np.dtype([("seq", "<u4"), ("code", "<u2"), ("worker", "<u2"), ("xcc", "<u4"),
                      ("hwid", "<u4"), ("t_pick", "<u8"), ("t_done", "<u8")])

_lib = None


def lib():
    """Load liblk.so (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(hipcc, gfx950); there is no fallback path")
    # PyTorch bundles its own HIP runtime under the same soname; importing it first makes
    # liblk.so bind to that one copy, so tensors and the library share one runtime.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    P, U32, U64, I64, I32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int64, ctypes.c_int32
    PU32, PU64, PI64, PD = (ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint64),
                            ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double))
    sig = {
        "lk_config_default": (None, [ctypes.POINTER(Config)]),
        "lk_init": (ctypes.c_int, [ctypes.POINTER(Config), ctypes.POINTER(P)]),
        "lk_submit": (ctypes.c_int, [P, U32, ctypes.POINTER(Desc), P, P, PU64]),
        "lk_submit_batch": (ctypes.c_int, [P, U32, P, U32, P, PU64]),
        "lk_batch_plan": (ctypes.c_int, [P, P, P, U32, U64, P, P, U32, PU32]),
        "lk_wait": (ctypes.c_int, [P, U32, U64, I64, PI64]),
        "lk_wait_info": (ctypes.c_int, [P, U32, U64, I64, ctypes.POINTER(Completion)]),
        "lk_poll": (ctypes.c_int, [P, U32, U64, ctypes.POINTER(ctypes.c_int)]),
        "lk_try_wait": (ctypes.c_int, [P, U32, U64, ctypes.POINTER(Completion)]),
        "lk_prefetch": (ctypes.c_int, [P, U32, U64]),
        "lk_dispose": (ctypes.c_int, [P]),
        "lk_free": (ctypes.c_int, [P]),
        "lk_get_info": (ctypes.c_int, [P, ctypes.POINTER(Info)]),
        "lk_topology": (ctypes.c_int, [P, U32, PU32, PU32, PU32, PU32]),
        "lk_cluster_members": (ctypes.c_int, [P, U32, PU32, U32, PU32]),
        "lk_read_log": (ctypes.c_int, [P, U32, P, U32, PU32]),
        "lk_slice": (ctypes.c_int, [U64, U32, U32, PU64, PU64]),
        "lk_strerror": (ctypes.c_char_p, [ctypes.c_int]),
        "lk_last_error": (ctypes.c_char_p, []),
        "lkb_serial": (ctypes.c_int, [P, U32, P, U64, I64, P, P, P, P]),
        "lkb_lanes": (ctypes.c_int, [P, P, U32, P, U64, U32, U32, I64, P, P, PD, P]),
        "lkb_isolation": (ctypes.c_int, [P, U32, P, U64, I64, P, U32, P, P, P, P, P, P, PD]),
        "lkb_replay": (ctypes.c_int, [I32, U32, U32, U32, P, P, P, P, P]),
        "lkb_batch": (ctypes.c_int, [P, U32, P, U32, P, U32, I64, P, P]),
        "lkb_launch_burst": (ctypes.c_int, [I32, P, U32, U64, U32, U32, U32, P]),
        "lkb_launch_serial": (ctypes.c_int, [I32, U32, U32, P, U64, U32, P, P, P]),
        "lkb_launch_serial_static": (ctypes.c_int, [I32, U32, U32, P, U64, P, P, P]),
        "lks_run": (ctypes.c_int, [P, ctypes.POINTER(ServeConfig), P, U64, P, ctypes.POINTER(ServeStats)]),
        "lkb_launch_lanes": (ctypes.c_int, [I32, U32, P, U64, U32, U32, U32, U32, P, P, PD]),
        "lkb_pingpong": (ctypes.c_int, [I32, U32, U64, U32, ctypes.c_int, P]),
        "lkb_copy": (ctypes.c_int, [I32, P, P, U64, U32, U32, U32, U32, U32, PD, PD]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def strerror(code):
    try:
        return lib().lk_strerror(code).decode()
    except ImportError:
        return str(code)


def last_error():
    return lib().lk_last_error().decode()


def _check(rc, where):
    if rc != OK:
        raise LKError(rc, where, last_error())
    return rc


def slice_bounds(n, k, j):
    lo, hi = ctypes.c_uint64(), ctypes.c_uint64()
    _check(lib().lk_slice(n, k, j, ctypes.byref(lo), ctypes.byref(hi)), "lk_slice")
    return lo.value, hi.value


def _ptr(t):
    """Device address of a tensor (or an int address)."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _i32(v):
    """Any integer, reduced modulo 2^32 and read as a two's-complement int32."""
    v = int(v) & 0xffffffff
    return v - (1 << 32) if v >= (1 << 31) else v


def _np_ptr(a):
    return a.ctypes.data if a is not None else None


_OP_DTYPES = {OP_AFFINE_SUM_I32: "int32", OP_SUM_I32_I64: "int32", OP_SAXPY_F32: "float32",
              OP_COPY_F32: "float32", OP_AXPY_F32: "float32"}


def _check_tensor(t, op, what):
    if t is None:
        return
    if isinstance(t, int):
        return
    want = _OP_DTYPES.get(op)
    if not t.is_cuda:
        raise ValueError(f"{what} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    if want is not None and str(t.dtype) != "torch." + want:
        raise ValueError(f"{what} must be {want}, got {t.dtype}")


_READS_X = (OP_AFFINE_SUM_I32, OP_SUM_I32_I64, OP_SAXPY_F32, OP_COPY_F32, OP_AXPY_F32)
_WRITES_Y = (OP_AFFINE_SUM_I32, OP_SAXPY_F32, OP_COPY_F32, OP_AXPY_F32)


def submit_extent(op, n, x=None, y=None, aux=None, members=1):
    """Element count of an item given as tensors (or addresses), checked against their
    extent: n defaults to x's (else y's) element count; a tensor x the op reads, a tensor y
    it writes (SAXPY_F32 also reads it) or a tensor aux holding AXPY_F32's y must hold at
    least n elements, and a tensor aux receiving per-member int64 results at least
    `members` of them, else ValueError.  Bare integer addresses are not checked."""
    def size(t):
        return None if t is None or isinstance(t, int) else int(t.numel())
    if n is None:
        ref = x if x is not None else y
        n = size(ref) or 0
    n = int(n)
    if n < 0:
        raise ValueError(f"n = {n} < 0")
    sx, sy, sa = size(x), size(y), size(aux)
    if n and op in _READS_X and sx is not None and n > sx:
        raise ValueError(f"n = {n} exceeds x's {sx} elements")
    if n and op in _WRITES_Y and sy is not None and n > sy:
        raise ValueError(f"n = {n} exceeds y's {sy} elements")
    if op == OP_AXPY_F32 and sa is not None:
        if str(aux.dtype) != "torch.float32":
            raise ValueError(f"aux (y of AXPY_F32) must be float32, got {aux.dtype}")
        if n > sa:
            raise ValueError(f"n = {n} exceeds aux's {sa} elements (y of AXPY_F32)")
    if op in (OP_AFFINE_SUM_I32, OP_SUM_I32_I64) and sa is not None:
        if str(aux.dtype) != "torch.int64":
            raise ValueError(f"aux (per-member results) must be int64, got {aux.dtype}")
        if members > sa:
            raise ValueError(f"aux holds {sa} results, the cluster has {members} members")
    return n


class Context:
    """A running LightKernel context (lk_init): persistent workers, workers_per_cu on each
    CU of the XCDs named by xcd_mask (0 = every XCD), grouped into clusters; depth ring
    slots per mailbox; flags F_* (F_NO_LOOKAHEAD, ...).  Use as a context manager or call
    close() (lk_dispose)."""

    def __init__(self, n_workers=0, threads=256, depth=1, clusters=CLUSTERS_PER_WORKER,
                 cluster_of_worker=None, poll_sleep=0, flags=0, log_capacity=0,
                 idle_timeout_ms=10000, init_timeout_s=5.0, device=0, workers_per_cu=1,
                 first_poll_delay=POLL_DELAY_ADAPTIVE, xcd_mask=0):
        L = lib()
        cfg = Config()
        L.lk_config_default(ctypes.byref(cfg))
        cfg.device = device
        cfg.n_workers = n_workers
        cfg.threads_per_worker = threads
        cfg.queue_depth = depth
        cfg.poll_sleep = poll_sleep
        cfg.flags = flags
        cfg.log_capacity = log_capacity
        cfg.idle_timeout_ms = idle_timeout_ms
        cfg.init_timeout_ns = int(init_timeout_s * 1e9)
        cfg.workers_per_cu = workers_per_cu
        cfg.first_poll_delay = first_poll_delay
        cfg.xcd_mask = xcd_mask
        self._cow = None
        if cluster_of_worker is not None:
            cow = np.ascontiguousarray(cluster_of_worker, dtype=np.uint32)
            self._cow = cow
            cfg.cluster_policy = CLUSTERS_EXPLICIT
            cfg.n_clusters = int(cow.max()) + 1 if cow.size else 0
            cfg.cluster_of_worker = cow.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))
        else:
            cfg.cluster_policy = clusters
        self._sizes = None
        self._h = ctypes.c_void_p()
        rc = L.lk_init(ctypes.byref(cfg), ctypes.byref(self._h))
        if rc != OK:
            detail = last_error()
            if self._h:
                L.lk_free(self._h)
            self._h = None
            raise LKError(rc, "lk_init", detail)
        self._closed = False

    # -- phases ---------------------------------------------------------------------------
    def _cluster_size(self, cluster):
        if self._sizes is None:
            self._sizes = {}
        if cluster not in self._sizes:
            self._sizes[cluster] = len(self.members(cluster))
        return self._sizes[cluster]

    def submit(self, cluster, op, x=None, y=None, a=0, b=0, alpha=0.0, n=None, aux=None, flags=0):
        """Trigger: post one item; returns its ticket.  Raises LKError(EAGAIN) if full.
        flags: DF_PIN_INPUT / DF_PIN_RELOAD (keep x in the members' LDS across items).
        Raises ValueError when a tensor given for x, y or aux is too short for n (the C ABI
        receives bare addresses and cannot check their extent)."""
        _check_tensor(x, op, "x")
        _check_tensor(y, op, "y")
        k = self._cluster_size(cluster) if (aux is not None and not isinstance(aux, int)
                                            and op in (OP_AFFINE_SUM_I32, OP_SUM_I32_I64)) else 1
        n = submit_extent(op, n, x, y, aux, k)
        d = Desc(op, flags, n, _i32(a), _i32(b), float(np.float32(alpha)), 0, _ptr(aux) or 0, 0)
        t = ctypes.c_uint64()
        rc = lib().lk_submit(self._h, cluster, ctypes.byref(d), _ptr(x), _ptr(y), ctypes.byref(t))
        _check(rc, "lk_submit")
        return t.value

    def submit_batch(self, cluster, tiles, n_tiles, partials):
        """Trigger a batch: tiles = device array of lk_tile records (tensor or address),
        partials = device or host-coherent int64 array of n_tiles entries."""
        t = ctypes.c_uint64()
        _check(lib().lk_submit_batch(self._h, cluster, _ptr(tiles), n_tiles, _ptr(partials), ctypes.byref(t)),
               "lk_submit_batch")
        return t.value

    def run_batch(self, cluster, tiles, n_tiles, partials, reps=1, timeout=30.0, with_info=False):
        """Submit-then-wait the same batch `reps` times natively; returns makespans (us)."""
        ms = np.zeros(reps, np.float64)
        info = np.zeros(reps, COMPLETION_DTYPE)
        _check(lib().lkb_batch(self._h, cluster, _ptr(tiles), n_tiles, _ptr(partials), reps, int(timeout * 1e9),
                               _np_ptr(ms), _np_ptr(info)), "lkb_batch")
        return (ms, info) if with_info else ms

    def try_submit(self, cluster, op, **kw):
        """Like submit but returns None when the ring is full."""
        try:
            return self.submit(cluster, op, **kw)
        except LKError as e:
            if e.code == EAGAIN:
                return None
            raise

    def wait(self, cluster, ticket, timeout=10.0):
        """Wait: returns the item's int64 result.  timeout in seconds (None = no deadline)."""
        r = ctypes.c_int64()
        ns = -1 if timeout is None else int(timeout * 1e9)
        _check(lib().lk_wait(self._h, cluster, ticket, ns, ctypes.byref(r)), "lk_wait")
        return r.value

    def wait_info(self, cluster, ticket, timeout=10.0):
        c = Completion()
        ns = -1 if timeout is None else int(timeout * 1e9)
        _check(lib().lk_wait_info(self._h, cluster, ticket, ns, ctypes.byref(c)), "lk_wait_info")
        return {f: getattr(c, f) for f, _ in Completion._fields_}

    def poll(self, cluster, ticket):
        d = ctypes.c_int()
        _check(lib().lk_poll(self._h, cluster, ticket, ctypes.byref(d)), "lk_poll")
        return bool(d.value)

    def try_wait(self, cluster, ticket):
        """Non-blocking Wait: the completion dict if every member finished (the ticket is
        then released), else None."""
        c = Completion()
        rc = lib().lk_try_wait(self._h, cluster, ticket, ctypes.byref(c))
        if rc == EAGAIN:
            return None
        _check(rc, "lk_try_wait")
        return {f: getattr(c, f) for f, _ in Completion._fields_}

    def prefetch(self, cluster, ticket=0):
        """Hint: fetch the cluster's status lines of `ticket` and its next command slots."""
        _check(lib().lk_prefetch(self._h, cluster, ticket), "lk_prefetch")

    def close(self):
        """Dispose: THREAD_EXIT to every worker, join the kernel, free GPU resources."""
        if self._h and not self._closed:
            _check(lib().lk_dispose(self._h), "lk_dispose")
            self._closed = True

    def __del__(self):
        try:
            if self._h:
                lib().lk_free(self._h)
                self._h = None
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- introspection ---------------------------------------------------------------------
    def info(self):
        i = Info()
        _check(lib().lk_get_info(self._h, ctypes.byref(i)), "lk_get_info")
        return {f: getattr(i, f) for f, _ in Info._fields_}

    def topology(self, worker):
        v = [ctypes.c_uint32() for _ in range(4)]
        _check(lib().lk_topology(self._h, worker, *[ctypes.byref(x) for x in v]), "lk_topology")
        return tuple(x.value for x in v)  # (xcc, se, sh, cu)

    def members(self, cluster):
        cnt = ctypes.c_uint32()
        _check(lib().lk_cluster_members(self._h, cluster, None, 0, ctypes.byref(cnt)), "lk_cluster_members")
        out = (ctypes.c_uint32 * max(cnt.value, 1))()
        _check(lib().lk_cluster_members(self._h, cluster, out, cnt.value, ctypes.byref(cnt)), "lk_cluster_members")
        return [out[i] for i in range(cnt.value)]

    def log(self, worker, cap=1 << 20):
        """Device log of a worker (after close()), as a LOG_DTYPE array, oldest first."""
        out = np.zeros(cap, dtype=LOG_DTYPE)
        cnt = ctypes.c_uint32()
        _check(lib().lk_read_log(self._h, worker, _np_ptr(out), cap, ctypes.byref(cnt)), "lk_read_log")
        return out[:cnt.value]

    @property
    def handle(self):
        return self._h

    # -- serving (lk_serve.h) ---------------------------------------------------------------
    def serve(self, requests, arena, arena_bytes, tile_elems=65536, threads=None, retain=False, timeout=10.0):
        """Run a request trace (REQUEST_DTYPE, sorted by arrival) with continuous batching;
        arena = device buffer (tensor or address) of arena_bytes for request outputs;
        threads = scheduler threads (default 4, or one per worker when there are fewer).
        Returns (OUTCOME_DTYPE array, stats dict)."""
        if threads is None:
            threads = min(4, self.info()["n_workers"])
        requests = np.ascontiguousarray(requests, dtype=REQUEST_DTYPE).ravel()
        cfg = ServeConfig(_ptr(arena), int(arena_bytes), int(tile_elems), int(threads), 1 if retain else 0,
                          int(timeout * 1e9))
        outc = np.zeros(max(requests.size, 1), OUTCOME_DTYPE)
        st = ServeStats()
        rc = lib().lks_run(self._h, ctypes.byref(cfg), _np_ptr(requests), requests.size, _np_ptr(outc),
                           ctypes.byref(st))
        _check(rc, "lks_run")
        return outc[:requests.size], {f: getattr(st, f) for f, _ in ServeStats._fields_}

    # -- native runners (lk_bench.h) -------------------------------------------------------
    def run_serial(self, cluster, items, timeout=10.0):
        """Submit-then-wait every item (ITEM_DTYPE array) on one cluster, natively timed.
        Returns (results, lat_us, trigger_us, completions)."""
        items = np.ascontiguousarray(items, dtype=ITEM_DTYPE)
        n = items.size
        res = np.zeros(n, np.int64)
        lat = np.zeros(n, np.float64)
        trig = np.zeros(n, np.float64)
        comp = np.zeros(n, COMPLETION_DTYPE)
        rc = lib().lkb_serial(self._h, cluster, _np_ptr(items), n, int(timeout * 1e9), _np_ptr(res),
                              _np_ptr(lat), _np_ptr(trig), _np_ptr(comp))
        _check(rc, "lkb_serial")
        return res, lat, trig, comp

    def run_lanes(self, lane_cluster, items, in_flight=1, threads=8, timeout=10.0, with_info=False, out=None):
        """items: (n_lanes, items_per_lane) ITEM_DTYPE array.
        Returns (results, lat_us, elapsed_s), plus the per-item COMPLETION_DTYPE array when
        with_info is set.  out = (results, lat_us, info) arrays from lanes_outputs() may be
        given so that the runner writes into memory allocated (and touched) beforehand."""
        items = np.ascontiguousarray(items, dtype=ITEM_DTYPE)
        lanes, per = items.shape
        lc = np.ascontiguousarray(lane_cluster, dtype=np.uint32)
        assert lc.size == lanes
        if out is None:
            res, lat, info = lanes_outputs(lanes, per, with_info)
        else:
            res, lat, info = out
            if (res.shape != (lanes, per) or res.dtype != np.int64 or not res.flags.c_contiguous or
                    lat.shape != (lanes, per) or lat.dtype != np.float64 or not lat.flags.c_contiguous or
                    (with_info and (info is None or info.shape != (lanes, per) or info.dtype != COMPLETION_DTYPE
                                    or not info.flags.c_contiguous))):
                raise ValueError("out arrays must be C-contiguous (lanes, items_per_lane) int64, float64 "
                                 "and COMPLETION_DTYPE")
            if not with_info:
                info = None
        el = ctypes.c_double()
        rc = lib().lkb_lanes(self._h, _np_ptr(lc), lanes, _np_ptr(items), per, in_flight, threads,
                             int(timeout * 1e9), _np_ptr(res), _np_ptr(lat), ctypes.byref(el),
                             _np_ptr(info))
        _check(rc, "lkb_lanes")
        if with_info:
            return res, lat, el.value, info
        return res, lat, el.value

    def run_isolation(self, crit_cluster, crit_items, period_s, bg_clusters, bg_items):
        """Periodic critical items on one cluster beside back-to-back background items on
        others.  Returns dict(results, lat_us, late_us, info, bg_done, elapsed_s)."""
        crit_items = np.ascontiguousarray(crit_items, dtype=ITEM_DTYPE)
        bg_items = np.ascontiguousarray(bg_items, dtype=ITEM_DTYPE)
        bgc = np.ascontiguousarray(bg_clusters, dtype=np.uint32)
        k = crit_items.size
        res = np.zeros(k, np.int64)
        lat = np.zeros(k, np.float64)
        late = np.zeros(k, np.float64)
        info = np.zeros(k, COMPLETION_DTYPE)
        done = np.zeros(max(bgc.size, 1), np.uint64)
        el = ctypes.c_double()
        rc = lib().lkb_isolation(self._h, crit_cluster, _np_ptr(crit_items), k, int(period_s * 1e9),
                                 _np_ptr(bgc), bgc.size, _np_ptr(bg_items), _np_ptr(res), _np_ptr(lat),
                                 _np_ptr(late), _np_ptr(info), _np_ptr(done), ctypes.byref(el))
        _check(rc, "lkb_isolation")
        return dict(results=res, lat_us=lat, late_us=late, info=info, bg_done=done[:bgc.size], elapsed_s=el.value)


def lanes_outputs(lanes, per, with_info=False):
    """Output arrays for Context.run_lanes, every page written once (so no page is first
    touched while the runner's host threads write results)."""
    res = np.empty((lanes, per), np.int64)
    lat = np.empty((lanes, per), np.float64)
    res.fill(0)
    lat.fill(0)
    info = None
    if with_info:
        info = np.empty((lanes, per), COMPLETION_DTYPE)
        info.view(np.uint8).fill(0)
    return res, lat, info


def launch_serial(items, k=1, threads=256, mode=COMPLETE_SYNC, device=0):
    """One ordinary kernel launch per item.  Returns (results, lat_us, launch_us)."""
    items = np.ascontiguousarray(items, dtype=ITEM_DTYPE)
    n = items.size
    res = np.zeros(n, np.int64)
    lat = np.zeros(n, np.float64)
    lau = np.zeros(n, np.float64)
    _check(lib().lkb_launch_serial(device, k, threads, _np_ptr(items), n, mode, _np_ptr(res),
                                   _np_ptr(lat), _np_ptr(lau)), "lkb_launch_serial")
    return res, lat, lau


def launch_serial_static(items, k=1, threads=256, device=0):
    """launch_serial with stream-synchronised completion through the library's
    allocation-free entry point (null stream, partials in a static device array; k at
    most 4096).  Returns (results, lat_us, launch_us)."""
    items = np.ascontiguousarray(items, dtype=ITEM_DTYPE)
    n = items.size
    res = np.zeros(n, np.int64)
    lat = np.zeros(n, np.float64)
    lau = np.zeros(n, np.float64)
    _check(lib().lkb_launch_serial_static(device, k, threads, _np_ptr(items), n, _np_ptr(res), _np_ptr(lat),
                                          _np_ptr(lau)), "lkb_launch_serial_static")
    return res, lat, lau


def batch_plan(items, tile_elems):
    """Cut ITEM_DTYPE items into tiles (lk_batch_plan).  Returns (tiles TILE_DTYPE array,
    tile_item uint32 array)."""
    items = np.ascontiguousarray(items, dtype=ITEM_DTYPE).ravel()
    count = items.size
    descs = (Desc * max(count, 1))()
    for i in range(count):
        op = int(items["op"][i])
        descs[i] = Desc(op, int(items["flags"][i]), int(items["n"][i]), int(items["a"][i]), int(items["b"][i]),
                        float(items["alpha"][i]), 0, int(items["in2"][i]) if op == OP_AXPY_F32 else 0, 0)
    ins = np.ascontiguousarray(items["inp"], dtype=np.uint64)
    outs = np.ascontiguousarray(items["out"], dtype=np.uint64)
    need = ctypes.c_uint32()
    L = lib()
    cap = int(sum(max(1, -(-int(n) // tile_elems)) for n in items["n"]))
    tiles = np.zeros(max(cap, 1), TILE_DTYPE)
    tile_item = np.zeros(max(cap, 1), np.uint32)
    _check(L.lk_batch_plan(descs, _np_ptr(ins), _np_ptr(outs), count, tile_elems, _np_ptr(tiles),
                           _np_ptr(tile_item), cap, ctypes.byref(need)), "lk_batch_plan")
    return tiles[:need.value], tile_item[:need.value]


def launch_burst(items, elems_per_wg=16384, threads=256, graph=True, reps=1, device=0):
    """The burst as per-item launches (graph=False) or one captured hipGraph; makespans (us)."""
    items = np.ascontiguousarray(items, dtype=ITEM_DTYPE).ravel()
    ms = np.zeros(reps, np.float64)
    _check(lib().lkb_launch_burst(device, _np_ptr(items), items.size, elems_per_wg, threads,
                                  USE_GRAPH if graph else 0, reps, _np_ptr(ms)), "lkb_launch_burst")
    return ms


def launch_lanes(items, streams=4, threads_host=8, threads=256, mode=0, device=0):
    """The lanes workload as ordinary launches (lkb_launch_lanes): mode 0 one launch per
    item, USE_GRAPH a single-node graph relaunched per item, GRAPH_CHAIN one captured
    chain per lane (no per-item latency: lat is all zeros).  Returns (results, lat_us,
    elapsed_s)."""
    items = np.ascontiguousarray(items, dtype=ITEM_DTYPE)
    lanes, per = items.shape
    res = np.zeros((lanes, per), np.int64)
    lat = np.zeros((lanes, per), np.float64)
    el = ctypes.c_double()
    _check(lib().lkb_launch_lanes(device, lanes, _np_ptr(items), per, streams, threads_host, threads,
                                  mode, _np_ptr(res), _np_ptr(lat), ctypes.byref(el)),
           "lkb_launch_lanes")
    return res, lat, el.value


REPLAY_PHASES_LK = ("Init", "Trigger", "Wait", "Dispose")
REPLAY_PHASES_HIP = ("Alloc", "Spawn", "Wait", "Dispose")


def replay(n_workers, spin_iters=20000, runs=100, device=0, with_results=False):
    """The paper's phase protocol; returns (lk_us, hip_us, lk_cycles, hip_cycles), each (runs, 4),
    plus the (runs, 2) item results (persistent, per-launch) when with_results is set."""
    lk_us = np.zeros((runs, 4), np.float64)
    hip_us = np.zeros((runs, 4), np.float64)
    lk_cy = np.zeros((runs, 4), np.uint64)
    hip_cy = np.zeros((runs, 4), np.uint64)
    res = np.full((runs, 2), -1, np.int64)
    _check(lib().lkb_replay(device, n_workers, spin_iters, runs, _np_ptr(lk_us), _np_ptr(hip_us),
                            _np_ptr(lk_cy), _np_ptr(hip_cy), _np_ptr(res)), "lkb_replay")
    if with_results:
        return lk_us, hip_us, lk_cy, hip_cy, res
    return lk_us, hip_us, lk_cy, hip_cy


def pingpong(workers=1, iters=10000, poll_sleep=0, spread=True, device=0):
    rtt = np.zeros(workers * iters, np.float64)
    _check(lib().lkb_pingpong(device, workers, iters, poll_sleep, 1 if spread else 0, _np_ptr(rtt)),
           "lkb_pingpong")
    return rtt.reshape(workers, iters)


COPY_PLAIN, COPY_NONTEMPORAL, COPY_SYSTEM = 0, 1, 2


def copy_bandwidth(src, dst, nbytes, grid, reps=10, threads=256, unroll=8, policy=COPY_NONTEMPORAL, device=0):
    """Streaming-copy probe (lkb_copy): returns (average ms per copy, GB/s read + written)."""
    ms, gbps = ctypes.c_double(), ctypes.c_double()
    _check(lib().lkb_copy(device, _ptr(src), _ptr(dst), nbytes, grid, threads, unroll, policy, reps,
                          ctypes.byref(ms), ctypes.byref(gbps)), "lkb_copy")
    return ms.value, gbps.value


def make_items(op, n, inp, out, a=0, b=0, alpha=0.0, in2=0, flags=0):
    """Build an ITEM_DTYPE array from per-item columns (scalars broadcast).  in2 is the y
    address of AXPY_F32 items; flags are DF_* descriptor flags."""
    cols = np.broadcast_arrays(np.asarray(op), np.asarray(n), np.asarray(inp, dtype=np.uint64),
                               np.asarray(out, dtype=np.uint64), np.asarray(a), np.asarray(b),
                               np.asarray(alpha, dtype=np.float32), np.asarray(in2, dtype=np.uint64),
                               np.asarray(flags, dtype=np.uint32))
    shape = cols[0].shape
    it = np.zeros(shape, ITEM_DTYPE)
    it["op"], it["n"], it["inp"], it["out"], it["in2"] = cols[0], cols[1], cols[2], cols[3], cols[7]
    it["flags"] = cols[8]
    it["a"] = (np.asarray(cols[4]).astype(np.int64) & 0xffffffff).astype(np.uint32).view(np.int32)
    it["b"] = (np.asarray(cols[5]).astype(np.int64) & 0xffffffff).astype(np.uint32).view(np.int32)
    it["alpha"] = cols[6]
    return it
