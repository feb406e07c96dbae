"""Plain CPU oracle for the LightKernel persistent-thread dispatch path.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this package.  The product library never loads it, and it
shares no code with the HIP path: ``oracle.c`` is plain scalar C, ``brute.py`` is
arbitrary-precision Python for tiny cases, and ``protocol_model.py`` is an exhaustive
state-machine model of the mailbox protocol.

What each piece follows in the paper:
  * Sec. 1 / Sec. 2.3: a persistent worker receives a work descriptor plus references to
    its in/out data and executes it; ``orc_run_fifo`` is the sequential specification of
    one mailbox (posted order, each descriptor exactly once).
  * Sec. 1 / Sec. 2.1 / Sec. 3: work is mapped onto one cluster and a stage triggers one
    or several clusters; ``orc_exec_cluster`` splits an item into per-member slices.
  * The item bodies (int32 affine mod 2^32 + int64 sum, int64 sum, fp32 fma SAXPY,
    fp32 copy) are the evaluation workloads' items; the paper's only item is a
    compute-only loop (Sec. 3), ``orc_spin``: no memory effect, result 0.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")

NOP, AFFINE_SUM_I32, SUM_I32_I64, SAXPY_F32, COPY_F32, SPIN, AXPY_F32 = 0, 1, 2, 3, 4, 5, 7

CFLAGS = ["-O2", "-fno-fast-math", "-ffp-contract=off", "-std=c11", "-Wall", "-Wextra",
          "-shared", "-fPIC"]


def build(force=True):
    """Compile liboracle.so with gcc (plain C, no GPU)."""
    if not force and os.path.exists(_LIB_PATH):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp"
    subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Item(ctypes.Structure):
    _fields_ = [("op", ctypes.c_uint32), ("n", ctypes.c_uint64), ("a", ctypes.c_int32),
                ("b", ctypes.c_int32), ("alpha", ctypes.c_float), ("inp", ctypes.c_void_p),
                ("out", ctypes.c_void_p), ("in2", ctypes.c_void_p)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        L.orc_affine_sum_i32.argtypes = [P, P, ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32]
        L.orc_affine_sum_i32.restype = ctypes.c_int64
        L.orc_sum_i32_i64.argtypes = [P, ctypes.c_uint64]
        L.orc_sum_i32_i64.restype = ctypes.c_int64
        L.orc_saxpy_f32.argtypes = [P, P, ctypes.c_uint64, ctypes.c_float]
        L.orc_saxpy_f32.restype = None
        L.orc_axpy_f32.argtypes = [P, P, P, ctypes.c_uint64, ctypes.c_float]
        L.orc_axpy_f32.restype = None
        L.orc_copy_f32.argtypes = [P, P, ctypes.c_uint64]
        L.orc_copy_f32.restype = None
        L.orc_spin.argtypes = [ctypes.c_int32]
        L.orc_spin.restype = ctypes.c_int64
        L.orc_slice.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64)]
        L.orc_slice.restype = None
        L.orc_exec.argtypes = [ctypes.POINTER(_Item)]
        L.orc_exec.restype = ctypes.c_int64
        L.orc_exec_cluster.argtypes = [ctypes.POINTER(_Item), ctypes.c_uint32]
        L.orc_exec_cluster.restype = ctypes.c_int64
        L.orc_run_fifo.argtypes = [ctypes.POINTER(_Item), ctypes.c_uint64, P]
        L.orc_run_fifo.restype = ctypes.c_int
        L.orc_saxpy_chain_elem.argtypes = [ctypes.c_float, ctypes.c_float, P, ctypes.c_uint64]
        L.orc_saxpy_chain_elem.restype = ctypes.c_float
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data if a is not None else None


def _check(a, dtype):
    if not (isinstance(a, np.ndarray) and a.dtype == dtype and a.flags.c_contiguous):
        raise ValueError(f"expected a C-contiguous {np.dtype(dtype)} numpy array")
    return a


def affine_sum_i32(x, a, b, y=None):
    """Return (y, s): y = (a*x + b) mod 2^32 as int32, s = int64 sum of y."""
    x = _check(x, np.int32)
    if y is None:
        y = np.empty_like(x)
    _check(y, np.int32)
    s = lib().orc_affine_sum_i32(_ptr(x), _ptr(y), x.size, int(a), int(b))
    return y, int(s)


def sum_i32_i64(x):
    x = _check(x, np.int32)
    return int(lib().orc_sum_i32_i64(_ptr(x), x.size))


def saxpy_f32(alpha, x, y):
    """In place: y <- fmaf(alpha, x, y)."""
    _check(x, np.float32)
    _check(y, np.float32)
    assert x.size == y.size
    lib().orc_saxpy_f32(_ptr(x), _ptr(y), x.size, float(np.float32(alpha)))
    return y


def axpy_f32(alpha, x, y, out=None):
    """out <- fmaf(alpha, x, y), y unchanged."""
    _check(x, np.float32)
    _check(y, np.float32)
    assert x.size == y.size
    if out is None:
        out = np.empty_like(y)
    _check(out, np.float32)
    lib().orc_axpy_f32(_ptr(x), _ptr(y), _ptr(out), x.size, float(np.float32(alpha)))
    return out


def copy_f32(src, dst=None):
    _check(src, np.float32)
    if dst is None:
        dst = np.empty_like(src)
    _check(dst, np.float32)
    lib().orc_copy_f32(_ptr(src), _ptr(dst), src.size)
    return dst


def spin(iters):
    """The paper's compute-only item: returns its result (0); -1 for a negative count."""
    return int(lib().orc_spin(int(iters)))


def slice_bounds(n, k, j):
    lo, hi = ctypes.c_uint64(), ctypes.c_uint64()
    lib().orc_slice(n, k, j, ctypes.byref(lo), ctypes.byref(hi))
    return lo.value, hi.value


def _item(op, n, a=0, b=0, alpha=0.0, inp=None, out=None, in2=None):
    return _Item(op, n, int(a), int(b), float(np.float32(alpha)), _ptr(inp), _ptr(out), _ptr(in2))


def exec_item(op, inp=None, out=None, a=0, b=0, alpha=0.0, n=None, in2=None):
    if n is None:
        n = (inp if inp is not None else out).size
    it = _item(op, n, a, b, alpha, inp, out, in2)
    return int(lib().orc_exec(ctypes.byref(it)))


def exec_cluster(op, k, inp=None, out=None, a=0, b=0, alpha=0.0, n=None):
    if n is None:
        n = (inp if inp is not None else out).size
    it = _item(op, n, a, b, alpha, inp, out)
    return int(lib().orc_exec_cluster(ctypes.byref(it), k))


def run_fifo(items):
    """items: list of dicts with keys op, inp, out, a, b, alpha, n. Returns int64 results."""
    arr = (_Item * len(items))()
    for i, d in enumerate(items):
        n = d.get("n")
        if n is None:
            src = d.get("inp") if d.get("inp") is not None else d.get("out")
            n = 0 if src is None else src.size
        arr[i] = _item(d["op"], n, d.get("a", 0), d.get("b", 0), d.get("alpha", 0.0),
                       d.get("inp"), d.get("out"), d.get("in2"))
    res = np.zeros(len(items), dtype=np.int64)
    rc = lib().orc_run_fifo(arr, len(items), _ptr(res))
    if rc != 0:
        raise ValueError("unknown op, or a negative SPIN count, in item list")
    return res


# numpy view of the orc_item layout, so that long item lists are marshalled without a
# Python loop (the executor itself is orc_run_fifo either way).
_ITEM_NP = np.dtype({"names": [f[0] for f in _Item._fields_],
                     "formats": [np.uint32, np.uint64, np.int32, np.int32, np.float32,
                                 np.uint64, np.uint64, np.uint64],
                     "offsets": [getattr(_Item, f[0]).offset for f in _Item._fields_],
                     "itemsize": ctypes.sizeof(_Item)})


class PackedChain:
    """Item records for orc_run_fifo plus references to the arrays they point into."""

    def __init__(self, items, keep):
        self.items = items
        self._keep = keep


def pack_chain(op, inp, out, alphas, a=0, b=0, n=None, in2=None):
    """A FIFO list of len(alphas) items that share op, operands and (a, b) and differ in
    alpha, for run_packed (the list keeps its operand arrays alive)."""
    if n is None:
        n = (inp if inp is not None else out).size
    alphas = np.ascontiguousarray(alphas, dtype=np.float32)
    arr = np.zeros(alphas.size, dtype=_ITEM_NP)
    arr["op"], arr["n"], arr["a"], arr["b"] = op, n, a, b
    arr["alpha"] = alphas
    arr["inp"], arr["out"], arr["in2"] = (_ptr(inp) or 0), (_ptr(out) or 0), (_ptr(in2) or 0)
    return PackedChain(arr, (inp, out, in2))


def run_packed(chain):
    """orc_run_fifo over a list made by pack_chain; returns the int64 results."""
    arr = chain.items if isinstance(chain, PackedChain) else None
    if arr is None or arr.dtype != _ITEM_NP or not arr.flags.c_contiguous:
        raise ValueError("not a packed item list")
    res = np.zeros(arr.size, dtype=np.int64)
    rc = lib().orc_run_fifo(ctypes.cast(arr.ctypes.data, ctypes.POINTER(_Item)), arr.size, _ptr(res))
    if rc != 0:
        raise ValueError("unknown op in item list")
    return res


def saxpy_chain_elem(x, y, alphas):
    alphas = _check(np.ascontiguousarray(alphas, dtype=np.float32), np.float32)
    return np.float32(lib().orc_saxpy_chain_elem(float(x), float(y), _ptr(alphas), alphas.size))
