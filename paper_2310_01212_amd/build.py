"""Build liblk.so (HIP kernels + C ABI) for gfx950, in-tree, with hipcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblk.so")
WORKER_CO = os.path.join(HERE, "lk_worker.hsaco")

SOURCES = ["lk_backend_hip.cpp", "lk_device.hip", "lk_host.cpp", "lk_queue.cpp", "lk_bench.cpp", "lk_serve.cpp"]
WORKER_SOURCE = "lk_worker.hip"

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# -Xclang -target-feature -Xclang -packed-fp32-ops: no packed fp32 instructions are
# generated; -ffp-contract=off: only the explicit fmaf of SAXPY fuses.
COMMON = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-Wall",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-ffp-contract=off", "-fno-gpu-flush-denormals-to-zero",
          "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]
LIB_FLAGS = ["-fPIC", "-shared", "-fvisibility=hidden"]
# The persistent worker is a standalone gfx950 code object, loaded and dispatched by the
# library on its own HSA queue.
WORKER_FLAGS = ["--cuda-device-only", "--no-gpu-bundle-output"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in res.stderr.splitlines() if "packed-fp32-ops" not in l and l.strip())
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed ({res.returncode}):\n{err}")
    if err and verbose:
        print(err, file=sys.stderr)


def build(verbose=False):
    """Compile liblk.so and lk_worker.hsaco in-tree (always recompiles)."""
    tmp_co = WORKER_CO + ".tmp"
    _run([HIPCC, *COMMON, *WORKER_FLAGS, "-o", tmp_co, os.path.join(CSRC, WORKER_SOURCE)], verbose)
    tmp = LIB + ".tmp"
    _run([HIPCC, *COMMON, *LIB_FLAGS, "-o", tmp, *[os.path.join(CSRC, s) for s in SOURCES],
          "-lhsa-runtime64", "-lpthread"], verbose)
    os.replace(tmp_co, WORKER_CO)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
