"""Build libmqct.so (HIP, gfx950) in-tree with hipcc."""
import concurrent.futures as cf
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libmqct.so")
SOURCES = ["api.hip", "prep.hip", "gemv.hip", "binned.hip", "adjoint.hip", "queue.hip",
           "queue_r64.hip", "queue_c128.hip", "queue_r32.hip", "queue_c64.hip",
           "coupling.hip", "postproc.hip", "measure.hip", "columns.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wno-unused-result",
         "-Wno-unused-value",
         # packed FP32 arithmetic is kept out of every kernel
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include")]


def _compile(src):
    obj = os.path.join(OBJ, src.replace(".hip", ".o"))
    subprocess.check_call([HIPCC] + FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj])
    return obj


def build(verbose=False):
    """Compile every HIP source for gfx950 and link libmqct.so (always rebuilds)."""
    os.makedirs(OBJ, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
