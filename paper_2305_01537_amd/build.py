"""Build libsphfilt.so (HIP, gfx950) in-tree.

    python -m paper_2305_01537_amd.build        # or build() from Python

Every source is compiled by hipcc for gfx950 only, -O3, no fast-math, into an
object file under _build/ (the translation units compile in parallel), and the
objects are linked into paper_2305_01537_amd/libsphfilt.so.  Packed FP32
instructions are disabled for every HIP translation unit.
"""
import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(ROOT, "_build", "sphfilt")
LIB = os.path.join(HERE, "libsphfilt.so")
SOURCES = ["host_tables.cpp", "tune_cache.cpp", "plan.cpp", "batch.cpp", "kernels.hip", "kernels_theta.hip",
           "kernels_phi.hip", "batch.hip", "batch_plain.hip", "batch_hybrid.hip",
           "batch_mixed.hip", "batch_mixed_hybrid.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-command-line-argument",
         "-I", os.path.join(ROOT, "include"), "-I", CSRC]

# The batch kernels loop over work items (and over tiles and ring groups
# inside an item).  Machine-level loop-invariant code motion hoists the
# constants of every exp() in the loop body out of those loops, keeps them
# live across the whole item and spills them (the persistent plain kernel
# reloaded them from scratch ~140 times per item; the hybrid one-shot kernel
# spilled 83 registers).  Without that pass the batch kernels do not spill.
# The plan kernels have no such loops and are built unchanged.
PER_SOURCE_FLAGS = {s: ["-mllvm", "-disable-machine-licm"]
                    for s in ("batch_plain.hip", "batch_hybrid.hip", "batch_mixed.hip",
                              "batch_mixed_hybrid.hip")}


def _jobs() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16, len(SOURCES)))


def _compile(src, extra, verbose):
    obj = os.path.join(OBJ, os.path.basename(src) + ".o")
    per = PER_SOURCE_FLAGS.get(os.path.basename(src), [])
    cmd = [HIPCC, *FLAGS, *per, *extra, "-x", "hip", "-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    msgs = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                     if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{msgs}")
    if verbose and msgs.strip():
        print(msgs, flush=True)
    return obj


def build(verbose: bool = False, extra=()) -> str:
    os.makedirs(OBJ, exist_ok=True)
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    with concurrent.futures.ThreadPoolExecutor(_jobs()) as ex:
        objs = list(ex.map(lambda s: _compile(s, list(extra), verbose), srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv, extra=[a for a in sys.argv[1:] if a != "-v"])
