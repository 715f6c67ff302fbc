"""Build libfv.so (the HIP kernels and the C ABI of include/fv.h) for gfx950.

    python -m paper_2302_09005_amd.build [-v]

The library is written in-tree to paper_2302_09005_amd/lib/libfv.so.  hipcc
cross-compiles for gfx950 without a GPU.  Packed-FP32 instructions are
disabled for every HIP translation unit, and floating-point contraction is
off: the kernels write their fused multiply-adds explicitly.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIBDIR = os.path.join(HERE, "lib")
LIB = os.path.join(LIBDIR, "libfv.so")
SOURCES = ["fv_api.hip", "fv_update.hip", "fv_update_f32.hip", "fv_reduce.hip", "fv_halo.hip",
           "fv_learned_train.hip",
           "fv_learned_infer.hip"]
ARCH = os.environ.get("FV_OFFLOAD_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH, "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-munsafe-fp-atomics", "-Wall", "-Wno-unused-function",
         "-Wno-unused-command-line-argument"]


# Per-source flags.  The learned update keeps its matrix-core accumulators in
# ordinary vector registers: tanh and the bfloat16 packing read every
# accumulator, and accumulation registers would cost one move per value.
SOURCE_FLAGS = {"fv_learned_infer.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
                # the float32 update instances: the instruction-level-parallelism
                # schedule (they keep four waves per SIMD with it)
                "fv_update_f32.hip": ["-mllvm", "-amdgpu-sched-strategy=max-ilp"]}


def build(verbose: bool = False, extra=()) -> str:
    os.makedirs(LIBDIR, exist_ok=True)
    objs = [os.path.join(LIBDIR, os.path.splitext(src)[0] + ".o") for src in SOURCES]
    cmds = [[HIPCC, *FLAGS, *SOURCE_FLAGS.get(src, []), *extra, "-c", os.path.join(CSRC, src),
             "-o", obj]
            for src, obj in zip(SOURCES, objs)]
    if verbose:
        for cmd in cmds:
            print(" ".join(cmd), flush=True)
    # the translation units compile independently: a few at a time
    jobs = max(1, min(len(cmds), int(os.environ.get("MAX_JOBS", "6"))))
    with ThreadPoolExecutor(jobs) as pool:
        for res in pool.map(lambda c: subprocess.run(c, check=True), cmds):
            pass
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH, *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
