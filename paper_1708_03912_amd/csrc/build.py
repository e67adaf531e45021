"""Build libfraclap.so (gfx950) in-tree with hipcc.

Translation units: the assembly kernels, the single-system solver kernels, the
batched product / solver kernels, the surrogate network kernels and the
multigrid kernels, the strong-form kernels and the cluster kernels (default
floating-point contraction), the host planner (no contraction, see
fl_api.hip), the batched host calls, the surrogate host calls, the
multigrid host calls, the strong-form host calls and the cluster host calls
(no contraction: the cluster boxes decide admissibility).
Packed FP32 instructions are disabled for all device code.  Units are built
in parallel.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.dirname(HERE)
LIB = os.path.join(PKG, "libfraclap.so")
ARCH = os.environ.get("FRACLAP_ARCH", "gfx950")
COMMON = ["-O3", "-fPIC", "-std=c++17", f"--offload-arch={ARCH}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics", "-Wall", "-Wno-unused-function", "-Wno-unused-variable"]
UNITS = [("fl_kernels.hip", []), ("fl_solve.hip", []), ("fl_batch.hip", []), ("fl_sur.hip", []), ("fl_mg.hip", []),
         ("fl_sf.hip", []), ("fl_cluster.hip", []), ("fl_api.hip", ["-ffp-contract=off"]),
         ("fl_batch_api.hip", []), ("fl_sur_api.hip", []), ("fl_mg_api.hip", []), ("fl_sf_api.hip", ["-ffp-contract=off"]),
         ("fl_cluster_api.hip", ["-ffp-contract=off"])]


def build(verbose=False):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objs, procs = [], []
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    for src, extra in UNITS:
        obj = os.path.join(bdir, src.replace(".hip", ".o"))
        cmd = [hipcc, "-c", os.path.join(HERE, src), "-o", obj] + COMMON + extra
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((cmd, subprocess.Popen(cmd)))
        objs.append(obj)
    for cmd, p in procs:
        if p.wait() != 0:
            raise subprocess.CalledProcessError(p.returncode, cmd)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
