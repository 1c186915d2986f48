"""Build of the gfx950 C-ABI library ``liblbm.so`` (hipcc, in-tree).

Each translation unit is compiled to an object in ``_build/`` by its own
hipcc process (in parallel), then the objects are linked into the shared
library.  The time-step kernels are instantiated in several translation
units (per precision and velocity set) so that they compile side by side.
"""
from __future__ import annotations

import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "liblbm.so")
ROOT = os.path.dirname(HERE)

SOURCES = ["lbm_step_f32q9.hip", "lbm_fstep_f32.hip", "lbm_step_f64q9.hip", "lbm_fstep_f64.hip",
           "lbm_step_f32q3.hip", "lbm_step_f64q3.hip", "lbm_kernels.hip", "lbm_api.hip", "lbm_fstar.hip",
           "lbm_mlp.hip", "lbm_mlp_infer.hip", "lbm_api_learn.hip", "lbm_spectrum.hip"]
HEADERS = ["lbm_device.hpp", "lbm_launch.hpp", "lbm_fstar.hpp", "lbm_fstar_dev.hpp", "lbm_internal.hpp",
           "lbm_fstar_site.hpp", "lbm_step.hpp", "lbm_mlp_dev.hpp"]

# -packed-fp32-ops: no packed FP32 instructions are generated
HIPCC_FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-Wall", "-Wno-unused-function"]


# per translation unit: the inference kernels keep the matrix-core results
# in ordinary vector registers, so the activations read them without a copy
# out of the accumulation registers
EXTRA_FLAGS = {"lbm_mlp_infer.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form=1"]}


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def sources():
    return [os.path.join(CSRC, s) for s in SOURCES]


def _deps():
    return [os.path.join(CSRC, h) for h in HEADERS] + [os.path.join(ROOT, "include", "lbm.h")]


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(d) > t for d in sources() + _deps() if os.path.exists(d))


def _compile(src: str, incremental: bool, verbose: bool) -> str:
    obj = os.path.join(OBJ, os.path.basename(src)[:-4] + ".o")
    if incremental and os.path.exists(obj):
        t = os.path.getmtime(obj)
        if all(os.path.getmtime(d) <= t for d in [src] + _deps()):
            return obj
    tmp = obj + ".tmp%d" % os.getpid()
    cmd = [hipcc()] + HIPCC_FLAGS + EXTRA_FLAGS.get(os.path.basename(src), []) + ["-c", src, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed on %s:\n%s%s" % (src, res.stdout, res.stderr))
    os.replace(tmp, obj)
    return obj


def build(verbose: bool = False, incremental: bool = False, jobs: int = 0) -> str:
    """Compile every HIP source for gfx950 and link liblbm.so.  By default
    every object is recompiled; incremental=True keeps objects newer than
    their source and the headers."""
    os.makedirs(OBJ, exist_ok=True)
    jobs = jobs or min(len(SOURCES), os.cpu_count() or 1)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, incremental, verbose), sources()))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc link failed:\n" + res.stdout + res.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    import sys
    print(build(verbose=True, incremental="-i" in sys.argv))
