"""Build libdiscover.so (gfx950) in-tree with hipcc.

    python -m paper_2602_06986_amd.build

Every HIP source is compiled with the packed-FP32 target feature disabled
(plain float code must not be turned into packed FP32 instructions)."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libdiscover.so")
SOURCES = ["dsc_abi.cpp", "dsc_space.cpp", "dsc_screen.hip", "dsc_r3.hip", "dsc_l0.hip", "dsc_batch.hip",
           "dsc_noalloc.hip", "dsc_anneal.hip", "dsc_bnb.hip"]
ARCH = os.environ.get("DISCOVER_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-x", "hip",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
         # kernel arguments arrive in SGPRs at wave start instead of by a
         # first scalar load (the argument tables' address heads each
         # kernel's chain of dependent loads)
         "-mllvm", "-amdgpu-kernarg-preload-count=16"]
# The FP64 matrix products of the Gram and rung-3 kernels keep their
# accumulators in VGPRs (otherwise they are copied between VGPRs and AGPRs
# on every chunk).
EXTRA = {"dsc_l0.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form=1"],
         "dsc_r3.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form=1"],
         # the annealing's decisions: one rounding per operation (no fused
         # multiply-add), so that its trajectory can be reproduced exactly
         "dsc_anneal.hip": ["-ffp-contract=off"]}


def _obj(src):
    return os.path.join(CSRC, "_build", os.path.splitext(src)[0] + ".o")


def build(verbose=False):
    os.makedirs(os.path.join(CSRC, "_build"), exist_ok=True)

    def one(src):
        cmd = [HIPCC] + FLAGS + EXTRA.get(src, []) + ["-c", os.path.join(CSRC, src), "-o", _obj(src)]
        r = subprocess.run(cmd, capture_output=True, text=True)
        msg = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                        if "packed-fp32-ops" not in l and l.strip())
        if r.returncode != 0:
            raise RuntimeError("hipcc failed on %s:\n%s" % (src, msg))
        if verbose and msg:
            print(msg)
        return src

    with ThreadPoolExecutor(max_workers=4) as ex:
        list(ex.map(one, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + \
          [_obj(s) for s in SOURCES]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
