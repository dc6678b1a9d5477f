"""Builds libvmcrnn.so (hand-written HIP for gfx950) in-tree with hipcc.

Each source is compiled to an object in parallel, then linked into one shared
library that exports the C ABI of include/vmcrnn.h.
"""
import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libvmcrnn.so")
BUILD = os.path.join(ROOT, "_build")
SOURCES = [
    "api.hip",
    "engine.hip",
    "engine_bf16_1d.hip",
    "engine_bf16_2d.hip",
    "engine_f32_1d.hip",
    "engine_f32_2d.hip",
    "backward.hip",
    "forward.hip",
    "grad.hip",
    "grow.hip",
    "optim.hip",
]
ARCH = "gfx950"


def hipcc():
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def _flags(csrc):
    # -ffp-contract=on: a multiply-add is fused only where it is written as one
    # expression, so every instantiation of a kernel template rounds alike
    return ["--offload-arch=" + ARCH, "-O3", "-ffp-contract=on", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
            "-Wno-unused-variable", "-Wno-unused-but-set-variable", "-I" + os.path.join(ROOT, "include"),
            "-I" + csrc, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _compile(src, csrc=CSRC, build_dir=BUILD):
    obj = os.path.join(build_dir, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc()] + _flags(csrc) + ["-c", os.path.join(csrc, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (src, out))
    return obj, out


def build(verbose=False, csrc=CSRC, lib=LIB, build_dir=BUILD):
    """Compile every source of `csrc` and link `lib` (defaults: the package)."""
    os.makedirs(build_dir, exist_ok=True)
    jobs = int(os.environ.get("MAX_JOBS", "8"))
    with concurrent.futures.ThreadPoolExecutor(max_workers=max(1, min(jobs, len(SOURCES)))) as ex:
        results = list(ex.map(lambda src: _compile(src, csrc, build_dir), SOURCES))
    objs = [o for o, _ in results]
    if verbose:
        for _, out in results:
            if out.strip():
                print(out)
    tmp = lib + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    subprocess.check_call(cmd)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
