"""Builds libqgw.so (HIP, gfx950) in-tree from csrc/.

    python -m paper_2604_22223_amd.build [--jobs N] [--verbose]

Each translation unit is compiled with hipcc to an object in _build/, then
linked into paper_2604_22223_amd/libqgw.so.  Packed FP32 instructions are
disabled for device code.
"""
import argparse
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libqgw.so")

SOURCES = ["api.cpp", "dlr_host.cpp", "kernels_fft.hip", "kernels_dlr.hip", "kernels_dyson.hip",
           "kernels_misc.hip", "kernels_bwd.hip", "kernels_qp.hip", "kernels_hf.hip", "kernels_fft3.hip", "kernels_mf.hip",
           "autotune.cpp"]

ARCH = os.environ.get("QGW_OFFLOAD_ARCH", "gfx950")

# Per-file device options.  The Dyson-W kernel keeps its matrix-core accumulators in ordinary VGPRs: in the
# split form they would take AGPRs on top of the elimination's VGPRs and cost a wave per SIMD.
SOURCE_FLAGS = {"kernels_dyson.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"]}


def hipcc():
    for c in [os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"]:
        if c and os.path.exists(c):
            return c
    return "hipcc"


def common_flags():
    return ["-O3", "-fPIC", "-std=c++17", "--offload-arch=%s" % ARCH, "-mcode-object-version=5",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wno-unused-command-line-argument", "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def compile_one(src, verbose=False, extra=()):
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = ([hipcc(), "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj] + common_flags()
           + SOURCE_FLAGS.get(src, []) + list(extra))
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s\n%s" % (src, res.stdout, res.stderr))
    return obj, res.stderr


def build(jobs=None, verbose=False, extra=()):
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(8, os.cpu_count() or 1)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        futs = {ex.submit(compile_one, s, verbose, extra): s for s in SOURCES}
        objs = {}
        for f in cf.as_completed(futs):
            obj, err = f.result()
            objs[futs[f]] = obj
            if verbose and err.strip():
                print(err, file=sys.stderr)
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", "--offload-arch=%s" % ARCH, "-o", tmp] + [objs[s] for s in SOURCES]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (res.stdout, res.stderr))
    os.replace(tmp, LIB)
    return LIB


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("--verbose", action="store_true")
    ap.add_argument("--resource-usage", action="store_true",
                    help="print per-kernel register / LDS usage")
    a = ap.parse_args()
    extra = ["-Rpass-analysis=kernel-resource-usage"] if a.resource_usage else []
    print(build(a.jobs, a.verbose or a.resource_usage, extra))


if __name__ == "__main__":
    main()
