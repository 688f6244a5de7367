"""Build the gfx950 rasterizer library (libdiffsoup.so) in-tree with hipcc.

Flags: -O3 for gfx950 only; -ffp-contract=off so that only the explicit
fused multiply-adds of the arithmetic contract are fused; packed FP32
instructions disabled (-packed-fp32-ops target feature off).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
OUT = os.path.join(HERE, "libdiffsoup.so")
SOURCES = ['fwd_k8_16_1_t8.hip', 'fwd_k8_16_1_t16.hip', 'fwd_k8_16_1_t32.hip', 'fwd_k16_32_2_t8.hip', 'fwd_k16_32_2_t16.hip', 'fwd_k16_32_2_t32.hip', 'fwd_k32_64_2_t8.hip', 'fwd_k32_64_2_t16.hip', 'fwd_k32_64_2_t32.hip', 'dbwd_k8_16_1.hip', 'dbwd_k16_32_2.hip', 'dbwd_k32_64_2.hip', 'fwd_paper_t8.hip', 'fwd_paper_t16.hip', 'fwd_paper_t32.hip'] + ["api.hip", "pform.hip", "bin.hip", "replay.hip", "raster_fwd.hip", "raster_bwd.hip", "adaptive.hip", "train.hip", "probe.hip"]
ARCH = os.environ.get("SOUP_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def flags():
    return ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-ffp-contract=off",
            "-fno-gpu-flush-denormals-to-zero", "-fhip-fp32-correctly-rounded-divide-sqrt",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
            "-I", os.path.join(ROOT, "include")]


OBJDIR = os.path.join(ROOT, "_build", "csrc")


def _newest_header() -> float:
    paths = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hpp", ".h"))]
    paths.append(os.path.join(ROOT, "include", "diffsoup.h"))
    return max(os.path.getmtime(p) for p in paths)


def build(verbose: bool = False, jobs: int = 0, force: bool = True) -> str:
    """Compile every source (force) or only those older than their object."""
    if jobs <= 0:
        jobs = max(1, min(len(SOURCES), os.cpu_count() or 4))
    os.makedirs(OBJDIR, exist_ok=True)
    hdr = _newest_header()
    objs = []
    procs = []
    for src in SOURCES:
        obj = os.path.join(OBJDIR, src.replace(".hip", ".o"))
        objs.append(obj)
        srcp = os.path.join(CSRC, src)
        if not force and os.path.exists(obj) and os.path.getmtime(obj) >= max(os.path.getmtime(srcp), hdr):
            continue
        cmd = [hipcc(), *flags(), "-c", "-x", "hip", srcp, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd)))
        if len(procs) >= jobs:
            src0, p0 = procs.pop(0)
            if p0.wait() != 0:
                raise RuntimeError(f"hipcc failed on {src0}")
    for src0, p0 in procs:
        if p0.wait() != 0:
            raise RuntimeError(f"hipcc failed on {src0}")
    link = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", OUT + ".tmp", *objs]
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.run(link, check=True)
    os.replace(OUT + ".tmp", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose="-v" in sys.argv, force="--force" in sys.argv)
