"""Build libfh.so (HIP for gfx950) in-tree with hipcc.

Flags: -ffp-contract=off keeps every binary64 operation of the index
arithmetic separately rounded (the explicit fma is the only fused one);
packed FP32 instructions are disabled."""
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libfh.so")
SOURCES = ["fh_plan.cpp", "fh_hough.hip", "fh_select.hip", "fh_cnn.hip", "fh_coinc.hip", "fh_follow.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"


def flags():
    return ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-ffp-contract=off", "-fno-fast-math",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wall", "-Wno-unused-result",
            "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def build(verbose: bool = False) -> str:
    objs = []
    build_dir = os.path.join(PKG, "_build")
    os.makedirs(build_dir, exist_ok=True)
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        if not os.path.exists(path):
            continue
        obj = os.path.join(build_dir, src + ".o")
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        cmd = [HIPCC] + flags() + lang + ["-c", path, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        err = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l and l.strip())
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{err}")
        if verbose and err:
            print(err, file=sys.stderr)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr)
    os.replace(tmp, LIB)
    build_ceilings(verbose)
    return LIB


CEILINGS = os.path.join(PKG, "_build", "fh_ceilings")


def build_ceilings(verbose: bool = False) -> str:
    """The measured-ceilings microbenchmark (csrc/ceilings.hip), a separate
    executable: run it with `python -m paper_1810_09784_amd.ceilings`."""
    os.makedirs(os.path.dirname(CEILINGS), exist_ok=True)
    tmp = CEILINGS + ".tmp"
    cmd = [HIPCC, "-O3", "-std=c++17", f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", "-Wall", "-x", "hip", os.path.join(CSRC, "ceilings.hip"), "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed on ceilings.hip:\n" + r.stderr)
    os.replace(tmp, CEILINGS)
    return CEILINGS


if __name__ == "__main__":
    print(build(verbose=True))
