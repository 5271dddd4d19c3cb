"""Build libmbe3osv.so for gfx950 in-tree with hipcc (cross-compiles without
a GPU).  Usage: python -m paper_2603_16575_amd.build"""
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "lib", "libmbe3osv.so")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # no packed-FP32 instruction selection
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-pass-failed",
]


# AddressSanitizer and UndefinedBehaviorSanitizer on the host code only
# (the planner, the C-ABI, the launch wrappers); the gfx950 code is built as
# usual.  The library then needs the ASan runtime preloaded into the process.
HOST_SANITIZE_FLAGS = [
    "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
    "-Xarch_host", "-fno-sanitize-recover=undefined",
    "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-g",
]


def asan_runtime():
    """Path of the ASan runtime of hipcc's clang (to preload), or None."""
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


def build(verbose=False, out=None, host_sanitize=False):
    out = OUT if out is None else out
    os.makedirs(os.path.dirname(out), exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip"))) + [os.path.join(CSRC, "api.cpp")]
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = out + ".tmp"
    flags = HIPCC_FLAGS + (HOST_SANITIZE_FLAGS if host_sanitize else [])
    cmd = [hipcc, *flags, "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           *srcs, "-o", tmp]
    if verbose:
        print(" ".join(cmd))
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libmbe3osv")
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
