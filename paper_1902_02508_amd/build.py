"""Compile the HIP sources into the in-tree shared library ``libeles.so``.

    python -m paper_1902_02508_amd.build

Every source is compiled for gfx950 only. Packed FP32 instructions are
disabled for all device code.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libeles.so")
BUILD_DIR = os.path.join(HERE, "_build")

ARCH = "gfx950"
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
    f"-I{INCLUDE}", f"-I{CSRC}",
]

# per-source additions. The perceptron kernels keep matrix-core results in
# ordinary VGPRs (the inference epilogue reads every accumulator, and the
# accumulator-register form costs one copy per value), and run with IEEE
# mode off: the GELU's min / max then take the matrix-core results as they
# are, where IEEE mode makes the compiler canonicalize each one first. The
# perceptron has no NaN inputs and tests none.
EXTRA = {
    "k_mlp.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form", "-mno-amdgpu-ieee", "-fno-honor-nans"],
}


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("build failed:\n" + " ".join(cmd) + "\n" + r.stdout)
    return r.stdout


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


# Host-side AddressSanitizer + UndefinedBehaviorSanitizer build of the same
# library, for the CPU tests of the validation paths (no GPU needed): each
# -fsanitize= applies to the host compilation only; device code is built as
# usual. Loaded with the clang ASan runtime preloaded.
SAN_DIR = os.path.join(HERE, "_build_san")
SAN_LIB = os.path.join(SAN_DIR, "libeles_san.so")
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined"]


def asan_runtime() -> str:
    """The clang ASan runtime shared library (to preload)."""
    import glob
    root = os.path.dirname(os.path.dirname(os.path.realpath(hipcc())))
    hits = sorted(glob.glob(os.path.join(root, "llvm", "lib", "clang", "*", "lib", "linux",
                                         "libclang_rt.asan-x86_64.so")))
    if not hits:
        raise RuntimeError("clang ASan runtime not found")
    return hits[-1]


def _compile_all(build_dir, extra_all, verbose):
    os.makedirs(build_dir, exist_ok=True)
    cc = hipcc()
    objs = []
    jobs = []
    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        for src in sources():
            obj = os.path.join(build_dir, os.path.basename(src)[:-4] + ".o")
            objs.append(obj)
            extra = EXTRA.get(os.path.basename(src), [])
            jobs.append(ex.submit(_run, [cc, *FLAGS, *extra, *extra_all, "-c", src, "-o", obj]))
        for j in jobs:
            out = j.result()
            if verbose and out.strip():
                print(out)
    return cc, objs


def build(verbose: bool = False) -> str:
    """Compile every source and link libeles.so; returns the library path."""
    cc, objs = _compile_all(BUILD_DIR, [], verbose)
    tmp = LIB + ".tmp"
    _run([cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp])
    os.replace(tmp, LIB)
    return LIB


def build_sanitized(verbose: bool = False) -> str:
    """The host-sanitized library (SAN_LIB); returns its path."""
    cc, objs = _compile_all(SAN_DIR, SAN_FLAGS, verbose)
    tmp = SAN_LIB + ".tmp"
    _run([cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-shared-libsan", "-Xarch_host",
          "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", *objs, "-o", tmp])
    os.replace(tmp, SAN_LIB)
    return SAN_LIB


if __name__ == "__main__":
    if "--sanitized" in sys.argv:
        print(build_sanitized(verbose="-v" in sys.argv))
    else:
        print(build(verbose="-v" in sys.argv))
