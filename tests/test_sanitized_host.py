"""The host code of the library under AddressSanitizer and
UndefinedBehaviorSanitizer.

Builds the library with the host compilation sanitized (device code as
usual; see paper_1902_02508_amd.build.build_sanitized) and runs the ABI
tests, which exercise every entry point's validation and size queries
without a GPU, in a child process with the ASan runtime preloaded. Any
heap error or undefined behaviour aborts the child.
"""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _stale(lib, srcs):
    if not os.path.exists(lib):
        return True
    t = os.path.getmtime(lib)
    return any(os.path.getmtime(s) > t for s in srcs)


def test_abi_validation_under_asan_and_ubsan():
    sys.path.insert(0, ROOT)
    from paper_1902_02508_amd import build as B
    srcs = B.sources() + [os.path.join(B.INCLUDE, "eles.h")] + \
        [os.path.join(B.CSRC, f) for f in os.listdir(B.CSRC) if f.endswith(".h")]
    if _stale(B.SAN_LIB, srcs):
        B.build_sanitized()
    env = dict(os.environ)
    env.update({
        "ELES_LIB": B.SAN_LIB,
        "LD_PRELOAD": B.asan_runtime(),
        "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",
        "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1",
    })
    probe = ("import sys; sys.path.insert(0, %r); from paper_1902_02508_amd import eles; "
             "maps = open('/proc/self/maps').read(); "
             "assert eles.LIB_PATH == %r and 'libeles_san.so' in maps and 'libclang_rt.asan' in maps; "
             "print('sanitized library loaded')" % (ROOT, B.SAN_LIB))
    r = subprocess.run([sys.executable, "-c", probe], env=env, cwd=ROOT, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu",
                        os.path.join(ROOT, "tests", "test_abi.py")], env=env, cwd=ROOT, capture_output=True,
                       text=True, timeout=900)
    print(r.stdout[-600:])
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-4000:]
