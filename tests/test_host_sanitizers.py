"""The host side of libmvf built with AddressSanitizer and
UndefinedBehaviorSanitizer (host code only: the device code is compiled as
usual), exercised on the CPU through the entry points that need no device:
the placement policy on random and degenerate inputs, the SE(3) helpers,
status strings, argument checks, and context creation failing cleanly
without a GPU.  A sanitizer report fails the test."""
import glob
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1511_07106_amd", "csrc")

DRIVER = r'''
import ctypes as C, sys
import numpy as np
lib = C.CDLL(sys.argv[1])
PI = C.POINTER(C.c_int32); PD = C.POINTER(C.c_double)
lib.mvf_status_string.restype = C.c_char_p
lib.mvf_last_error.restype = C.c_char_p
for s in range(-2, 10):
    lib.mvf_status_string(s)
rng = np.random.default_rng(1)
for trial in range(400):
    na = int(rng.integers(0, 20)); nc = int(rng.integers(0, 60)); nmax = int(rng.integers(0, 17))
    act = np.ascontiguousarray(rng.integers(-3, 3, (na, 3)), np.int32)
    cells = np.ascontiguousarray(rng.integers(-3, 3, (nc, 3)), np.int32)
    cnt = np.ascontiguousarray(rng.integers(0, 50, nc), np.int32)
    cap = na + nc + 1
    out = np.zeros((max(nmax, 1), 3), np.int32); add = np.zeros((cap, 3), np.int32); rem = np.zeros((cap, 3), np.int32)
    no, nad, nr = C.c_int32(), C.c_int32(), C.c_int32()
    lib.mvf_placement_policy(act.ctypes.data_as(PI), na, cells.ctypes.data_as(PI), cnt.ctypes.data_as(PI), nc,
                             nmax, C.c_float(1.5), out.ctypes.data_as(PI), C.byref(no), add.ctypes.data_as(PI),
                             C.byref(nad), rem.ctypes.data_as(PI), C.byref(nr))
    assert no.value <= max(nmax, 0)
# NULL and bad arguments are rejected, not dereferenced
assert lib.mvf_placement_policy(None, 1, None, None, 1, 4, C.c_float(1.5), None, None, None, None, None, None) != 0
for trial in range(200):
    T = np.ascontiguousarray(rng.normal(size=12)); xi = np.ascontiguousarray(rng.normal(size=6) * 10 ** rng.uniform(-12, 1))
    o = np.zeros(12); J = np.zeros(36)
    lib.mvf_pose_retract(T.ctypes.data_as(PD), xi.ctypes.data_as(PD), o.ctypes.data_as(PD))
    lib.mvf_pose_right_jacobian(xi.ctypes.data_as(PD), J.ctypes.data_as(PD))
assert lib.mvf_pose_retract(None, None, None) != 0
# without a GPU, context creation fails cleanly and leaves a message
ctx = C.c_void_p()
st = lib.mvf_create(C.byref(ctx), None)
assert st != 0 and not ctx.value, st
lib.mvf_last_error()
assert lib.mvf_destroy(None) == 0   # destroying NULL is a no-op
print("sanitized host calls ok")
'''


def _asan_runtime():
    hits = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
    return hits[0] if hits else None


@pytest.mark.skipif(_asan_runtime() is None or not os.path.exists("/opt/rocm/bin/hipcc"),
                    reason="needs ROCm's clang AddressSanitizer runtime and hipcc")
def test_host_code_under_asan_and_ubsan():
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("checks the no-device paths; run on a host without a GPU")
    except ImportError:
        pass
    out = tempfile.mkdtemp()
    lib = os.path.join(out, "libmvf_asan.so")
    flags = ("-O1 -g -fPIC -std=c++17 -ffp-contract=off --offload-arch=gfx950 "
             "-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined "
             "-Xarch_host -fno-omit-frame-pointer -Xarch_host -fno-sanitize-recover=all "
             f"-I{ROOT}/include -I{CSRC}").split()
    objs = []
    for src in ("mvf_kernels.hip", "mvf_track.hip", "mvf_runtime.cpp"):
        o = os.path.join(out, src + ".o")
        cmd = ["/opt/rocm/bin/hipcc", *flags, "-c", os.path.join(CSRC, src), "-o", o]
        if src.endswith(".cpp"):
            cmd.insert(1, "-xhip")
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        objs.append(o)
    link = ["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-shared", "-fPIC",
            "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-o", lib, *objs]
    r = subprocess.run(link, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, LD_PRELOAD=_asan_runtime(), ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", HIP_VISIBLE_DEVICES="")
    r = subprocess.run([sys.executable, "-c", DRIVER, lib], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0 and "sanitized host calls ok" in r.stdout, (r.stdout[-2000:], r.stderr[-4000:])
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
