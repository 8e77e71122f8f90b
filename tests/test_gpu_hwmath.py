"""The hardware square-root estimate (v_sqrt_f32) against the correctly
rounded root, over every non-negative finite binary32.  The integration
kernel takes the estimate and falls back to the correctly rounded root only
near the truncation band; that filter assumes an error of at most 2 ulp for
inputs >= 2^-96 and at most 2^-48 in absolute value below."""
import ctypes as C
import os

import pytest

pytestmark = pytest.mark.gpu

LIB = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1511_07106_amd",
                   "libmvf_selftest.so")


def test_sqrt_estimate_within_filter_bound():
    if not os.path.exists(LIB):
        raise ImportError(f"{LIB} not built; run paper_1511_07106_amd.build")
    import torch  # noqa: F401  (one HIP runtime per process: torch's, loaded first)
    lib = C.CDLL(LIB)
    lib.mvf_selftest_sqrt.argtypes = [C.c_uint32, C.c_uint32, C.POINTER(C.c_uint32), C.POINTER(C.c_float)]
    lib.mvf_selftest_sqrt.restype = C.c_int
    u = C.c_uint32()
    a = C.c_float()
    print("sqrt estimate: all non-negative finite binary32", flush=True)
    rc = lib.mvf_selftest_sqrt(0, 0x7F800000, C.byref(u), C.byref(a))
    assert rc == 0
    print(f"max ulp (x >= 2^-96) = {u.value}, max abs (x < 2^-96) = {a.value:.3e}", flush=True)
    assert u.value <= 2
    assert a.value <= 2.0 ** -48
