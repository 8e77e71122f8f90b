"""The C ABI library loads, exports every function include/mvf.h declares,
and its host-only entry points behave (no device needed)."""
import ctypes as C
import json
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mvf.h")
GOLDEN = os.path.join(ROOT, "tests", "golden", "placement_policy_cases.json")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:mvf_status|const char\*)\s+(mvf_\w+)\s*\(", txt, re.M)))


def test_library_exports_every_declared_symbol():
    from paper_1511_07106_amd import _lib
    lib = _lib.load()
    names = _declared()
    assert len(names) >= 28
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    # the binding declares exactly the header's functions
    assert sorted(_lib.exported_names()) == names


def test_struct_layouts_match_header_sizes():
    """ctypes mirrors must have the sizes the C compiler gives the header's
    structs (checked by compiling a tiny probe with gcc)."""
    import subprocess
    import tempfile
    from paper_1511_07106_amd import _lib as L
    structs = ["mvf_config", "mvf_grid_desc", "mvf_volume_desc", "mvf_intrinsics", "mvf_frame",
               "mvf_raycast_out", "mvf_stats", "mvf_stream_frame", "mvf_placement_params",
               "mvf_placement_result", "mvf_dense_tsdf", "mvf_placement_class", "mvf_placement_class_params",
               "mvf_track_model", "mvf_track_params", "mvf_track_stats"]
    src = '#include <stdio.h>\n#include "mvf.h"\nint main(){\n' + "".join(
        f'printf("{s} %zu\\n", sizeof({s}));\n' for s in structs) + "return 0;}\n"
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "p.c")
        open(c, "w").write(src)
        exe = os.path.join(d, "p")
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout
    sizes = dict(l.split() for l in out.strip().splitlines())
    for s in structs:
        assert C.sizeof(getattr(L, s)) == int(sizes[s]), s


def test_status_strings_and_version():
    from paper_1511_07106_amd import _lib
    lib = _lib.load()
    assert lib.mvf_status_string(0) == b"ok"
    assert lib.mvf_status_string(4) == b"exceeds device budget"
    assert lib.mvf_version().startswith(b"mvf")


def test_create_without_device_reports_error():
    """On a machine without a HIP device the context cannot be created and
    the call says why (no silent CPU fallback)."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    from paper_1511_07106_amd import _lib as L
    lib = L.load()
    h = C.c_void_p()
    st = lib.mvf_create(C.byref(h), C.byref(L.mvf_config(0, 0.5, 10.0, 0, 0)))
    assert st != 0 and not h.value
    assert len(lib.mvf_last_error()) > 0


def test_invalid_arguments_rejected_on_host():
    from paper_1511_07106_amd import _lib as L
    lib = L.load()
    h = C.c_void_p()
    bad = L.mvf_config(0, 1.5, 10.0, 0, 0)  # step must be < 1
    assert lib.mvf_create(C.byref(h), C.byref(bad)) == L.MVF_ERR_INVALID_ARG
    assert lib.mvf_create(None, None) == L.MVF_ERR_INVALID_ARG
    assert lib.mvf_integrate(None, 0, None, None, None, None) == L.MVF_ERR_INVALID_ARG
    assert lib.mvf_pose_retract(None, None, None) == L.MVF_ERR_INVALID_ARG


def _policy_cases():
    return json.load(open(GOLDEN))["cases"]


@pytest.mark.parametrize("case", _policy_cases(), ids=lambda c: c["name"])
def test_library_policy_matches_golden(case):
    """The library's insertion/removal step (host code) on the hand-derived
    cases of the paper's placement rule."""
    import paper_1511_07106_amd as mvf
    counts = {tuple(k): c for k, c in case["counts"]}
    H, added, removed = mvf.placement_policy([tuple(a) for a in case["active"]], counts, case["n"],
                                             case["beta"])
    assert sorted(H) == sorted(tuple(a) for a in case["expect_active"])
    assert sorted(added) == sorted(tuple(a) for a in case["expect_added"])
    assert sorted(removed) == sorted(tuple(a) for a in case["expect_removed"])


def test_library_policy_agrees_with_oracle_on_random_tables():
    import oracle as O
    import paper_1511_07106_amd as mvf
    rng = np.random.default_rng(0)
    for trial in range(300):
        n_cells = int(rng.integers(0, 25))
        keys = {tuple(int(x) for x in rng.integers(-3, 4, 3)) for _ in range(n_cells)}
        counts = {k: int(rng.integers(0, 50)) for k in keys}
        pool = list(keys) + [tuple(int(x) for x in rng.integers(-3, 4, 3)) for _ in range(5)]
        n_act = int(rng.integers(0, 8))
        active = list(dict.fromkeys(pool[int(i)] for i in rng.integers(0, len(pool), n_act))) if pool else []
        n_max = int(rng.integers(0, 10))
        active = active[:n_max]
        beta = float(rng.choice([1.0, 1.5, 2.0]))
        a = mvf.placement_policy(active, counts, n_max, beta)
        b = O.placement_policy(active, counts, n_max, beta)
        assert sorted(a[0]) == sorted(b[0]) and sorted(a[1]) == sorted(b[1]) and sorted(a[2]) == sorted(b[2])


def test_pose_retract_matches_oracle_exponential():
    import oracle as O
    import paper_1511_07106_amd as mvf
    rng = np.random.default_rng(1)
    for _ in range(20):
        T = O.compose(np.eye(3, 4), O.se3_exp(rng.normal(size=6)))
        xi = rng.normal(size=6) * rng.choice([1e-12, 1e-3, 0.5])
        np.testing.assert_allclose(mvf.pose_retract(T, xi), O.compose(T, O.se3_exp(xi)), atol=1e-12)


@pytest.mark.parametrize("scale", [1e-6, 3e-3, 0.4, 1.2])
def test_pose_right_jacobian_first_order(scale):
    """T Exp(xi + d) = T Exp(xi) Exp(J d) + O(|d|^2): the residual of the
    first-order step shrinks with |d|^2, while the identity (what the right
    perturbation gradient equals only at xi = 0) leaves an O(|d| |xi|) one."""
    from paper_1511_07106_amd.api import pose_retract, pose_right_jacobian
    rng = np.random.default_rng(int(scale * 1e6) % 1000)
    I34 = np.hstack([np.eye(3), np.zeros((3, 1))])
    for _ in range(5):
        xi = rng.normal(size=6) * scale
        xi[:3] += rng.normal(size=3) * 0.5  # translation part of ordinary size
        J = pose_right_jacobian(xi)
        base = pose_retract(I34, xi)
        res = {}
        for h in (1e-4, 1e-5):
            d = rng.normal(size=6) * h
            lhs = pose_retract(I34, xi + d)
            rhs = pose_retract(base, J @ d)
            res[h] = np.abs(lhs - rhs).max()
            wrong = np.abs(lhs - pose_retract(base, d)).max()
            if scale >= 3e-3 and h == 1e-4:
                assert wrong > 50 * res[h], (wrong, res[h])
        assert res[1e-4] < 1e-7 and res[1e-5] < 1e-9, res
