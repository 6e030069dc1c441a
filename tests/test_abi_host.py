"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every symbol include/mrpie.h declares, and validates problems on the host."""
import ctypes as C
import os
import re

import pytest

from paper_2205_04295_amd import _abi
from paper_2205_04295_amd._abi import Problem, make_params

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mrpie.h")


def header_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mrpie_[a-z0-9_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_abi.LIB_PATH):
        pytest.fail("libmrpie.so is not built (run __graft_entry__.build())")
    return _abi.load()


def test_header_symbols_exported(lib):
    names = header_functions()
    assert len(names) >= 6
    for n in names:
        assert hasattr(lib, n), n
        assert n in _abi.exported_symbols(), f"{n} has no ctypes signature"


def test_version(lib):
    assert b"gfx950" in lib.mrpie_version()


def _validate(lib, pb, **kw):
    return lib.mrpie_validate(C.byref(pb), C.byref(make_params(**kw)))


def test_validate_accepts_supported_shapes(lib):
    for N in (64, 128, 192, 256):
        for M in (1, 3, 8):
            assert _validate(lib, Problem(H=N + 7, W=2 * N, N=N, M=M, J=5)) == 0


@pytest.mark.parametrize("pb,kw,code", [
    (Problem(256, 256, 96, 1, 10), {}, _abi.MRPIE_EUNSUPPORTED),
    (Problem(256, 256, 64, 9, 10), {}, _abi.MRPIE_EUNSUPPORTED),
    (Problem(256, 256, 64, 0, 10), {}, _abi.MRPIE_EINVAL),
    (Problem(256, 256, 64, 1, 0), {}, _abi.MRPIE_EINVAL),
    (Problem(63, 256, 64, 1, 10), {}, _abi.MRPIE_EINVAL),
    (Problem(256, 256, 64, 1, 10), dict(beta=1.5), _abi.MRPIE_EINVAL),
    (Problem(256, 256, 64, 1, 10), dict(gamma=-0.1), _abi.MRPIE_EINVAL),
    (Problem(256, 256, 64, 1, 10), dict(iterations=-1), _abi.MRPIE_EINVAL),
    (Problem(256, 256, 64, 1, 10), dict(alpha_obj=float("nan")), _abi.MRPIE_EINVAL),
    (Problem(256, 256, 64, 1, 10), dict(subpixel=2), _abi.MRPIE_EINVAL),
    (Problem(256, 256, 64, 1, 10), dict(propagator=2), _abi.MRPIE_EINVAL),
    (Problem(256, 256, 64, 1, 10), dict(propagator=1, fresnel=0.0), _abi.MRPIE_EINVAL),
    (Problem(256, 256, 64, 1, 10), dict(propagator=1, fresnel=float("inf")), _abi.MRPIE_EINVAL),
    (Problem(256, 256, 64, 1, 10), dict(refine=1, xcorr_point=2), _abi.MRPIE_EINVAL),
])
def test_validate_rejects(lib, pb, kw, code):
    assert _validate(lib, pb, **kw) == code
    assert lib.mrpie_last_error() != b""


def test_null_arguments_rejected_before_launch(lib):
    pb = Problem(256, 256, 64, 1, 10)
    prm = make_params()
    assert lib.mrpie_validate(None, C.byref(prm)) == _abi.MRPIE_EINVAL
    n = C.c_size_t(0)
    assert lib.mrpie_workspace_size(C.byref(pb), C.byref(prm), C.byref(n)) == 0 and n.value > 0
    # null arrays are rejected on the host, nothing is launched
    rc = lib.mrpie_rpie(C.byref(pb), C.byref(prm), None, None, None, None, None, None, None, None,
                        C.c_size_t(0), None)
    assert rc == _abi.MRPIE_EINVAL
    assert lib.mrpie_fft2(96, 1, None, 0, None) == _abi.MRPIE_EUNSUPPORTED
    assert lib.mrpie_fft2(64, 0, None, 0, None) == 0     # empty batch: nothing to do


def test_validate_accepts_near_field_and_xcorr_b(lib):
    pb = Problem(256, 256, 64, 1, 10)
    assert _validate(lib, pb, propagator=1, fresnel=40.0) == 0
    assert _validate(lib, pb, refine=1, xcorr_point=1, propagator=1, fresnel=40.0, subpixel=1) == 0


@pytest.mark.parametrize("kw", [dict(subpixel=1), dict(refine=1), dict(propagator=1, fresnel=40.0)])
def test_batched_rejects_what_it_does_not_run(lib, kw):
    """The batched sweep takes integer crops, no refinement and the far
    field: other settings are refused on the host, before anything is
    launched (the job's device pointers are never touched)."""
    fake = C.c_void_p(0x1000)
    job = _abi.Job(Problem(256, 256, 64, 1, 10), fake, fake, fake, fake, None, None, fake, C.c_size_t(1 << 30))
    arr = (_abi.Job * 1)(job)
    prm = make_params(**kw)
    rc = lib.mrpie_rpie_batched(1, C.cast(arr, C.c_void_p), C.byref(prm), None, None)
    assert rc == _abi.MRPIE_EUNSUPPORTED
    assert b"batched" in lib.mrpie_last_error()


def test_workspace_too_small_rejected(lib):
    pb = Problem(256, 256, 64, 1, 10)
    prm = make_params()
    fake = C.c_void_p(0x1000)
    rc = lib.mrpie_rpie(C.byref(pb), C.byref(prm), fake, fake, fake, None, fake, None, None, fake,
                        C.c_size_t(16), None)
    assert rc == _abi.MRPIE_EWORKSPACE


def test_register_and_adam_argument_checks(lib):
    n = C.c_size_t(0)
    assert lib.mrpie_register_workspace_size(256, 1600, 100, C.byref(n)) == 0 and n.value > 0
    assert lib.mrpie_register_workspace_size(96, 4, 100, C.byref(n)) == _abi.MRPIE_EUNSUPPORTED
    assert lib.mrpie_register_workspace_size(64, 4, 0, C.byref(n)) == _abi.MRPIE_EINVAL
    assert lib.mrpie_register(64, 0, None, None, 100, 1, None, None, None, 0, None) == 0
    assert lib.mrpie_register(64, 2, None, None, 100, 1, None, None, None, 0, None) == _abi.MRPIE_EINVAL
    assert lib.mrpie_register(64, 2, None, None, 100, 3, None, None, None, 0, None) == _abi.MRPIE_EINVAL
    prm = make_params(adam_b1=1.0)
    assert lib.mrpie_adam(4, C.byref(prm), 10, 10, None, None, None, 1, None) == _abi.MRPIE_EINVAL
    prm = make_params()
    assert lib.mrpie_adam(4, C.byref(prm), 10, 10, None, None, None, 0, None) == _abi.MRPIE_EINVAL
    assert lib.mrpie_adam(0, C.byref(prm), 10, 10, None, None, None, 1, None) == 0


def _fields(t):
    return (t.rows_radix, t.cols_radix, t.rows_threads, t.lds_sweep, t.cols_width, t.rows_inplace, t.rows_split)


def test_tuning_round_trip(lib):
    d = _abi.Tuning()
    assert lib.mrpie_get_tuning(128, 3, 1, C.byref(d)) == 0
    assert (d.rows_radix, d.cols_radix, d.rows_threads, d.lds_sweep) == (8, 8, 256, 0)
    assert (d.cols_width, d.rows_inplace, d.rows_split) == (4, 1, 0)  # batches of 2-15 jobs
    dl = _abi.Tuning()
    assert lib.mrpie_get_tuning(128, 3, 2, C.byref(dl)) == 0
    assert (dl.cols_width, dl.rows_inplace, dl.rows_split) == (4, 1, 1)  # batches of 16 or more
    assert lib.mrpie_get_tuning(128, 3, 3, C.byref(dl)) == _abi.MRPIE_EINVAL
    d0 = _abi.Tuning()
    assert lib.mrpie_get_tuning(128, 3, 0, C.byref(d0)) == 0
    assert (d0.cols_width, d0.rows_inplace, d0.rows_split) == (1, 0, 0)
    d64 = _abi.Tuning()
    assert lib.mrpie_get_tuning(64, 1, 0, C.byref(d64)) == 0 and d64.lds_sweep == 1
    for cls in (1, 2):  # batches run small jobs through the shared passes by default
        assert lib.mrpie_get_tuning(64, 1, cls, C.byref(d64)) == 0 and d64.lds_sweep == 0
    d32 = _abi.Tuning()
    assert lib.mrpie_get_tuning(32, 5, 0, C.byref(d32)) == 0 and d32.lds_sweep == 8
    # per mode class: setting M = 3 changes the class of M = 3-4 only
    t = _abi.Tuning(8, 4, 256, 0, 4, 1)
    assert lib.mrpie_set_tuning(128, 3, 1, C.byref(t)) == 0
    for M, want in ((3, _fields(t)), (4, _fields(t)), (2, _fields(d)), (5, _fields(d))):
        u = _abi.Tuning()
        assert lib.mrpie_get_tuning(128, M, 1, C.byref(u)) == 0
        assert _fields(u) == want, M
    assert lib.mrpie_set_tuning(128, 0, 1, C.byref(t)) == 0   # M = 0: every mode class
    u = _abi.Tuning()
    assert lib.mrpie_get_tuning(128, 7, 1, C.byref(u)) == 0 and _fields(u) == _fields(t)
    assert lib.mrpie_set_tuning(128, 1, 1, C.byref(_abi.Tuning(5, 4, 256, 1, 1))) == _abi.MRPIE_EINVAL
    assert lib.mrpie_set_tuning(128, 1, 1, C.byref(_abi.Tuning(8, 4, 256, 9, 1))) == _abi.MRPIE_EINVAL
    assert lib.mrpie_set_tuning(128, 1, 1, C.byref(_abi.Tuning(8, 4, 256, 0, 2))) == _abi.MRPIE_EINVAL
    assert lib.mrpie_set_tuning(128, 1, 1, C.byref(_abi.Tuning(8, 4, 256, 0, 1, 3))) == _abi.MRPIE_EINVAL
    assert lib.mrpie_set_tuning(128, 1, 1, C.byref(_abi.Tuning(8, 4, 256, 0, 1, 1, 2))) == _abi.MRPIE_EINVAL
    assert lib.mrpie_set_tuning(128, 9, 1, C.byref(t)) == _abi.MRPIE_EINVAL
    assert lib.mrpie_get_tuning(128, 0, 1, C.byref(u)) == _abi.MRPIE_EINVAL
    assert lib.mrpie_set_tuning(100, 1, 1, C.byref(t)) == _abi.MRPIE_EUNSUPPORTED
    u2 = _abi.Tuning()
    assert lib.mrpie_get_tuning(128, 3, 2, C.byref(u2)) == 0 and _fields(u2) == _fields(dl)  # other class
    assert lib.mrpie_set_tuning(128, 0, 1, C.byref(d)) == 0  # restore the default
    # N = 32 (the fifth probe size) has a table entry of its own
    t32 = _abi.Tuning(4, 4, 512, 2, 1, 0)
    assert lib.mrpie_set_tuning(32, 0, 0, C.byref(t32)) == 0
    u = _abi.Tuning()
    assert lib.mrpie_get_tuning(32, 2, 0, C.byref(u)) == 0 and _fields(u) == _fields(t32)
    assert lib.mrpie_get_tuning(256, 2, 0, C.byref(u)) == 0 and _fields(u) == (8, 8, 256, 0, 1, 0, 0)
    assert lib.mrpie_set_tuning(32, 0, 0, C.byref(d32)) == 0


def test_autotuner_candidates_and_workspace(lib):
    """The autotuner's candidate list (the in-place and split options only
    for batches, the LDS sweep only where the modes fit it) and its
    workspace size; the timing itself needs a GPU."""
    assert lib.mrpie_tuning_candidates(256, 3, 0, None, 0) == 16
    assert lib.mrpie_tuning_candidates(256, 3, 1, None, 0) == 64
    assert lib.mrpie_tuning_candidates(64, 2, 0, None, 0) == 17
    assert lib.mrpie_tuning_candidates(64, 5, 1, None, 0) == 64
    arr = (_abi.Tuning * 17)()
    assert lib.mrpie_tuning_candidates(64, 2, 0, arr, 17) == 17
    assert _fields(arr[16]) == (8, 8, 256, 8, 1, 0, 0)
    assert all(arr[i].rows_inplace == 0 and arr[i].rows_split == 0 for i in range(17))
    arr = (_abi.Tuning * 64)()
    assert lib.mrpie_tuning_candidates(256, 3, 1, arr, 64) == 64
    assert {(arr[i].rows_inplace, arr[i].rows_split) for i in range(64)} == {(0, 0), (0, 1), (1, 0), (1, 1)}
    assert lib.mrpie_tuning_candidates(96, 2, 0, None, 0) == _abi.MRPIE_EUNSUPPORTED
    n = C.c_size_t(0)
    assert lib.mrpie_autotune_workspace_size(256, 3, 2, 16, C.byref(n)) == 0
    assert n.value >= 2 * (768 * 768 * 8 + 3 * 256 * 256 * 8 + 16 * 256 * 256 * 4)
    assert lib.mrpie_autotune_workspace_size(256, 3, 0, 16, C.byref(n)) == _abi.MRPIE_EINVAL
    best = _abi.Tuning()
    assert lib.mrpie_autotune(256, 3, 1, 16, 2, None, 0, C.byref(best), None, None) == _abi.MRPIE_EWORKSPACE


def test_bench_refuses_more_than_one_gpu():
    """bench.py runs on one GPU: --gpus 2 prints one JSON error line and
    exits with status 2 before touching a device."""
    import json
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=root)
    assert r.returncode == 2
    line = r.stdout.strip().splitlines()[-1]
    assert "one GPU" in json.loads(line)["error"]

