"""mrpie_rpie_noalloc (the sweep with its scratch in a static device array,
for callers that cannot allocate) against mrpie_rpie with a caller
workspace, called through the C ABI: two calls in a row on the same GPU, the
second with a smaller problem (the static scratch keeps the first call's
contents), each must equal mrpie_rpie's result bitwise (the same kernels on
the same inputs; the sweep is deterministic)."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_2205_04295_amd import _abi
from paper_2205_04295_amd._abi import make_params
from synth import workloads as wl

from gpu_util import need_gpu

pytestmark = pytest.mark.gpu


def _ptr(t):
    return C.c_void_p(t.data_ptr())


def _run(lib, w, prm, noalloc):
    dev = torch.device("cuda:0")
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    obj, probe, pos, I = t(w.O0.copy()), t(w.P0.copy()), t(w.pos0.copy()), t(w.I)
    T = prm["iterations"]
    err = torch.zeros(T, dtype=torch.float32, device=dev)
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    pr = make_params(**prm)
    M, N, _ = w.P0.shape
    H, W = w.O0.shape
    pb = _abi.Problem(H=H, W=W, N=N, M=M, J=w.pos0.shape[0])
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if noalloc:
        rc = lib.mrpie_rpie_noalloc(C.byref(pb), C.byref(pr), _ptr(obj), _ptr(probe), _ptr(pos), None, _ptr(I),
                                    _ptr(err), _ptr(status), stream)
    else:
        n = C.c_size_t(0)
        _abi.check(lib.mrpie_workspace_size(C.byref(pb), C.byref(pr), C.byref(n)))
        ws = torch.empty(n.value, dtype=torch.uint8, device=dev)
        rc = lib.mrpie_rpie(C.byref(pb), C.byref(pr), _ptr(obj), _ptr(probe), _ptr(pos), None, _ptr(I),
                            _ptr(err), _ptr(status), _ptr(ws), C.c_size_t(ws.numel()), stream)
    _abi.check(rc)
    torch.cuda.synchronize()
    return obj.cpu().numpy(), probe.cpu().numpy(), err.cpu().numpy(), int(status.item())


def test_noalloc_matches_workspace_call_twice_second_smaller():
    need_gpu()
    lib = _abi.load()
    # first call: 256^2 x 3 modes (row / column passes), second: 64^2 x 1
    # (one-workgroup LDS sweep), each compared with mrpie_rpie
    cases = [
        (wl.small_case(21, 384, 256, 3, 24, name="noalloc-large"), 3),
        (wl.small_case(22, 160, 64, 1, 15, name="noalloc-small"), 2),
    ]
    for w, T in cases:
        prm = dict(w.params, iterations=T)
        a = _run(lib, w, prm, noalloc=True)
        b = _run(lib, w, prm, noalloc=False)
        print(f"{w.name}: N={w.P0.shape[-1]} M={w.P0.shape[0]} J={w.pos0.shape[0]} T={T}: "
              f"max |dO| {np.max(np.abs(a[0] - b[0])):.3e} max |dP| {np.max(np.abs(a[1] - b[1])):.3e}")
        assert a[3] == b[3] == 0
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
        assert np.array_equal(a[2], b[2])


def test_noalloc_refuses_oversized_problem():
    need_gpu()
    lib = _abi.load()
    pb = _abi.Problem(H=1024, W=1024, N=256, M=8, J=1600)
    pr = make_params(iterations=1000)
    fake = C.c_void_p(0x1000)
    rc = lib.mrpie_rpie_noalloc(C.byref(pb), C.byref(pr), fake, fake, fake, None, fake, None, None, None)
    assert rc == _abi.MRPIE_EWORKSPACE
    assert b"static maximum" in lib.mrpie_last_error()
