"""Thin torch-facing wrappers over the libmrpie C ABI.

torch provides device memory and the current stream; every computation runs
in the HIP library.  Functions take CUDA (HIP) tensors and pass their data
pointers; they raise if the library is missing or a tensor is not on the GPU.
"""
from __future__ import annotations

import ctypes as C

import torch

from . import _abi
from ._abi import Problem, check, make_params


def _dev(t, dtype, name):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return C.c_void_p(t.data_ptr())


def _opt(t, dtype, name):
    return C.c_void_p(None) if t is None else _dev(t, dtype, name)


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def problem_of(obj, probe, pos):
    M, N, _ = probe.shape
    H, W = obj.shape
    return Problem(H=H, W=W, N=N, M=M, J=pos.shape[0])


def workspace_size(problem: Problem, params) -> int:
    lib = _abi.load()
    n = C.c_size_t(0)
    check(lib.mrpie_workspace_size(C.byref(problem), C.byref(params), C.byref(n)))
    return n.value


def rpie(obj, probe, pos, intens, adam=None, err=None, status=None, workspace=None, stream=None, **params):
    """Run the M-rPIE sweep in place on (obj, probe[, pos, adam]).

    obj [H, W] complex64, probe [M, N, N] complex64, pos [J, 2] float32,
    intens [J, N, N] float32 (FFT order), all on the GPU.  Keyword arguments
    are the fields of mrpie_params.  Returns the workspace tensor used (it
    can be passed back in to avoid a new allocation).
    """
    lib = _abi.load()
    prm = make_params(**params)
    pb = problem_of(obj, probe, pos)
    nbytes = workspace_size(pb, prm)
    if workspace is None or workspace.numel() < nbytes:
        workspace = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=obj.device)
    check(lib.mrpie_rpie(C.byref(pb), C.byref(prm), _dev(obj, torch.complex64, "obj"),
                         _dev(probe, torch.complex64, "probe"), _dev(pos, torch.float32, "pos"),
                         _opt(adam, torch.float32, "adam"), _dev(intens, torch.float32, "intens"),
                         _opt(err, torch.float32, "err"), _opt(status, torch.int32, "status"),
                         _dev(workspace, torch.uint8, "workspace"), C.c_size_t(workspace.numel()),
                         _stream(stream)))
    return workspace


def rpie_batched(jobs, stream=None, tuning=None, **params):
    """Run independent M-rPIE reconstructions lock-step in shared launches.

    jobs: list of dicts with GPU tensors obj, probe, pos, intens and optional
    err, status, workspace.  Keyword arguments are the shared mrpie_params;
    `tuning` (a dict of mrpie_tuning fields, optional) fixes the launch shape
    of this call.  Returns the list of workspaces used."""
    lib = _abi.load()
    prm = make_params(**params)
    arr = (_abi.Job * len(jobs))()
    keep = []
    for b, j in enumerate(jobs):
        pb = problem_of(j["obj"], j["probe"], j["pos"])
        nbytes = workspace_size(pb, prm)
        ws = j.get("workspace")
        if ws is None or ws.numel() < nbytes:
            ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=j["obj"].device)
        keep.append(ws)
        arr[b] = _abi.Job(pb, _dev(j["obj"], torch.complex64, "obj"), _dev(j["probe"], torch.complex64, "probe"),
                          _dev(j["pos"], torch.float32, "pos"), _dev(j["intens"], torch.float32, "intens"),
                          _opt(j.get("err"), torch.float32, "err"), _opt(j.get("status"), torch.int32, "status"),
                          _dev(ws, torch.uint8, "workspace"), C.c_size_t(ws.numel()))
    tu = None if tuning is None else C.byref(_abi.Tuning(**tuning))
    check(lib.mrpie_rpie_batched(len(jobs), C.cast(arr, C.c_void_p), C.byref(prm), tu, _stream(stream)))
    return keep


def register(ref, mov, upsample=100, norm=0, workspace=None, stream=None):
    """Subpixel registration of pairs ref[b], mov[b] ([B, N, N] complex64).
    Returns (shift [B, 2] float32, peak [B, 4] int32) on the GPU."""
    lib = _abi.load()
    B, N, _ = ref.shape
    if mov.shape != ref.shape:
        raise ValueError("ref and mov shapes differ")
    n = C.c_size_t(0)
    check(lib.mrpie_register_workspace_size(N, B, upsample, C.byref(n)))
    if workspace is None or workspace.numel() < n.value:
        workspace = torch.empty(n.value, dtype=torch.uint8, device=ref.device)
    shift = torch.empty(B, 2, dtype=torch.float32, device=ref.device)
    peak = torch.empty(B, 4, dtype=torch.int32, device=ref.device)
    check(lib.mrpie_register(N, B, _dev(ref, torch.complex64, "ref"), _dev(mov, torch.complex64, "mov"),
                             upsample, norm, _dev(shift, torch.float32, "shift"), _dev(peak, torch.int32, "peak"),
                             _dev(workspace, torch.uint8, "workspace"), C.c_size_t(workspace.numel()),
                             _stream(stream)))
    return shift, peak


def adam(pos, state, g, t, bounds, stream=None, **params):
    """Alg. 1 step in place on pos [J, 2] and state [J, 4] with gradient g [J, 2]."""
    lib = _abi.load()
    prm = make_params(**params)
    check(lib.mrpie_adam(pos.shape[0], C.byref(prm), int(bounds[0]), int(bounds[1]),
                         _dev(pos, torch.float32, "pos"), _dev(state, torch.float32, "state"),
                         _dev(g, torch.float32, "g"), int(t), _stream(stream)))
    return pos, state


def _grad_ws(pb, device, workspace):
    lib = _abi.load()
    n = C.c_size_t(0)
    check(lib.mrpie_grad_workspace_size(C.byref(pb), C.byref(n)))
    if workspace is None or workspace.numel() < n.value:
        workspace = torch.empty(n.value, dtype=torch.uint8, device=device)
    return workspace


def loss(obj, probe, pos, intens, subpixel=1, workspace=None, stream=None):
    """Amplitude loss (float64 GPU scalar tensor) of the forward model."""
    lib = _abi.load()
    pb = problem_of(obj, probe, pos)
    ws = _grad_ws(pb, obj.device, workspace)
    out = torch.empty((), dtype=torch.float64, device=obj.device)
    check(lib.mrpie_loss(C.byref(pb), int(subpixel), _dev(obj, torch.complex64, "obj"),
                         _dev(probe, torch.complex64, "probe"), _dev(pos, torch.float32, "pos"),
                         _dev(intens, torch.float32, "intens"), C.c_void_p(out.data_ptr()), C.c_void_p(None),
                         _dev(ws, torch.uint8, "workspace"), C.c_size_t(ws.numel()), _stream(stream)))
    return out


def adjoint(obj, probe, pos, intens, subpixel=1, workspace=None, stream=None):
    """(loss, grad_obj, grad_probe, grad_pos) of the amplitude loss."""
    lib = _abi.load()
    pb = problem_of(obj, probe, pos)
    ws = _grad_ws(pb, obj.device, workspace)
    out = torch.empty((), dtype=torch.float64, device=obj.device)
    gO = torch.empty_like(obj)
    gP = torch.empty_like(probe)
    gp = torch.empty_like(pos)
    check(lib.mrpie_adjoint(C.byref(pb), int(subpixel), _dev(obj, torch.complex64, "obj"),
                            _dev(probe, torch.complex64, "probe"), _dev(pos, torch.float32, "pos"),
                            _dev(intens, torch.float32, "intens"), C.c_void_p(out.data_ptr()),
                            _dev(gO, torch.complex64, "grad_obj"), _dev(gP, torch.complex64, "grad_probe"),
                            _dev(gp, torch.float32, "grad_pos"), C.c_void_p(None),
                            _dev(ws, torch.uint8, "workspace"), C.c_size_t(ws.numel()), _stream(stream)))
    return out, gO, gP, gp


class ForwardModel(torch.autograd.Function):
    """Amplitude loss of the mixed-state far-field model as an autograd
    Function: forward runs the HIP loss passes, backward the HIP adjoint
    (which recomputes the exit waves instead of saving them).

    ForwardModel.apply(obj, probe, pos, intens[, subpixel]) -> scalar loss.
    """

    @staticmethod
    def forward(ctx, obj, probe, pos, intens, subpixel=1):
        obj_c, probe_c, pos_c = obj.detach().contiguous(), probe.detach().contiguous(), pos.detach().contiguous()
        ctx.save_for_backward(obj_c, probe_c, pos_c, intens)
        ctx.subpixel = subpixel
        return loss(obj_c, probe_c, pos_c, intens, subpixel).to(torch.float32)

    @staticmethod
    def backward(ctx, g):
        obj, probe, pos, intens = ctx.saved_tensors
        _, gO, gP, gp = adjoint(obj, probe, pos, intens, ctx.subpixel)
        g = g.to(torch.float32)
        return gO * g, gP * g, gp * g, None, None


def fft2(x, inverse=False, stream=None):
    """In-place unitary 2-D DFT of x [..., N, N] complex64 (test hook)."""
    lib = _abi.load()
    N = x.shape[-1]
    B = x.numel() // (N * N)
    check(lib.mrpie_fft2(N, B, _dev(x, torch.complex64, "x"), int(bool(inverse)), _stream(stream)))
    return x


def modulus(psi, intens, stream=None):
    """In-place modulus replacement (Eq. 7) of psi [M, N, N] by intens [N, N]."""
    lib = _abi.load()
    M, N, _ = psi.shape
    check(lib.mrpie_modulus(N, M, _dev(psi, torch.complex64, "psi"), _dev(intens, torch.float32, "intens"),
                            _stream(stream)))
    return psi


def canvas(probe, pos, H, W, status=None, stream=None):
    """Canvas map [H, W] float32: sum over positions of sum_p |P_p|^2 placed
    at each box corner (how strongly each object pixel is illuminated)."""
    lib = _abi.load()
    M, N, _ = probe.shape
    pb = Problem(H=H, W=W, N=N, M=M, J=pos.shape[0])
    n = C.c_size_t(0)
    check(lib.mrpie_canvas_workspace_size(N, C.byref(n)))
    ws = torch.empty(n.value, dtype=torch.uint8, device=probe.device)
    out = torch.empty(H, W, dtype=torch.float32, device=probe.device)
    check(lib.mrpie_canvas(C.byref(pb), _dev(probe, torch.complex64, "probe"), _dev(pos, torch.float32, "pos"),
                           _dev(out, torch.float32, "canvas"), _opt(status, torch.int32, "status"),
                           _dev(ws, torch.uint8, "workspace"), C.c_size_t(ws.numel()), _stream(stream)))
    return out


def validate(problem: Problem, **params) -> int:
    """Host-only validation; returns the C return code (0 = OK)."""
    lib = _abi.load()
    prm = make_params(**params)
    return lib.mrpie_validate(C.byref(problem), C.byref(prm))


TIMED_KERNELS = ("k_rows", "k_cols", "k_reg_cols", "k_reg_gemm1", "k_adj_p3", "k_lds_sweep", "k_upd", "k_gat")


def timing_enable(stride: int):
    """Sample every `stride`-th launch of each timed kernel with HIP events."""
    check(_abi.load().mrpie_timing_enable(int(stride)))


def timing_read():
    """{kernel: (mean ms, launches timed, mean grid.y of the timed launches)}
    since timing_enable; clears."""
    n = len(TIMED_KERNELS)
    avg = (C.c_double * n)()
    cnt = (C.c_int64 * n)()
    units = (C.c_double * n)()
    check(_abi.load().mrpie_timing_read(avg, cnt, units, n))
    return {k: (avg[i], cnt[i], units[i]) for i, k in enumerate(TIMED_KERNELS)}
