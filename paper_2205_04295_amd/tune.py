"""Launch-shape tuning of the sweep: thin wrappers over the library's
autotuner (mrpie_autotune, which times every candidate on the device and
installs the fastest) and its tuning table (mrpie_set_tuning /
mrpie_get_tuning, per probe size N, mode class of M and call class).

Call classes (`batched`): 0 (or False) a single-job call, 1 (or True) a
batched call of 2 to 15 jobs, 2 a batched call of 16 or more jobs."""
from __future__ import annotations

import ctypes as C

import torch

from . import _abi

_KEYS = ("rows_radix", "cols_radix", "rows_threads", "lds_sweep", "cols_width", "rows_inplace", "rows_split")


def _as_dict(t):
    return {k: getattr(t, k) for k in _KEYS}


def candidates(N, M, batched):
    """The candidate launch shapes mrpie_autotune times, in its order."""
    lib = _abi.load()
    n = lib.mrpie_tuning_candidates(N, M, int(batched), None, 0)
    if n < 0:
        _abi.check(n)
    arr = (_abi.Tuning * n)()
    lib.mrpie_tuning_candidates(N, M, int(batched), arr, n)
    return [_as_dict(arr[i]) for i in range(n)]


# every launch shape of the row / column passes (the LDS sweep off): the
# single-sweep candidates plus the in-place and split options of batches
CANDIDATES = [dict(rows_radix=rr, cols_radix=cr, rows_threads=th, lds_sweep=0, cols_width=cw, rows_inplace=ip,
                   rows_split=sp)
              for rr in (4, 8) for cr in (4, 8) for th in (256, 512) for cw in (1, 4) for ip in (0, 1)
              for sp in (0, 1)]
LDS_CANDIDATE = dict(rows_radix=8, cols_radix=8, rows_threads=256, lds_sweep=8, cols_width=1, rows_inplace=0,
                     rows_split=0)


def call_class(jobs):
    """The tuning class of a call with `jobs` jobs (0, 1 or 2)."""
    return 0 if jobs <= 1 else 1 if jobs < 16 else 2


def lds_fits(N, M):
    """True when the M modes of an N x N probe fit the LDS together (the
    one-workgroup sweep applies)."""
    return N <= 128 and M * N * N <= 16384


def set_tuning(N, batched, rows_radix, cols_radix, rows_threads, lds_sweep=0, cols_width=1, rows_inplace=0,
               rows_split=0, M=0):
    """Install a launch shape for (N, mode class of M, batch class); M = 0
    sets every mode class."""
    t = _abi.Tuning(rows_radix, cols_radix, rows_threads, lds_sweep, cols_width, rows_inplace, rows_split)
    _abi.check(_abi.load().mrpie_set_tuning(N, M, int(batched), C.byref(t)))


def get_tuning(N, batched, M=1):
    t = _abi.Tuning()
    _abi.check(_abi.load().mrpie_get_tuning(N, M, int(batched), C.byref(t)))
    return _as_dict(t)


def autotune(N, M, batch=1, J=64, reps=3, device="cuda:0", stream=None):
    """Time every candidate launch shape on a synthetic (N, M) sweep of J
    positions with `batch` jobs (mrpie_autotune) and install the fastest.
    Returns (best, {candidate tuple: ms})."""
    lib = _abi.load()
    n = C.c_size_t(0)
    _abi.check(lib.mrpie_autotune_workspace_size(N, M, batch, J, C.byref(n)))
    ws = torch.empty(max(n.value, 1), dtype=torch.uint8, device=device)
    cands = candidates(N, M, call_class(batch))
    ms = (C.c_float * len(cands))()
    best = _abi.Tuning()
    s = torch.cuda.current_stream(device) if stream is None else stream
    _abi.check(lib.mrpie_autotune(N, M, batch, J, reps, C.c_void_p(ws.data_ptr()), C.c_size_t(ws.numel()),
                                  C.byref(best), ms, C.c_void_p(s.cuda_stream)))
    times = {tuple(c[k] for k in _KEYS): float(ms[i]) for i, c in enumerate(cands)}
    return _as_dict(best), times
