"""Autotuner of the sweep's launch shapes (FFT radix plan per pass, threads
per row workgroup, and, for probes whose modes fit the LDS, the
one-workgroup LDS sweep against the row / column passes).

For a given probe size N, mode count M and batch size it runs a short
synthetic sweep with every candidate shape through the C ABI, times it with
HIP events, and installs the fastest with mrpie_set_tuning.  The inputs are
random but well-conditioned; only the timing matters.
"""
from __future__ import annotations

import ctypes as C
import itertools

import torch

from . import _abi, api

CANDIDATES = [dict(rows_radix=rr, cols_radix=cr, rows_threads=th, lds_sweep=0, cols_width=cw, rows_inplace=ip)
              for rr, cr, th, cw, ip in itertools.product((4, 8), (4, 8), (256, 512), (1, 4), (0, 1))]
LDS_CANDIDATE = dict(rows_radix=8, cols_radix=8, rows_threads=256, lds_sweep=8, cols_width=1, rows_inplace=0)
_KEYS = ("rows_radix", "cols_radix", "rows_threads", "lds_sweep", "cols_width", "rows_inplace")


def lds_fits(N, M):
    """True when the M modes of an N x N probe fit the LDS together (the
    one-workgroup sweep applies)."""
    return N <= 128 and M * N * N <= 16384


def set_tuning(N, batched, rows_radix, cols_radix, rows_threads, lds_sweep=0, cols_width=1, rows_inplace=0):
    t = _abi.Tuning(rows_radix, cols_radix, rows_threads, lds_sweep, cols_width, rows_inplace)
    _abi.check(_abi.load().mrpie_set_tuning(N, int(bool(batched)), C.byref(t)))


def get_tuning(N, batched):
    t = _abi.Tuning()
    _abi.check(_abi.load().mrpie_get_tuning(N, int(bool(batched)), C.byref(t)))
    return {k: getattr(t, k) for k in _KEYS}


def _problem(N, M, J, dev, seed):
    g = torch.Generator(device="cpu").manual_seed(seed)
    H = N + 2 * N
    obj = torch.polar(torch.ones(H, H), 0.2 * torch.rand(H, H, generator=g)).to(torch.complex64).to(dev)
    probe = (torch.randn(M, N, N, generator=g) + 1j * torch.randn(M, N, N, generator=g)).to(torch.complex64).to(dev)
    pos = (torch.rand(J, 2, generator=g) * (H - N)).floor().to(torch.float32).to(dev)
    I = (torch.rand(J, N, N, generator=g) * 100).to(torch.float32).to(dev)
    return dict(obj=obj, probe=probe, pos=pos, intens=I)


def autotune(N, M, batch=1, J=64, reps=3, device="cuda:0", verbose=False):
    """Time every candidate on a synthetic (N, M) sweep of J positions with
    `batch` jobs and install the fastest.  Returns (best, {candidate: ms})."""
    dev = torch.device(device)
    jobs = [_problem(N, M, J, dev, 1234 + b) for b in range(batch)]
    batched = batch > 1
    times = {}
    cands = CANDIDATES + ([LDS_CANDIDATE] if lds_fits(N, M) else [])
    if not batched:  # the in-place option only shapes multi-job launches
        cands = [c for c in cands if not c["rows_inplace"]]
    for cand in cands:
        set_tuning(N, batched, **cand)
        best = float("inf")
        for _ in range(reps + 1):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            if batched:
                api.rpie_batched([dict(j) for j in jobs], iterations=1)
            else:
                j = jobs[0]
                api.rpie(j["obj"], j["probe"], j["pos"], j["intens"], iterations=1)
            e1.record()
            torch.cuda.synchronize()
            best = min(best, e0.elapsed_time(e1))
        times[tuple(cand.values())] = best
        if verbose:
            print(cand, f"{best:.3f} ms")
    key = min(times, key=times.get)
    best = dict(zip(_KEYS, key))
    set_tuning(N, batched, **best)
    return best, times
