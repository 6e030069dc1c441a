"""Helpers for the GPU tests: move synthetic workloads to the device and run
the HIP path through the C ABI."""
import contextlib

import numpy as np
import pytest
import torch

import oracle


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def rel_l2(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def to_dev(w, dev="cuda:0"):
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    return dict(obj=t(w.O0.copy()), probe=t(w.P0.copy()), pos=t(w.pos0.copy()), I=t(w.I))


def run_gpu(w, prm, adam=None):
    from paper_2205_04295_amd import api
    d = to_dev(w)
    T = prm.get("iterations", 1)
    err = torch.zeros(max(T, 1), dtype=torch.float32, device="cuda:0")
    status = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    ad = None if adam is None else torch.from_numpy(adam).to("cuda:0")
    api.rpie(d["obj"], d["probe"], d["pos"], d["I"], adam=ad, err=err, status=status, **prm)
    torch.cuda.synchronize()
    out = dict(O=d["obj"].cpu().numpy(), P=d["probe"].cpu().numpy(), pos=d["pos"].cpu().numpy(),
               err=err.cpu().numpy(), status=int(status.item()))
    if ad is not None:
        out["adam"] = ad.cpu().numpy()
    return out


def run_oracle(w, prm):
    return oracle.rpie64(w.O0, w.P0, w.pos0, w.I, oracle.Params(**prm))


@contextlib.contextmanager
def tuning(N, batched=False, **kw):
    """Temporarily override fields of the launch tuning of (N, batched)."""
    from paper_2205_04295_amd import tune
    saved = tune.get_tuning(N, batched)
    tune.set_tuning(N, batched, **dict(saved, **kw))
    try:
        yield
    finally:
        tune.set_tuning(N, batched, **saved)
