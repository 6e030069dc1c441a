"""GPU parity of the subpixel (Fourier-shift) sweep and of XCORR_A position
refinement against the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle
from synth import workloads as wl

from gpu_util import need_gpu, rel_l2, run_gpu, run_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


SP_CASES = {
    "n64m1": dict(seed=101, H=192, N=64, M=1, J=30),
    "n128m2": dict(seed=102, H=320, N=128, M=2, J=16),
    "n192m3": dict(seed=103, H=384, N=192, M=3, J=8),
    "n256m3": dict(seed=104, H=512, N=256, M=3, J=8),
    "n32m8_rect": dict(seed=105, H=96, W=80, N=32, M=8, J=16),
    "n64m5_rect": dict(seed=106, H=160, W=224, N=64, M=5, J=20),
}


@pytest.mark.parametrize("name", list(SP_CASES))
def test_subpixel_sweep_one_iteration(name):
    w = wl.small_case(name=name, subpixel=True, **SP_CASES[name])
    prm = dict(w.params, iterations=1, subpixel=1)
    g = run_gpu(w, prm)
    o = run_oracle(w, prm)
    eo, ep = rel_l2(g["O"], o["O"]), rel_l2(g["P"], o["P"])
    print(f"{name}: rel L2 O {eo:.2e} P {ep:.2e}")
    assert g["status"] == 0
    assert eo < 1e-4 and ep < 1e-4
    assert abs(g["err"][0] - o["err"][0]) <= 1e-4 * o["err"][0]


def test_subpixel_off_equals_integer_path():
    """refine = 0, subpixel = 1 with integer positions equals the two-launch
    integer-crop sweep to rounding (the Fourier moves are identities)."""
    w = wl.small_case(name="int", **SP_CASES["n128m2"])
    a = run_gpu(w, dict(w.params, iterations=2, subpixel=0))
    b = run_gpu(w, dict(w.params, iterations=2, subpixel=1))
    assert rel_l2(b["O"], a["O"]) < 1e-5 and rel_l2(b["P"], a["P"]) < 1e-5


def test_subpixel_multi_iteration():
    w = wl.small_case(name="multi", subpixel=True, **SP_CASES["n128m2"])
    prm = dict(wl.R2_PARAMS, iterations=10, subpixel=1)
    g = run_gpu(w, prm)
    o = run_oracle(w, prm)
    assert rel_l2(g["O"], o["O"]) < 1e-3 and rel_l2(g["P"], o["P"]) < 1e-3


@pytest.mark.parametrize("subpixel,norm", [(1, 0), (0, 0), (1, 1)])
def test_refinement_one_iteration(subpixel, norm):
    """One refining iteration: the sweep itself matches the oracle; the
    measured shifts (recovered from Adam's first moment, m = (1-b1) g at
    t = 1) agree with the oracle's to the window spacing; where the shifts
    agree the positions move identically (by lr * sign(g)).  upsample = 1000
    so that the shifts of this short run are mostly non-zero (at 100 they
    round to zero)."""
    w = wl.small_case(111, 384, 128, 2, 12, subpixel=True, name="refine")
    w.pos0 = (w.pos_true + np.random.default_rng(3).normal(0, 2.0, size=w.pos_true.shape)).astype(np.float32)
    w.pos0 = np.clip(w.pos0, 0, 384 - 128).astype(np.float32)
    up = 1000
    prm = dict(w.params, iterations=1, subpixel=subpixel, refine=1, upsample=up, xcorr_norm=norm,
               adam_lr=0.5, adam_b1=0.9, adam_b2=0.999, adam_eps=1e-8)
    adam0 = np.zeros((w.pos0.shape[0], 4), np.float32)
    g = run_gpu(w, prm, adam=adam0)
    o = run_oracle(w, prm)
    assert rel_l2(g["O"], o["O"]) < 1e-4 and rel_l2(g["P"], o["P"]) < 1e-4
    g_gpu = g["adam"][:, :2].astype(np.float64) / (1 - np.float32(0.9))
    g_orc = o["adam"][:, :2] / (1 - 0.9)
    assert np.mean(g_orc != 0) > 0.5                      # the run does exercise the controller
    diff = np.abs(g_gpu - g_orc)
    print("shifts gpu", np.round(g_gpu[:4], 4).tolist(), "oracle", np.round(g_orc[:4], 4).tolist())
    assert np.mean(diff <= 1.01 / up) >= 0.75 and diff.max() < 0.01
    same = np.abs(g_gpu - g_orc) < 0.5 / up
    moved = np.abs(g["pos"] - w.pos0) > 0.4
    assert np.any(moved)
    assert np.allclose(g["pos"][same], o["pos"][same], atol=1e-3)


FRESH = r"""
import sys, numpy as np
sys.path.insert(0, {root!r}); sys.path.insert(0, {tests!r})
from synth import workloads as wl
from gpu_util import run_gpu, run_oracle, rel_l2
w = wl.small_case(name='fresh', subpixel=True, seed=102, H=320, N=128, M=2, J=4)
prm = dict(w.params, iterations=1, subpixel=1, refine={refine}, upsample=20)
adam = np.zeros((4, 4), np.float32) if {refine} else None
g = run_gpu(w, prm, adam=adam); o = run_oracle(w, prm)
e = max(rel_l2(g['O'], o['O']), rel_l2(g['P'], o['P']))
print('REL', e)
sys.exit(0 if e < 1e-4 else 1)
"""


@pytest.mark.parametrize("refine", [0, 1])
def test_subpixel_sweep_as_first_call_of_a_process(refine):
    """Regression: every library entry point initialises the constant tables
    of the kernels it launches, also when it is the first call a process
    makes (a missing initialisation used to pass only after another entry
    point had run)."""
    import os
    import subprocess
    import sys
    tests = os.path.dirname(os.path.abspath(__file__))
    code = FRESH.format(root=os.path.dirname(tests), tests=tests, refine=refine)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=110)
    print(r.stdout[-500:], r.stderr[-500:])
    assert r.returncode == 0
