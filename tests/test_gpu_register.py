"""GPU registration and Adam against the FP64 oracle.

Teacher forcing: both sides register the very same complex64 patches (the
oracle upcasts them), so the integer peaks (coarse lag and upsampled-window
argmax) must be identical and the shifts equal to float rounding."""
import numpy as np
import pytest
import torch

import oracle
from synth import workloads as wl

from gpu_util import need_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def crandn(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def pairs_shifted(rng, B, N, max_shift=5.0, noise=0.05):
    ref = crandn(rng, B, N, N)
    mov = np.empty_like(ref)
    s = rng.uniform(-max_shift, max_shift, size=(B, 2))
    for b in range(B):
        mov[b] = oracle.fourier_shift(ref[b], s[b]) + noise * crandn(rng, N, N)
    return ref.astype(np.complex64), mov.astype(np.complex64), s


def gpu_register(ref, mov, up, norm):
    from paper_2205_04295_amd import api
    sh, pk = api.register(torch.from_numpy(ref).cuda(), torch.from_numpy(mov).cuda(), upsample=up, norm=norm)
    torch.cuda.synchronize()
    return sh.cpu().numpy(), pk.cpu().numpy()


@pytest.mark.parametrize("N", [64, 128, 192, 256])
@pytest.mark.parametrize("norm", [0, 1])
def test_register_peaks_exact(N, norm):
    rng = np.random.default_rng(N + norm)
    B = 6
    ref, mov, s = pairs_shifted(rng, B, N)
    up = 100
    sh, pk = gpu_register(ref, mov, up, norm)
    for b in range(B):
        so, po = oracle.register64(ref[b].astype(np.complex128), mov[b].astype(np.complex128), up, norm)
        assert list(pk[b]) == list(po), (b, pk[b], po)
        assert np.allclose(sh[b], so, atol=1e-5)
        if norm == 1:
            assert np.all(np.abs(sh[b] - s[b]) < 0.05)


@pytest.mark.parametrize("up", [1, 4, 10, 37])
def test_register_other_upsampling_and_integer_rolls(up):
    rng = np.random.default_rng(up)
    N = 64
    ref = crandn(rng, 4, N, N).astype(np.complex64)
    shifts = [(0, 0), (5, -7), (-31, 32), (32, 1)]
    mov = np.stack([np.roll(ref[b], (-shifts[b][0], -shifts[b][1]), axis=(0, 1)) for b in range(4)])
    sh, pk = gpu_register(ref, mov, up, 1)
    for b in range(4):
        so, po = oracle.register64(ref[b].astype(np.complex128), mov[b].astype(np.complex128), up, 1)
        assert list(pk[b]) == list(po)
        assert np.allclose(sh[b], so, atol=1e-6)
    assert np.allclose(sh[0], 0) and np.allclose(sh[1], (5, -7)) and np.allclose(sh[2], (-31, 32))
    assert np.allclose(sh[3], (32, 1))   # a lag of exactly N/2 is reported as +N/2


@pytest.mark.parametrize("norm", [0, 1])
def test_register_rpie_patches_teacher_forced(norm):
    """The pairs XCORR_A registers inside a refining reconstruction: a patch
    before and after its M-rPIE update (oracle step on spiral-scan data),
    with the plain cross-power (the refinement default) and phase
    normalisation."""
    w = wl.small_case(91, 512, 256, 3, 6, subpixel=True, name="reg")
    prm = oracle.Params(**dict(w.params, iterations=1, subpixel=1, refine=1, xcorr_norm=norm))
    rec = []
    oracle.rpie64(w.O0, w.P0, w.pos0, w.I, prm, record=rec)
    ref = np.stack([r[2] for r in rec]).astype(np.complex64)
    mov = np.stack([r[3] for r in rec]).astype(np.complex64)
    sh, pk = gpu_register(ref, mov, 100, norm)
    for b in range(len(rec)):
        so, po = oracle.register64(ref[b].astype(np.complex128), mov[b].astype(np.complex128), 100, norm)
        assert list(pk[b]) == list(po)
        assert np.allclose(sh[b], so, atol=1e-5)


def test_register_empty_and_zero_inputs():
    from paper_2205_04295_amd import api
    z = torch.zeros(0, 64, 64, dtype=torch.complex64, device="cuda")
    sh, pk = api.register(z, z)
    assert sh.shape == (0, 2)
    # all-zero pair: cross-power 0 everywhere -> first maximum is lag 0, window centre
    ref = np.zeros((1, 64, 64), np.complex64)
    sh, pk = gpu_register(ref, ref, 20, 1)
    so, po = oracle.register64(ref[0].astype(complex), ref[0].astype(complex), 20, 1)
    assert list(pk[0]) == list(po) and np.allclose(sh[0], so)


def test_adam_matches_oracle():
    from paper_2205_04295_amd import api
    rng = np.random.default_rng(5)
    J = 1000
    pos = rng.uniform(0, 100, size=(J, 2)).astype(np.float32)
    pos[:3] = [[0.1, 99.9], [50, 50], [0, 0]]
    st = np.zeros((J, 4), np.float32)
    # the C ABI carries the hyper-parameters as float32: feed the oracle the same values
    f32 = lambda v: float(np.float32(v))
    prm = oracle.Params(adam_lr=f32(0.5), adam_b1=f32(0.9), adam_b2=f32(0.999), adam_eps=f32(1e-8))
    tp, ts = torch.from_numpy(pos.copy()).cuda(), torch.from_numpy(st.copy()).cuda()
    po, so = pos.astype(np.float64), st.astype(np.float64)
    for t in range(1, 5):
        g = rng.normal(0, 2, size=(J, 2)).astype(np.float32)
        g[5] = 0.0
        api.adam(tp, ts, torch.from_numpy(g).cuda(), t, (100, 100), adam_lr=0.5, adam_b1=0.9,
                 adam_b2=0.999, adam_eps=1e-8)
        for j in range(J):
            oracle.adam64(po[j], so[j], g[j].astype(np.float64), t, prm, (100.0, 100.0))
        torch.cuda.synchronize()
        assert np.allclose(tp.cpu().numpy(), po, atol=1e-4)
        assert np.allclose(ts.cpu().numpy(), so, rtol=1e-5, atol=1e-7)


@pytest.mark.parametrize("N,up", [(256, 1000), (128, 500)])
def test_register_peaks_exact_large_windows(N, up):
    """Upsampling factors whose window (U = ceil(1.5 up) > 320 lags) takes
    the GEMMs' 64 x 64 output tiles: peaks equal the oracle's."""
    rng = np.random.default_rng(N + up)
    B = 3
    ref, mov, s = pairs_shifted(rng, B, N, noise=0.1)
    sh, pk = gpu_register(ref, mov, up, 0)
    for b in range(B):
        so, po = oracle.register64(ref[b].astype(np.complex128), mov[b].astype(np.complex128), up, 0)
        assert list(pk[b]) == list(po), (b, pk[b], po)
        assert np.allclose(sh[b], so, atol=1e-6)


@pytest.mark.parametrize("norm", [0, 1])
def test_register_across_pair_chunks(norm):
    """300 pairs: the registration passes take 256 pairs per launch, so the
    batch crosses a chunk boundary; every pair's peaks equal the oracle's."""
    rng = np.random.default_rng(300 + norm)
    B, N, up = 300, 64, 100
    ref, mov, s = pairs_shifted(rng, B, N, noise=0.1)
    sh, pk = gpu_register(ref, mov, up, norm)
    bad = []
    for b in range(B):
        so, po = oracle.register64(ref[b].astype(np.complex128), mov[b].astype(np.complex128), up, norm)
        if list(pk[b]) != list(po) or not np.allclose(sh[b], so, atol=1e-5):
            bad.append((b, pk[b].tolist(), po.tolist()))
    assert not bad, bad[:5]
