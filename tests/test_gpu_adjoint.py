"""GPU amplitude loss and hand-written adjoint against the FP64 oracle's
analytic gradient (which the CPU suite pins to FP64 finite differences on the
same 128^2 / 32^2 / 3-mode / 25-position subset)."""
import numpy as np
import pytest
import torch

import oracle
from synth import workloads as wl

from gpu_util import need_gpu, rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def gpu_grad(O, P, pos, I, subpixel=1):
    from paper_2205_04295_amd import api
    L, gO, gP, gp = api.adjoint(dev(O), dev(P), dev(pos), dev(I), subpixel=subpixel)
    torch.cuda.synchronize()
    return float(L.item()), gO.cpu().numpy(), gP.cpu().numpy(), gp.cpu().numpy()


def subset():
    w = wl.gradient_subset(seed=3)
    O = (w.O_true * (1 + 0.05j)).astype(np.complex64)
    P = (w.P_true * 0.97).astype(np.complex64)
    pos = (w.pos0 + 0.13).astype(np.float32)
    return O, P, pos, w.I


def test_gradient_subset_matches_oracle():
    O, P, pos, I = subset()
    L, gO, gP, gp = gpu_grad(O, P, pos, I)
    Lo, gOo, gPo, gpo = oracle.loss_grad64(O.astype(complex), P.astype(complex), pos.astype(float), I.astype(float))
    print(f"loss {L:.6e} vs {Lo:.6e}; rel gO {rel_l2(gO, gOo):.2e} gP {rel_l2(gP, gPo):.2e} gpos {rel_l2(gp, gpo):.2e}")
    assert abs(L - Lo) <= 1e-5 * Lo
    assert rel_l2(gO, gOo) < 1e-4 and rel_l2(gP, gPo) < 1e-4
    assert rel_l2(gp, gpo) < 1e-3


@pytest.mark.parametrize("N,M,subpixel", [(64, 1, 1), (128, 2, 0), (256, 3, 1), (192, 5, 1), (32, 8, 0)])
def test_gradient_larger_probes(N, M, subpixel):
    w = wl.small_case(120 + N, 2 * N, N, M, 7, subpixel=bool(subpixel), name="g")
    O = w.O0.copy()
    O[N // 2:, :] = w.O_true[N // 2:, :]
    L, gO, gP, gp = gpu_grad(O, w.P0, w.pos0, w.I, subpixel)
    Lo, gOo, gPo, gpo = oracle.loss_grad64(O.astype(complex), w.P0.astype(complex), w.pos0.astype(float),
                                           w.I.astype(float), subpixel)
    assert abs(L - Lo) <= 1e-5 * Lo
    assert rel_l2(gO, gOo) < 1e-4 and rel_l2(gP, gPo) < 1e-4
    if subpixel:
        assert rel_l2(gp, gpo) < 1e-3
    else:
        assert np.all(gp == 0)


def test_adjoint_is_deterministic_and_linear():
    """Bitwise repeatable; ForwardModel.backward scales with the upstream
    gradient (G3) and equals the adjoint entry point."""
    from paper_2205_04295_amd import api
    O, P, pos, I = subset()
    a = gpu_grad(O, P, pos, I)
    b = gpu_grad(O, P, pos, I)
    assert a[0] == b[0] and all(np.array_equal(x, y) for x, y in zip(a[1:], b[1:]))
    tO, tP, tp = dev(O).requires_grad_(), dev(P).requires_grad_(), dev(pos).requires_grad_()
    Loss = api.ForwardModel.apply(tO, tP, tp, dev(I))
    (3.0 * Loss).backward()
    assert abs(float(Loss.item()) - a[0]) <= 1e-6 * a[0]
    assert np.allclose(tO.grad.cpu().numpy(), 3.0 * a[1], rtol=1e-6, atol=1e-6 * np.abs(a[1]).max())
    assert np.allclose(tP.grad.cpu().numpy(), 3.0 * a[2], rtol=1e-6, atol=1e-6 * np.abs(a[2]).max())
    assert np.allclose(tp.grad.cpu().numpy(), 3.0 * a[3], rtol=1e-6, atol=1e-6 * np.abs(a[3]).max())


def test_loss_entry_point_and_zero_at_truth():
    from paper_2205_04295_amd import api
    w = wl.gradient_subset(seed=3)
    I, scale = wl.simulate_patterns(np.random.default_rng(1), w.O_true.astype(complex),
                                    w.P_true.astype(complex), w.pos0.astype(float), 1e6, noise=False)
    P = (w.P_true.astype(complex) * np.sqrt(scale)).astype(np.complex64)
    L = api.loss(dev(w.O_true), dev(P), dev(w.pos0), dev(I))
    torch.cuda.synchronize()
    assert float(L.item()) < 1e-9 * float(I.sum())


def test_gradient_across_position_chunks():
    """300 positions: the adjoint passes take 256 positions per launch, so
    the loss, the probe-gradient sum and the scattered object gradient
    cross a chunk boundary."""
    w = wl.small_case(301, 192, 64, 2, 300, subpixel=True, name="chunks")
    O = w.O0.copy()
    L, gO, gP, gp = gpu_grad(O, w.P0, w.pos0, w.I, 1)
    Lo, gOo, gPo, gpo = oracle.loss_grad64(O.astype(complex), w.P0.astype(complex), w.pos0.astype(float),
                                           w.I.astype(float), 1)
    print(f"J=300: loss {L:.6e} vs {Lo:.6e}; gO {rel_l2(gO, gOo):.2e} gP {rel_l2(gP, gPo):.2e} "
          f"gpos {rel_l2(gp, gpo):.2e}")
    assert abs(L - Lo) <= 1e-5 * Lo
    assert rel_l2(gO, gOo) < 1e-4 and rel_l2(gP, gPo) < 1e-4
    assert rel_l2(gp, gpo) < 1e-3
    # the positions on both sides of the chunk boundary
    for j in (254, 255, 256, 257):
        assert np.linalg.norm(gp[j] - gpo[j]) <= 1e-3 * max(np.linalg.norm(gpo[j]), 1e-3 * np.abs(gpo).max())


@pytest.mark.timeout(600)
def test_gradient_full_size_across_chunks():
    """The 256^2 x 3 spiral workload's first 300 positions (1024^2 object)
    with fractional offsets: loss and gradients across the 256-position
    chunk boundary of the full-size launch shape."""
    w = wl.spiral_case(seed=1)
    J = 300
    rng = np.random.default_rng(17)
    pos = np.clip(w.pos0[:J] + rng.uniform(-0.4, 0.4, size=(J, 2)), 0, 1024 - 256).astype(np.float32)
    O, P, I = w.O0, w.P0, w.I[:J]
    L, gO, gP, gp = gpu_grad(O, P, pos, I, 1)
    Lo, gOo, gPo, gpo = oracle.loss_grad64(O.astype(complex), P.astype(complex), pos.astype(float),
                                           I.astype(float), 1)
    print(f"256^2x3, J=300: loss {L:.6e} vs {Lo:.6e}; gO {rel_l2(gO, gOo):.2e} gP {rel_l2(gP, gPo):.2e} "
          f"gpos {rel_l2(gp, gpo):.2e}")
    assert abs(L - Lo) <= 1e-5 * Lo
    assert rel_l2(gO, gOo) < 1e-4 and rel_l2(gP, gPo) < 1e-4
    assert rel_l2(gp, gpo) < 1e-3
