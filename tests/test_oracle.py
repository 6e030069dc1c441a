"""Pins of the FP64 oracle against facts fixed outside it (CPU only).

Each test checks the oracle against something other than itself: a brute-force
DFT, a closed form, an invariant, a textbook special case, literal values from
a hand calculation, or finite differences.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle import Params
from synth import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def dft_matrix(n):
    """Unitary DFT matrix written from the definition (no FFT library)."""
    j = np.arange(n)
    return np.exp(-2j * np.pi * np.outer(j, j) / n) / math.sqrt(n)


def brute_fft2u(x):
    F = dft_matrix(x.shape[-1])
    return F @ x @ F.T


def crandn(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


# ---------------------------------------------------------------- FFT (F1-F3)
@pytest.mark.parametrize("n", [1, 2, 3, 8, 12, 32])
def test_fft_matches_bruteforce_dft(n):
    rng = np.random.default_rng(n)
    x = crandn(rng, n, n)
    assert np.allclose(oracle.fft2u(x), brute_fft2u(x), rtol=0, atol=1e-13 * n)
    assert np.allclose(oracle.ifft2u(x), np.conj(brute_fft2u(np.conj(x))), rtol=0, atol=1e-13 * n)


def test_parseval_and_roundtrip():
    rng = np.random.default_rng(1)
    x = crandn(rng, 3, 64, 64)
    X = oracle.fft2u(x)
    assert abs(np.sum(np.abs(X) ** 2) / np.sum(np.abs(x) ** 2) - 1) < 1e-13
    assert np.max(np.abs(oracle.ifft2u(X) - x)) < 1e-13


# ------------------------------------------------------------ modulus (M1-M3)
def test_modulus_projection_invariants():
    rng = np.random.default_rng(2)
    Psi = crandn(rng, 3, 16, 16)
    Psi[:, 0, 0] = 0  # zero amplitude pixel
    I = rng.uniform(0, 5, size=(16, 16))
    I[1, 1] = -1.0    # negative counts are clamped
    Pc, A, sqI = oracle.modulus_project(Psi, I)
    S2 = np.sum(np.abs(Pc) ** 2, axis=0)
    m = np.sum(np.abs(Psi) ** 2, axis=0) > 0
    # M2: the corrected modes carry the measured intensity
    assert np.allclose(S2[m], np.maximum(I, 0)[m], atol=1e-12)
    assert np.all(Pc[:, ~m] == 0)
    # M1: idempotence
    Pc2, _, _ = oracle.modulus_project(Pc, I)
    assert np.allclose(Pc2, Pc, atol=1e-12)
    # M3: per-pixel ratios equal, real and non-negative across modes
    r = Pc[:, m] / Psi[:, m]
    assert np.allclose(r.imag, 0, atol=1e-12)
    assert np.all(r.real >= -1e-15)
    assert np.allclose(r - r[0:1], 0, atol=1e-12)


# ------------------------------------------------------- update closed forms
def _one_step(O, P, pos, I, **kw):
    prm = Params(iterations=1, **kw)
    return oracle.rpie64(O, P, pos, I, prm)


@pytest.mark.parametrize("beta,gamma", [(1.0, 1.0), (0.3, 0.7), (0.0, 0.0)])
def test_n1_closed_form(beta, gamma):
    """U1: with N = 1 the DFT is the identity, so every quantity of Eq. 5-7 is
    a scalar; two complex modes exercise the mode sums and conjugates."""
    a = 0.8 * np.exp(0.3j)
    b = np.array([1.1 * np.exp(-0.7j), 0.4 * np.exp(1.9j)])
    q = 2.5
    aP, aO = 0.6, 0.9
    S = abs(a) ** 2 * np.sum(np.abs(b) ** 2)
    kappa = math.sqrt(q) / math.sqrt(S) - 1.0
    r = _one_step(np.array([[a]]), b.reshape(2, 1, 1), np.zeros((1, 2)), np.array([[[q]]]),
                  alpha_obj=aO, alpha_probe=aP, beta=beta, gamma=gamma)
    assert np.allclose(r["P"].ravel(), b * (1 + aP * kappa), atol=1e-14)
    assert np.allclose(r["O"].ravel(), a * (1 + aO * kappa), atol=1e-14)
    # the worked example: o = P = 1, I = 4 gives P' = 1 + aP, o' = 1 + aO
    r = _one_step(np.ones((1, 1), complex), np.ones((1, 1, 1), complex), np.zeros((1, 2)),
                  np.full((1, 1, 1), 4.0), alpha_obj=aO, alpha_probe=aP, beta=beta, gamma=gamma)
    assert np.allclose(r["P"].ravel(), 1 + aP) and np.allclose(r["O"].ravel(), 1 + aO)


@pytest.mark.parametrize("beta,gamma", [(1.0, 0.1), (0.25, 0.6), (0.0, 1.0)])
def test_scaled_data_closed_form(beta, gamma):
    """U2: if I = lam^2 sum_p |D_z(P_p o)|^2 (brute-force DFT), the corrected
    waves are lam * psi, so Delta_p = (lam-1) P_p o and Eq. 5-6 reduce to
    P' = P (1 + aP (lam-1) |o|^2 / dP), o' = o (1 + aO (lam-1) sum|P|^2 / dO)."""
    rng = np.random.default_rng(3)
    N, M, lam, aP, aO = 4, 3, 1.7, 0.8, 0.6
    o = crandn(rng, N, N)
    P = crandn(rng, M, N, N)
    I = lam ** 2 * np.sum(np.abs(np.stack([brute_fft2u(P[p] * o) for p in range(M)])) ** 2, axis=0)
    r = _one_step(o, P, np.zeros((1, 2)), I[None], alpha_obj=aO, alpha_probe=aP,
                  beta=beta, gamma=gamma)
    o2 = np.abs(o) ** 2
    dP = beta * o2.max() + (1 - beta) * o2
    Ps = np.sum(np.abs(P) ** 2, axis=0)
    dO = gamma * Ps.max() + (1 - gamma) * Ps
    assert np.allclose(r["P"], P * (1 + aP * (lam - 1) * o2 / dP)[None], atol=1e-12)
    assert np.allclose(r["O"], o * (1 + aO * (lam - 1) * Ps / dO), atol=1e-12)


def test_epie_special_case():
    """U6: beta = gamma = 1 and M = 1 give the ePIE update of Maiden &
    Rodenburg (2009), whose denominators are max|o|^2 and max|P|^2."""
    rng = np.random.default_rng(4)
    N = 4
    o = crandn(rng, N, N)
    P = crandn(rng, 1, N, N)
    I = rng.uniform(0.5, 3, size=(1, N, N))
    r = _one_step(o, P, np.zeros((1, 2)), I, alpha_obj=0.7, alpha_probe=0.5, beta=1.0, gamma=1.0)
    # ePIE with a brute-force unitary DFT
    psi = P[0] * o
    Psi = brute_fft2u(psi)
    Psi_c = np.sqrt(I[0]) * np.exp(1j * np.angle(Psi))
    F = dft_matrix(N)
    psi_c = np.conj(F).T @ Psi_c @ np.conj(F)
    d = psi_c - psi
    P_e = P[0] + 0.5 * np.conj(o) * d / np.max(np.abs(o) ** 2)
    o_e = o + 0.7 * np.conj(P[0]) * d / np.max(np.abs(P[0]) ** 2)
    assert np.allclose(r["P"][0], P_e, atol=1e-12)
    assert np.allclose(r["O"], o_e, atol=1e-12)


def test_zero_denominator_and_zero_amplitude():
    """Zero probe: Eq. 6's denominator is 0 everywhere and the object must not
    move; zero data amplitude gives zero corrected waves, not NaN."""
    N = 4
    o = np.ones((N, N), complex)
    P = np.zeros((1, N, N), complex)
    I = np.ones((1, N, N))
    r = _one_step(o, P, np.zeros((1, 2)), I, beta=1.0, gamma=1.0)
    assert np.all(np.isfinite(r["O"])) and np.allclose(r["O"], o)
    assert np.all(np.isfinite(r["P"]))


# ---------------------------------------------------------- fixed point (U3)
def test_fixed_point_on_consistent_data():
    rng = np.random.default_rng(5)
    H, N, M = 12, 4, 2
    O = crandn(rng, H, H)
    P = crandn(rng, M, N, N)
    pos = np.array([[0, 0], [3, 5], [8, 8], [6, 1]], dtype=float)
    I = np.stack([np.sum(np.abs(np.stack([brute_fft2u(P[p] * O[int(y):int(y) + N, int(x):int(x) + N])
                                           for p in range(M)])) ** 2, axis=0) for y, x in pos])
    r = oracle.rpie64(O, P, pos, I, Params(iterations=3, beta=0.5, gamma=0.2))
    assert np.max(np.abs(r["O"] - O)) < 1e-12
    assert np.max(np.abs(r["P"] - P)) < 1e-12
    assert np.max(r["err"]) < 1e-24


# --------------------------------------------------------- covariance (U4/U5)
def test_scale_phase_and_translation_covariance():
    w = wl.small_case(7, 96, 32, 2, 8, name="cov")
    O, P, pos, I = (w.O0.astype(complex) * np.exp(0.2j), w.P0.astype(complex),
                    w.pos0.astype(float), w.I.astype(float))
    O = O * (1 + 0.1 * np.random.default_rng(0).standard_normal(O.shape))
    prm = Params(iterations=2, beta=0.9, gamma=0.3)
    base = oracle.rpie64(O, P, pos, I, prm)
    c = 1.7 * np.exp(0.4j)
    sc = oracle.rpie64(c * O, P / c, pos, I, prm)
    assert np.allclose(sc["O"], c * base["O"], atol=1e-9 * np.abs(base["O"]).max())
    assert np.allclose(sc["P"], base["P"] / c, atol=1e-9 * np.abs(base["P"]).max())
    # integer translation of object and scan
    O2 = np.zeros((O.shape[0] + 5, O.shape[1] + 3), complex)
    O2[5:, 3:] = O
    tr = oracle.rpie64(O2, P, pos + [5, 3], I, prm)
    assert np.allclose(tr["O"][5:, 3:], base["O"], atol=1e-10)
    assert np.allclose(tr["P"], base["P"], atol=1e-10)


# ----------------------------------------------------------- convergence (V1)
def test_monotone_error_on_noise_free_raster():
    """Noise-free raster data, probe held at the truth: the end-of-iteration
    Fourier error never increases and the object approaches the truth."""
    w = wl.raster_case(seed=0, noise=False, iterations=20)
    prm = Params(**dict(w.params, iterations=20, probe_update_start=10 ** 6))
    r = oracle.rpie64(w.O0, w.P_true, w.pos0, w.I, prm)
    e = r["err"]
    assert np.all(np.diff(e) <= 1e-12), e
    assert e[-1] < 1e-2 * e[0]
    # object error vs truth on the well-illuminated region, global phase removed
    N = w.P0.shape[-1]
    mask = np.zeros(w.O0.shape, bool)
    for y, x in w.pos0.astype(int):
        mask[y + N // 4:y + 3 * N // 4, x + N // 4:x + 3 * N // 4] = True

    def oerr(O):
        a, b = O[mask], w.O_true[mask].astype(complex)
        g = np.vdot(a, b) / np.vdot(a, a)
        return np.linalg.norm(g * a - b) / np.linalg.norm(b)
    r5 = oracle.rpie64(w.O0, w.P_true, w.pos0, w.I, Params(**dict(prm.__dict__, iterations=5)))
    assert oerr(r["O"]) < oerr(r5["O"]) < oerr(w.O0.astype(complex))


# --------------------------------------------------------------- shifts
def test_split_position_rounds_half_up():
    n, f = oracle.split_position([2.5, -0.5], 1)
    assert list(n) == [3, 0] and np.allclose(f, [-0.5, -0.5])
    n, f = oracle.split_position([2.49, 7.0], 1)
    assert list(n) == [2, 7] and np.allclose(f, [0.49, 0.0])


def test_fourier_shift_integer_and_bandlimited():
    rng = np.random.default_rng(8)
    c = crandn(rng, 16, 16)
    assert np.allclose(oracle.fourier_shift(c, (2.0, -3.0)), np.roll(c, (-2, 3), axis=(0, 1)))
    # a single Fourier mode is shifted exactly: o(r) = c(r + f)
    k = (3, -5)
    r = np.mgrid[0:16, 0:16]
    mode = lambda fy, fx: np.exp(2j * np.pi * (k[0] * (r[0] + fy) + k[1] * (r[1] + fx)) / 16)
    assert np.allclose(oracle.fourier_shift(mode(0, 0), (0.3, -0.45)), mode(0.3, -0.45))


# --------------------------------------------------------- registration (R1-R5)
def _bandlimited(rng, n, cutoff=0.35):
    x = crandn(rng, n, n)
    k = oracle.freq_grid(n) / n
    X = np.fft.fft2(x) * ((np.abs(k)[:, None] < cutoff) & (np.abs(k)[None, :] < cutoff))
    return np.fft.ifft2(X)


@pytest.mark.parametrize("norm", [0, 1])
def test_register_integer_roll(norm):
    """R1/R3: mov(r) = ref(r + s) (a circular roll by -s) returns s exactly;
    a lag of exactly N/2 is reported as +N/2."""
    rng = np.random.default_rng(9)
    ref = crandn(rng, 32, 32)
    for s in [(0, 0), (3, -5), (-7, 2), (15, 16), (-15, -1)]:
        mov = np.roll(ref, (-s[0], -s[1]), axis=(0, 1))
        sh, peak = oracle.register64(ref, mov, up=10, norm=norm)
        assert np.allclose(sh, s), (s, sh)
        assert list(peak[2:]) == [7, 7]        # window centre c = 15 // 2


@pytest.mark.parametrize("up", [20, 100])
@pytest.mark.parametrize("norm", [0, 1])
def test_register_subpixel_recovery(up, norm):
    """R2/R5: a Fourier-shifted copy with a known subpixel shift is recovered
    to within 1/up; swapping the arguments negates the shift.  The plain
    cross-power uses a band-limited patch; the phase-normalised one a
    full-band patch (phase normalisation would amplify the rounding noise
    outside a band limit to unit weight)."""
    rng = np.random.default_rng(10 + norm)
    for _ in range(4):
        ref = _bandlimited(rng, 64) if norm == 0 else crandn(rng, 64, 64)
        s = rng.uniform(-4, 4, size=2)
        mov = oracle.fourier_shift(ref, s)
        sh, _ = oracle.register64(ref, mov, up=up, norm=norm)
        assert np.all(np.abs(sh - s) <= 1.0 / up + 1e-9), (s, sh)
        sh2, _ = oracle.register64(mov, ref, up=up, norm=norm)
        assert np.all(np.abs(sh2 + s) <= 1.0 / up + 1e-9), (s, sh2)


def test_register_zero_pad_equivalence():
    """R4: the matrix-product window equals an inverse FFT of the spectrum
    zero-padded by `up` (N = 16, up = 4), sampled on the window."""
    rng = np.random.default_rng(11)
    n, up = 16, 4
    X = crandn(rng, n, n)
    s0 = (2, -3)
    C, c = oracle.upsampled_window(X, s0, up)
    L = n * up
    Z = np.zeros((L, L), complex)
    k = oracle.freq_grid(n).astype(int)
    Z[np.ix_(k % L, k % L)] = X
    Zi = np.fft.ifft2(Z) * L * L
    U = C.shape[0]
    for u in range(U):
        for v in range(U):
            m0 = (s0[0] * up + u - c) % L
            m1 = (s0[1] * up + v - c) % L
            assert abs(C[u, v] - Zi[m0, m1]) < 1e-9 * np.abs(Zi).max()


def test_register_window_geometry():
    X = np.ones((8, 8), complex)
    C, c = oracle.upsampled_window(X, (0, 0), 100)
    assert C.shape == (150, 150) and c == 75


# ------------------------------------------------------------------- Adam
def test_adam_hand_calculation():
    g = json.load(open(os.path.join(GOLDEN, "adam_three_steps.json")))
    prm = Params(adam_lr=g["lr"], adam_b1=g["b1"], adam_b2=g["b2"], adam_eps=g["eps"])
    pos = np.zeros(2)
    st = np.zeros(4)
    for t, gt in enumerate(g["g"], start=1):
        oracle.adam64(pos, st, np.array([gt, 0.0]), t, prm, (100.0, 100.0))
        pos[0] = pos[0] if pos[0] > 0 else pos[0]
        assert abs(st[0] - g["m"][t - 1]) < 1e-15 and abs(st[2] - g["v"][t - 1]) < 1e-15
        assert abs(pos[0] - g["x"][t - 1]) < 1e-12
    assert pos[1] == 0.0 and st[1] == 0.0 and st[3] == 0.0   # D2: g = 0 gives no move


def test_adam_first_step_is_sign_and_clamped():
    prm = Params(adam_lr=0.5)
    pos = np.array([10.0, 0.2])
    st = np.zeros(4)
    oracle.adam64(pos, st, np.array([3e-3, -7.0]), 1, prm, (20.0, 20.0))
    assert abs(pos[0] - 10.5) < 1e-5          # D1: lr * sign(g)
    assert pos[1] == 0.0                       # clamped at the object edge


# -------------------------------------------------------------- gradient (G1)
def _fd_check(fun, x, grad, idx, h):
    for i in idx:
        for comp in ([1.0, 1j] if np.iscomplexobj(x) else [1.0]):
            xp = x.copy(); xp.flat[i] += h * comp
            xm = x.copy(); xm.flat[i] -= h * comp
            fd = (fun(xp) - fun(xm)) / (2 * h)
            an = grad.flat[i].real if comp == 1.0 else grad.flat[i].imag
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)) + 1e-6 * np.abs(grad).max(), (i, comp, fd, an)


def test_gradient_matches_finite_differences():
    w = wl.gradient_subset(seed=3)
    O = w.O_true.astype(complex) * (1 + 0.05j)
    P = w.P_true.astype(complex) * 0.97
    pos = w.pos0.astype(float) + 0.13
    I = w.I.astype(float)
    L, gO, gP, gpos = oracle.loss_grad64(O, P, pos, I)
    rng = np.random.default_rng(0)
    so = 1e-6 * np.abs(O).max()
    cov = np.flatnonzero(np.abs(gO) > 0.05 * np.abs(gO).max())
    _fd_check(lambda z: oracle.loss_grad64(z, P, pos, I)[0], O, gO, rng.choice(cov, 6), so)
    sp = 1e-6 * np.abs(P).max()
    idx = rng.choice(np.flatnonzero(np.abs(gP) > 0.05 * np.abs(gP).max()), 6)
    _fd_check(lambda z: oracle.loss_grad64(O, z, pos, I)[0], P, gP, idx, sp)
    _fd_check(lambda z: oracle.loss_grad64(O, P, z, I)[0], pos, gpos, range(0, 50, 7), 1e-6)


def test_gradient_vanishes_at_truth_without_noise():
    """On noise-free data simulated by the virtual experiment (an independent
    scipy.fft code path) the loss and every gradient vanish at the truth."""
    w = wl.gradient_subset(seed=3)
    rng = np.random.default_rng(1)
    O = w.O_true.astype(complex)
    P = w.P_true.astype(complex)
    pos = w.pos0.astype(float)
    I, scale = wl.simulate_patterns(rng, O, P, pos, 1e6, noise=False)
    Ps = P * math.sqrt(scale)
    L, gO, gP, gpos = oracle.loss_grad64(O, Ps, pos, I.astype(float))
    ref = math.sqrt(float(np.sum(I)))
    assert L < 1e-9 * float(np.sum(I))
    assert np.abs(gO).max() < 1e-4 * ref and np.abs(gP).max() < 1e-4 * ref
    assert np.abs(gpos).max() < 1e-3 * ref
