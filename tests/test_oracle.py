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


# ------------------------------------------------- planted mistakes (CPU only)
ORACLE_SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "mrpie64.py")


def mutated_oracle(old, new):
    """A copy of the oracle module with one planted mistake (`old` replaced
    by `new` in its source), compiled in a fresh namespace.  Used to show
    that a pin fails on the mistake it is meant to catch."""
    import sys
    import types
    src = open(ORACLE_SRC).read()
    assert src.count(old) == 1, old
    mod = types.ModuleType("oracle_mutant")
    sys.modules["oracle_mutant"] = mod      # dataclasses resolve annotations through it
    try:
        exec(compile(src.replace(old, new), "oracle_mutant", "exec"), mod.__dict__)
    finally:
        del sys.modules["oracle_mutant"]
    return mod.__dict__


# ------------------------------------------------------ subpixel (R-crop)
def test_subpixel_on_integer_positions_equals_integer_crop():
    """With every position an integer, the Fourier move has f = 0 and the
    subpixel sweep must be the integer-crop sweep, bit for bit."""
    w = wl.small_case(21, 96, 32, 2, 9, name="int")
    a = oracle.rpie64(w.O0, w.P0, w.pos0, w.I, Params(**dict(w.params, iterations=2, subpixel=0)))
    b = oracle.rpie64(w.O0, w.P0, w.pos0, w.I, Params(**dict(w.params, iterations=2, subpixel=1)))
    assert np.array_equal(a["O"], b["O"]) and np.array_equal(a["P"], b["P"])


def _subpixel_errors(mod, w):
    prm = mod["Params"](**dict(w.params, iterations=20, subpixel=1, probe_update_start=10 ** 6))
    return mod["rpie64"](w.O0, w.P_true, w.pos0, w.I, prm)["err"]


def _subpixel_pin_holds(e):
    return bool(np.all(np.diff(e) <= 1e-12) and e[-1] < 1e-2 * e[0])


def test_subpixel_monotone_on_fractional_raster():
    """Noise-free data at continuous (fractional) stage positions, probe
    frozen at the truth: with the Fourier move of the crop (o(r) =
    O(n + r + f)) and the update moved back by -f, the end-of-iteration
    error never increases and ends below 1e-2 of the first.  Catches a
    back-move by +f (the updates land 2f away and the error diverges), a
    crop moved by -f, and an integer crop (the data's fractions ignored)."""
    w = wl.raster_case(seed=0, H=128, N=32, R=10.0, nside=6, step=12.0, origin=16.0, noise=False,
                       fractional=True)
    assert np.any(np.abs(w.pos0 - np.round(w.pos0)) > 0.1)
    assert _subpixel_pin_holds(_subpixel_errors(vars(oracle.mrpie64), w))
    for old, new in [("O[box] = O[box] + fourier_shift(d_o, -f)", "O[box] = O[box] + fourier_shift(d_o, f)"),
                     ("o = fourier_shift(O[box], f)\n            d_o",
                      "o = fourier_shift(O[box], -f)\n            d_o"),
                     ("f = pos - n if subpixel else", "f = 0 * pos if subpixel else")]:
        assert not _subpixel_pin_holds(_subpixel_errors(mutated_oracle(old, new), w)), new


# ------------------------------------------------------------ probe carry
def test_probe_carried_between_positions_n1_closed_form():
    """Eq. 5 is applied position by position: the second position's update
    uses the probe the first one produced.  N = 1 (the DFT is the
    identity), two object pixels a1, a2 visited in turn with intensities
    q1, q2: kappa_j = sqrt(q_j) / (|a_j| |P_{j-1}|) - 1, P_j = P_{j-1} (1 +
    aP kappa_j), a_j' = a_j (1 + aO kappa_j).  Using the initial probe at the
    second position (no carry) gives a different kappa_2."""
    a1, a2, b = 0.9 * np.exp(0.4j), 1.3 * np.exp(-1.1j), 0.7 * np.exp(0.25j)
    q1, q2, aP, aO = 2.0, 0.6, 0.8, 0.5
    O = np.array([[a1, 0], [0, a2]])
    r = _one_step(O, np.array([[[b]]]), np.array([[0.0, 0.0], [1.0, 1.0]]), np.array([[[q1]], [[q2]]]),
                  alpha_obj=aO, alpha_probe=aP, beta=0.5, gamma=0.5)
    k1 = math.sqrt(q1) / (abs(a1) * abs(b)) - 1
    P1 = b * (1 + aP * k1)
    k2 = math.sqrt(q2) / (abs(a2) * abs(P1)) - 1
    P2 = P1 * (1 + aP * k2)
    assert abs(r["P"][0, 0, 0] - P2) < 1e-14
    assert abs(r["O"][0, 0] - a1 * (1 + aO * k1)) < 1e-14 and abs(r["O"][1, 1] - a2 * (1 + aO * k2)) < 1e-14
    k2_nocarry = math.sqrt(q2) / (abs(a2) * abs(b)) - 1
    assert abs(k2 - k2_nocarry) > 0.1


# --------------------------------------------------- refinement (XCORR_A)
def _refine_case(seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    N, H = 32, 128
    O = wl.object_field(rng, H, H)
    P = wl.probe_modes(N, 8.0, 1)
    true = np.floor(wl.raster_scan(rng, 5, 12.0, 24.0, 1.0) + 0.5)
    I, scale = wl.simulate_patterns(rng, O, P, true, 1e6, noise=False)
    start = true + rng.choice([-1.5, 1.5], size=true.shape) * rng.uniform(0.6, 1.0, size=true.shape)
    return wl._finish("refine_pin", O, P, true, start, I, scale, 8.0, dict(wl.R1_PARAMS), seed=seed)


def _rms(p, t):
    d = np.asarray(p, float) - np.asarray(t, float)
    return float(np.sqrt(np.mean(np.sum(d * d, axis=1))))


@pytest.mark.parametrize("seed", [5, 6])
def test_refinement_xcorr_a_moves_positions_toward_truth(seed):
    """Noise-free data at integer true positions, estimates off by 0.9-1.5
    px per axis, object and probe started at the truth (probe frozen):
    XCORR_A (the patch against its own update) with Adam (lr 0.25, up 100)
    more than halves the position RMS in 20 iterations.  With ref and mov
    swapped (the sign of Eq. 8-9 reversed) the positions run away."""
    w = _refine_case(seed)
    prm = dict(w.params, iterations=20, subpixel=1, refine=1, refine_start=0, upsample=100, adam_lr=0.25,
               probe_update_start=10 ** 6)
    r0 = _rms(w.pos0, w.pos_true)
    r = oracle.rpie64(w.O_true, w.P_true, w.pos0, w.I, Params(**prm))
    assert _rms(r["pos"], w.pos_true) < 0.5 * r0
    m = mutated_oracle("ref, mov = (o, o + d_o) if", "ref, mov = (o + d_o, o) if")
    r2 = m["rpie64"](w.O_true, w.P_true, w.pos0, w.I, m["Params"](**prm))
    assert _rms(r2["pos"], w.pos_true) > 2.0 * r0


def test_refinement_waits_for_refine_start():
    """Positions do not move in iterations before refine_start (also when
    resuming with iter_offset) and the Adam state stays zero."""
    w = _refine_case(5)
    prm = dict(w.params, iterations=3, subpixel=1, refine=1, refine_start=4, upsample=100, adam_lr=0.25)
    r = oracle.rpie64(w.O_true, w.P_true, w.pos0, w.I, Params(**prm))
    assert np.array_equal(r["pos"], w.pos0.astype(float)) and not np.any(r["adam"])
    r = oracle.rpie64(w.O_true, w.P_true, w.pos0, w.I, Params(**dict(prm, iterations=1, iter_offset=4)))
    assert not np.array_equal(r["pos"], w.pos0.astype(float))


# ---------------------------------------------------------- XCORR_B (R-xcb)
def _periodic_flat_case(prop, nf, refine_start=0, xcorr_point=1):
    """An object that repeats with the probe's period N (so every N x N crop
    is a circular shift of one pattern) under a constant probe: the model of
    a box at the wrong corner is exactly the truth's pattern circularly
    shifted by the error e, in the object plane and, D_z being a circular
    convolution, at the detector."""
    rng = np.random.default_rng(0)
    N, H = 32, 96
    base = rng.uniform(0.5, 1.0, (N, N)) * np.exp(1j * rng.uniform(-1, 1, (N, N)))
    O = np.tile(base, (H // N, H // N))
    P = np.full((1, N, N), 1.7 + 0.4j)
    true = np.array([[20., 30.], [33., 41.], [50., 17.], [40., 40.]])
    e = np.array([[1, -2], [0, 1], [-1, -1], [2, 0]], float)
    prm = Params(alpha_obj=0.0, alpha_probe=0.0, iterations=refine_start + 1, refine=1, refine_start=refine_start,
                 xcorr_point=xcorr_point, upsample=10, adam_lr=0.5, propagator=prop, fresnel=nf)
    I = np.stack([oracle.forward_intensity64(P, O[int(y):int(y) + N, int(x):int(x) + N], prm) for y, x in true])
    return O, P, true - e, I, e, prm


@pytest.mark.parametrize("nf", [40.0, 300.0])
def test_xcorr_b_recovers_integer_error_near_field(nf):
    """Near field, the periodic object under a flat probe, updates off (alpha
    = 0): XCORR_B registers the model amplitude against the measured one and
    finds exactly the error e (truth minus estimate), so the first Adam step
    (t = 1 in the first refining iteration, refine_start = 1) moves every
    axis by lr e / (|e| + eps), i.e. +-lr toward the truth.  A swapped
    ref / mov moves away; Adam's t counted from iteration 0 (t = 2) gives a
    shorter step."""
    O, P, start, I, e, prm = _periodic_flat_case(1, nf, refine_start=1)
    rec = []
    r = oracle.rpie64(O, P, start, I, prm, record=rec)
    want = prm.adam_lr * e / (np.abs(e) + prm.adam_eps)
    assert np.max(np.abs(r["pos"] - start - want)) < 1e-12
    assert len(rec) == 4 and all(it == 1 for it, _, _, _ in rec)
    m = mutated_oracle("ref, mov = (o, o + d_o) if prm.xcorr_point == 0 else (A, sqI)",
                       "ref, mov = (o, o + d_o) if prm.xcorr_point == 0 else (sqI, A)")
    r2 = m["rpie64"](O, P, start, I, m["Params"](**prm.__dict__))
    assert np.max(np.abs(r2["pos"] - start + want)) < 1e-12
    m = mutated_oracle("adam64(pos[j], adam[j], s, it - prm.refine_start + 1, prm, bounds)",
                       "adam64(pos[j], adam[j], s, it + 1, prm, bounds)")
    r3 = m["rpie64"](O, P, start, I, m["Params"](**prm.__dict__))
    assert np.max(np.abs(r3["pos"] - start - want)) > 0.1


def test_xcorr_b_is_blind_in_the_far_field_under_a_flat_probe():
    """The far-field amplitude of a translated patch is the same amplitude:
    XCORR_B measures no shift and the positions stay (the paper's argument
    for XCORR_A: the detector-plane signal carries less of the error)."""
    O, P, start, I, e, prm = _periodic_flat_case(0, 0.0)
    r = oracle.rpie64(O, P, start, I, prm)
    assert np.array_equal(r["pos"], start)


def test_xcorr_a_sees_the_error_where_xcorr_b_is_blind():
    """Same far-field flat-probe data with the updates on: XCORR_A's pair
    (o, o') is unchanged too (the modulus constraint is already met), so
    neither point can see a translation under a flat probe — the probe's
    structure is what makes the position observable."""
    O, P, start, I, e, prm = _periodic_flat_case(0, 0.0, xcorr_point=0)
    prm.alpha_obj = prm.alpha_probe = 1.0
    r = oracle.rpie64(O, P, start, I, prm)
    assert np.max(np.abs(r["pos"] - start)) < 1e-9


# ------------------------------------------------------ near field (R-near)
def _gauss_closed_form(N, w0, nf):
    """Fresnel propagation of exp(-(y^2 + x^2) / w0^2) (centred on the
    window) written from the textbook Gaussian-beam result: per axis
    sqrt(q0 / q) exp(-x^2 / q) with q = w0^2 + i lambda z / pi, and lambda z
    = N^2 / N_F in pixel units (delta = 1)."""
    x = np.arange(N) - N // 2
    q = w0 ** 2 + 1j * N ** 2 / (math.pi * nf)
    u = np.sqrt(w0 ** 2 / q) * np.exp(-x ** 2 / q)
    return np.outer(u, u)


@pytest.mark.parametrize("nf", [188.0, 400.0, 1000.0])
def test_fresnel_propagator_gaussian_beam(nf):
    N, w0 = 128, 4.0
    x = np.arange(N) - N // 2
    u0 = np.outer(np.exp(-x ** 2 / w0 ** 2), np.exp(-x ** 2 / w0 ** 2))
    prm = Params(propagator=1, fresnel=nf)
    got = oracle.propagate(u0, prm)
    want = _gauss_closed_form(N, w0, nf)
    assert np.max(np.abs(got - want)) < 1e-12
    back = oracle.propagate(got, prm, inverse=True)          # D_{-z} D_z = 1
    assert np.max(np.abs(back - u0)) < 1e-12
    assert abs(np.sum(np.abs(got) ** 2) / np.sum(np.abs(u0) ** 2) - 1) < 1e-13   # unitary


def test_fresnel_propagator_talbot_self_images():
    """A field with period p = N/m in both axes images itself at the Talbot
    distance (N_F = m^2 / 2) and is shifted by half a period at half of it
    (N_F = m^2): its spectrum lives on multiples of m, where the transfer
    function is 1, resp. (-1)^n per axis."""
    rng = np.random.default_rng(12)
    N, m = 64, 8
    p = N // m
    cell = rng.standard_normal((p, p)) + 1j * rng.standard_normal((p, p))
    u = np.tile(cell, (m, m))
    assert np.max(np.abs(oracle.propagate(u, Params(propagator=1, fresnel=m * m / 2.0)) - u)) < 1e-12
    half = oracle.propagate(u, Params(propagator=1, fresnel=float(m * m)))
    assert np.max(np.abs(half - np.roll(u, (p // 2, p // 2), axis=(0, 1)))) < 1e-12


def test_forward_intensity_matches_bruteforce():
    """Eq. 4 with brute-force DFT matrices: far field sum_p |F P_p o F^T|^2;
    near field with the transfer function applied between F and its
    inverse written out pixel by pixel."""
    rng = np.random.default_rng(13)
    n, nf = 8, 11.0
    o = crandn(rng, n, n)
    P = crandn(rng, 3, n, n)
    far = sum(np.abs(brute_fft2u(P[p] * o)) ** 2 for p in range(3))
    assert np.allclose(oracle.forward_intensity64(P, o), far, rtol=0, atol=1e-12)
    F = dft_matrix(n)
    Hk = np.empty((n, n), complex)
    for a in range(n):
        for b in range(n):
            ka = a if a < n / 2 else a - n
            kb = b if b < n / 2 else b - n
            Hk[a, b] = np.exp(-1j * np.pi * (ka * ka + kb * kb) / nf)
    near = sum(np.abs(np.conj(F).T @ (Hk * (F @ (P[p] * o) @ F.T)) @ np.conj(F)) ** 2 for p in range(3))
    assert np.allclose(oracle.forward_intensity64(P, o, Params(propagator=1, fresnel=nf)), near, rtol=0, atol=1e-12)


def test_near_field_fixed_point():
    """U3 in the near field: data simulated (by the virtual experiment's own
    Fresnel code) from (O*, P*) leave O*, P* unchanged.  Catches a
    back-propagation without the conjugate transfer function."""
    rng = np.random.default_rng(14)
    H, N, M, nf = 48, 16, 2, 30.0
    O = crandn(rng, H, H)
    P = crandn(rng, M, N, N)
    pos = np.array([[0, 0], [5, 9], [20, 31], [32, 12]], dtype=float)
    I, scale = wl.simulate_patterns(rng, O, P, pos, 1e6, noise=False, fresnel=nf)
    Ps = P * math.sqrt(scale)
    prm = Params(iterations=2, beta=0.6, gamma=0.3, propagator=1, fresnel=nf)
    r = oracle.rpie64(O, Ps, pos, I.astype(float), prm)
    assert np.max(np.abs(r["O"] - O)) < 1e-5 * np.abs(O).max()      # float32 data
    assert np.max(np.abs(r["P"] - Ps)) < 1e-5 * np.abs(Ps).max()
    m = mutated_oracle("ifft2u(fft2u(psi) * (np.conj(H) if inverse else H))", "ifft2u(fft2u(psi) * H)")
    r2 = m["rpie64"](O, Ps, pos, I.astype(float), m["Params"](**prm.__dict__))
    assert np.max(np.abs(r2["O"] - O)) > 1e-2 * np.abs(O).max()


def test_near_field_monotone_error_with_diffuser_probe():
    """V1 in the near field: noise-free patterns of a diffuser-phase probe,
    probe held at the truth: the error never increases and falls below
    1e-2 of the first in 20 iterations."""
    w = wl.nearfield_case(seed=8, noise=False)
    prm = Params(**dict(w.params, iterations=20, probe_update_start=10 ** 6))
    e = oracle.rpie64(w.O0, w.P_true, w.pos0, w.I, prm)["err"]
    assert np.all(np.diff(e) <= 1e-12) and e[-1] < 1e-2 * e[0], e


# ---------------------------------------------------------- canvas (R-canv)
def test_canvas_map_counts_boxes():
    """A constant probe makes the canvas map the number of boxes covering
    each pixel times |P|^2 summed over modes (counted pixel by pixel), and
    its total is J N^2 sum_p |P_p|^2 for any probe."""
    H, W, N = 20, 24, 6
    pos = np.array([[0, 0], [3.4, 2.6], [14, 18], [7.5, 10.49], [14, 0]])
    P = np.stack([np.full((N, N), 0.5 + 1j), np.full((N, N), 0.25)])
    C = oracle.canvas64(P, pos, H, W)
    corners = [(int(math.floor(y + 0.5)), int(math.floor(x + 0.5))) for y, x in pos]
    p2 = abs(0.5 + 1j) ** 2 + 0.25 ** 2
    for yy in range(H):
        for xx in range(W):
            cnt = sum(1 for y, x in corners if y <= yy < y + N and x <= xx < x + N)
            assert abs(C[yy, xx] - cnt * p2) < 1e-12
    rng = np.random.default_rng(15)
    Pr = crandn(rng, 3, N, N)
    assert abs(oracle.canvas64(Pr, pos, H, W).sum() - len(pos) * np.sum(np.abs(Pr) ** 2)) < 1e-9


# ------------------------------------------- float rounding under reading R1
def test_r1_raster_amplifies_float_rounding():
    """Why the raster workload under R1 cannot be matched to 1e-4 by any
    float32 implementation: one float rounding of the initial object (a
    relative 2^-24 perturbation) grows to > 1e-3 after one iteration and >
    1e-2 after 20 in the FP64 oracle itself, whereas under R2 it stays below
    1e-6 / 1e-4 (the tolerances the GPU meets there)."""
    w = wl.raster_case(seed=0)
    rng = np.random.default_rng(1)
    O0 = w.O0.astype(complex)
    dO = O0 * (1 + 2.0 ** -24 * (rng.standard_normal(O0.shape) + 1j * rng.standard_normal(O0.shape)))
    rel = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
    out = {}
    for name, prm in (("R1", wl.R1_PARAMS), ("R2", wl.R2_PARAMS)):
        for T in (1, 20):
            p = Params(**dict(prm, iterations=T))
            a = oracle.rpie64(O0, w.P0, w.pos0, w.I, p)
            b = oracle.rpie64(dO, w.P0, w.pos0, w.I, p)
            out[name, T] = max(rel(b["O"], a["O"]), rel(b["P"], a["P"]))
    assert out["R1", 1] > 1e-3 and out["R1", 20] > 1e-2, out
    assert out["R2", 1] < 1e-6 and out["R2", 20] < 1e-4, out


def test_near_field_raster_r1_is_chaotic_r2_is_not():
    """The near-field raster under the rPIE weights (gamma = 0.1) amplifies a
    1e-7 relative perturbation of the starting object to more than 1e-2
    after 20 iterations in FP64 (so no FP32 implementation can stay within
    1e-3 of the oracle there), while the unit-step M-ePIE weights (alpha =
    0.1, beta = gamma = 1) keep it below 1e-5.  Evidence for the near-field
    tolerances of the GPU tests, not a pin of the oracle's arithmetic."""
    w = wl.nearfield_case(seed=8)
    rng = np.random.default_rng(0)
    O1 = w.O0.astype(complex) * (1 + 1e-7 * rng.standard_normal(w.O0.shape))
    rel = lambda x, y: np.linalg.norm(x - y) / np.linalg.norm(y)
    for extra, lo, hi in ((dict(), 1e-2, np.inf), (dict(alpha_obj=0.1, alpha_probe=0.1, beta=1.0, gamma=1.0), 0, 1e-5)):
        prm = Params(**dict(w.params, iterations=20, **extra))
        a = oracle.rpie64(w.O0, w.P0, w.pos0, w.I, prm)
        b = oracle.rpie64(O1, w.P0, w.pos0, w.I, prm)
        d = rel(b["O"], a["O"])
        assert lo <= d < hi, (extra, d)
