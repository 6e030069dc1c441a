"""FP64 CPU oracle for the multi-mode rPIE hot path (test infrastructure).

This module is TEST INFRASTRUCTURE. It is the plain, slow, obviously correct
reference that the HIP path is checked against. Only the test-suite, the smoke
check and the CPU-baseline leg of the benchmark may import it; the product path
never calls it and shares no code with it.

Everything is numpy complex128 / float64.  The 2-D far-field propagator is the
unitary DFT (``numpy.fft`` with ``norm="ortho"``), used as a library step.

Paper: Guzzi et al., "A modular software framework for the design and
implementation of ptychography algorithms" (SciComPty), arXiv 2205.04295.
Citations below name the section / equation / algorithm of that paper.

Readings where the paper is silent, garbled or ambiguous (each one is also
listed in the design notes):
  R-eq7   The modulus-corrected wave (Methods, "M-rPIE algorithm", the
          unnumbered-label equation after Eq. 6; Eq. 7 as rendered) sums
          |Psi_n|^2 over the M probe modes at the detector plane and scales
          each detector-plane mode Psi_p by sqrt(I)/sqrt(sum); where the sum
          is zero the corrected wave is zero.
  R-dz    D_z is the unitary 2-D DFT and D_{-z} its inverse, with no
          fftshift: intensities are stored in FFT order (DC at [0, 0]).
  R-order Eq. 5 and Eq. 6 both use the pre-update o_j and P_p (simultaneous).
  R-max   |o_j|^2_max is the max over the patch pixels; (sum_p |P_p|^2)_max
          is the max over pixels of the mode sum.
  R-zero  An update term is 0 where its denominator is 0; intensities are
          clamped at >= 0 before the square root.
  R-scan  Positions are visited in the given order, every iteration.
  R-crop  The crop corner is n = floor(pos + 0.5); with the subpixel switch
          on, the fractional part f = pos - n in [-1/2, 1/2) is applied as a
          band-limited Fourier shift o(r) = c(r + f) and the object update is
          shifted back by -f.  With it off, f is ignored.
  R-reg   Registration (Methods, "Adam-based position refinement", after
          Guizar-Sicairos et al. 2008, whose SciPy-ecosystem implementation
          the paper follows): X = F(ref) conj(F(mov)), unnormalised by
          default as in that implementation, optionally phase-normalised;
          integer peak of |F^-1 X| (first maximum in
          row-major order, lags above N//2 wrap negative); then a
          matrix-product DFT on a window of U = ceil(1.5 up) samples per axis
          at spacing 1/up centred (index floor(U/2)) on the integer peak.
          The returned shift s satisfies mov(r) ~ ref(r + s).
  R-adam  Alg. 1 (modified Adam): the registration shift is the gradient
          g_t; the moments follow Kingma & Ba with bias correction; t counts
          reconstruction iterations since refinement started; the position
          moves by +lr * mhat / (sqrt(vhat) + eps) (Eq. 8-9 use "+"), then is
          clamped so the box stays inside the object.
  R-grad  Loss L = sum_j sum_r (A_j - sqrt(I_j))^2 with A = sqrt(sum_p
          |Psi_p|^2); gradients follow the torch convention
          dL/dRe + i dL/dIm for complex arrays; (1 - sqrt(I)/A) is taken as 0
          where A = 0.  Not in the paper (an extension of its forward model,
          Eq. 4).  Far field only.
  R-near  Eq. 2 leaves D_z general.  The near-field option is the paraxial
          (Fresnel) transfer-function propagator D_z = F^-1 H F with
          H(k) = exp(-i pi (k_y^2 + k_x^2) / N_F) on the signed integer
          frequencies k of the N x N window, N_F = (N delta)^2 / (lambda z)
          its Fresnel number; D_{-z} = F^-1 conj(H) F.  The intensities are
          then detector pixels in real-space order.
  R-xcb   XCORR_B (Methods, "Adam-based position refinement": the switch
          that compares the model with the measured data) registers the
          modelled detector amplitude A_j = sqrt(sum_p |D_z(P_p o_j)|^2)
          (ref, taken before the modulus replacement) against the measured
          amplitude sqrt(I_j) (mov), both real.  With mov(r) ~ ref(r + s),
          s is the position error (truth minus estimate), the same sign as
          XCORR_A's, so Eq. 8-9 use it unchanged.
  R-canv  The canvas map (Results, sparse-scan figure) is the sum over
          positions of the mode-summed probe intensity sum_p |P_p|^2 placed
          at each position's integer box corner floor(pos + 0.5).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np

__all__ = [
    "Params", "fft2u", "ifft2u", "freq_grid", "split_position",
    "fourier_shift", "fresnel_transfer", "propagate", "modulus_project",
    "rpie_position_update", "rpie64", "register64", "upsampled_window",
    "adam64", "loss_grad64", "forward_intensity64", "canvas64",
]


# ----------------------------------------------------------------------------
# Parameters
# ----------------------------------------------------------------------------
@dataclass
class Params:
    """Reconstruction parameters (Methods, Eq. 5-6, Eq. 8-9, Alg. 1)."""
    alpha_obj: float = 1.0        # alpha_O in Eq. 6
    alpha_probe: float = 1.0      # alpha_P in Eq. 5
    beta: float = 1.0             # probe-denominator weight, Eq. 5
    gamma: float = 1.0            # object-denominator weight, Eq. 6
    iterations: int = 1
    iter_offset: int = 0          # first iteration index (resume)
    probe_update_start: int = 0   # probe is updated from this iteration on
    subpixel: int = 0             # 0 = nearest-integer crop, 1 = Fourier shift
    refine: int = 0               # position refinement (Eq. 8-9, Alg. 1) on/off
    refine_start: int = 0
    upsample: int = 100
    xcorr_norm: int = 0           # 0 = plain cross-power (default), 1 = phase-normalised
    adam_lr: float = 0.5
    adam_b1: float = 0.9
    adam_b2: float = 0.999
    adam_eps: float = 1e-8
    xcorr_point: int = 0          # 0 = XCORR_A (o_j vs o'_j), 1 = XCORR_B (model vs measured amplitude)
    propagator: int = 0           # 0 = far field (unitary DFT), 1 = near field (Fresnel transfer function)
    fresnel: float = 0.0          # Fresnel number N_F of the N x N window (near field)


# ----------------------------------------------------------------------------
# Propagator and shifts
# ----------------------------------------------------------------------------
def fft2u(x):
    """Unitary 2-D DFT over the last two axes: D_z of Eq. 2 in the far field."""
    return np.fft.fft2(x, norm="ortho")


def ifft2u(x):
    """Inverse unitary 2-D DFT: D_{-z}."""
    return np.fft.ifft2(x, norm="ortho")


def freq_grid(n):
    """Signed integer frequencies k (fftfreq * n); the Nyquist bin is -n/2."""
    return np.fft.fftfreq(n) * n


def split_position(pos, subpixel=1):
    """Crop corner n = floor(pos + 0.5) and fraction f = pos - n (reading R-crop)."""
    pos = np.asarray(pos, dtype=np.float64)
    n = np.floor(pos + 0.5).astype(np.int64)
    f = pos - n if subpixel else np.zeros_like(pos)
    return n, f


def _ramp(n, f):
    """exp(+2 pi i (k_y f_y + k_x f_x) / n) on the FFT-ordered grid."""
    k = freq_grid(n)
    ry = np.exp(2j * np.pi * k * f[0] / n)
    rx = np.exp(2j * np.pi * k * f[1] / n)
    return ry[:, None] * rx[None, :]


def fresnel_transfer(n, nf):
    """Paraxial free-space transfer function on the FFT grid (reading
    R-near): H(k) = exp(-i pi (k_y^2 + k_x^2) / N_F), k signed integers."""
    k = freq_grid(n)
    return np.exp(-1j * np.pi * (k[:, None] ** 2 + k[None, :] ** 2) / nf)


def propagate(psi, prm, inverse=False):
    """D_z of Eq. 2 (inverse=True: D_{-z}) over the last two axes.

    Far field: the unitary DFT and its inverse (reading R-dz).  Near field:
    F^-1 H F and F^-1 conj(H) F with the Fresnel transfer function."""
    if prm.propagator == 0:
        return ifft2u(psi) if inverse else fft2u(psi)
    H = fresnel_transfer(psi.shape[-1], prm.fresnel)
    return ifft2u(fft2u(psi) * (np.conj(H) if inverse else H))


def fourier_shift(c, f):
    """Band-limited circular shift: returns o with o(r) = c(r + f)."""
    if f[0] == 0.0 and f[1] == 0.0:
        return np.array(c, dtype=np.complex128, copy=True)
    return ifft2u(fft2u(c) * _ramp(c.shape[-1], f))


# ----------------------------------------------------------------------------
# Forward model and modulus constraint
# ----------------------------------------------------------------------------
def forward_intensity64(P, o, prm=None):
    """Mixed-state intensity, Eq. 4: I = sum_p |D_z{P_p o}|^2."""
    Psi = propagate(P * o[None], prm if prm is not None else Params())
    return np.sum(np.abs(Psi) ** 2, axis=0)


def modulus_project(Psi, I):
    """Modulus replacement of Eq. 7 (reading R-eq7).

    Psi: [M, N, N] detector-plane waves; I: [N, N] measured intensity.
    Returns (Psi', A, sqrt(I)) with Psi'_p = sqrt(I)/A * Psi_p, 0 where A = 0.
    """
    S = np.sum(np.abs(Psi) ** 2, axis=0)
    A = np.sqrt(S)
    sqI = np.sqrt(np.maximum(I, 0.0))
    fac = np.zeros_like(A)
    nz = S > 0
    fac[nz] = sqI[nz] / A[nz]
    return Psi * fac[None], A, sqI


# ----------------------------------------------------------------------------
# One M-rPIE position update (Eq. 5-7)
# ----------------------------------------------------------------------------
def rpie_position_update(o, P, I, prm: Params, update_probe=True):
    """One M-rPIE step on a patch (Methods, Eq. 4-7).

    o: [N, N] object patch o_j (already shifted), P: [M, N, N] probe modes,
    I: [N, N] intensity (FFT order in the far field).  Returns (delta_o,
    P_new, err_sum, A, sqrt(I)) where delta_o is the additive object-patch
    update of Eq. 6, P_new the probe after Eq. 5 (or P unchanged), err_sum =
    sum (A - sqrt(I))^2, and A the modelled detector amplitude before the
    modulus replacement.
    """
    psi = P * o[None]                              # Eq. 1 / Eq. 4, per mode
    Psi = propagate(psi, prm)                      # Eq. 2
    Psi_c, A, sqI = modulus_project(Psi, I)        # Eq. 7
    err = float(np.sum((A - sqI) ** 2))
    psi_c = propagate(Psi_c, prm, inverse=True)    # D_{-z}
    diff = psi_c - psi                             # psi'_{p,j} - P_p o_j

    # Eq. 6: object update, weighted by the (old) mode-summed probe power.
    Psum = np.sum(np.abs(P) ** 2, axis=0)
    dO = prm.gamma * Psum.max() + (1.0 - prm.gamma) * Psum
    num_o = np.sum(diff * np.conj(P), axis=0)
    delta_o = np.zeros_like(o)
    nz = dO != 0
    delta_o[nz] = prm.alpha_obj * num_o[nz] / dO[nz]

    # Eq. 5: probe update, weighted by the (old) patch power.
    if update_probe:
        o2 = np.abs(o) ** 2
        dP = prm.beta * o2.max() + (1.0 - prm.beta) * o2
        P_new = np.array(P, copy=True)
        nzp = dP != 0
        upd = diff * np.conj(o)[None]
        P_new[:, nzp] += prm.alpha_probe * upd[:, nzp] / dP[nzp]
    else:
        P_new = np.array(P, copy=True)
    return delta_o, P_new, err, A, sqI


# ----------------------------------------------------------------------------
# Registration (Guizar-Sicairos 2008 as the paper uses it) and Adam (Alg. 1)
# ----------------------------------------------------------------------------
def _coarse_peak(X):
    """Integer lag of the maximum of |F^-1 X| (first max, row-major)."""
    n0, n1 = X.shape
    cc = np.abs(np.fft.ifft2(X))
    p = int(np.argmax(cc))
    py, px = divmod(p, n1)
    sy = py - n0 if py > n0 // 2 else py
    sx = px - n1 if px > n1 // 2 else px
    return sy, sx, (py, px)


def upsampled_window(X, s0, up):
    """C(u, v) = sum_k X(k) exp(+2 pi i [k_y a_u + k_x b_v] / N) as two
    matrix products (the matrix-multiply DFT of the refinement step), with
    a_u = s0_y + (u - c)/up, b_v = s0_x + (v - c)/up, U = ceil(1.5 up)."""
    n0, n1 = X.shape
    U = int(math.ceil(1.5 * up))
    c = U // 2
    a = s0[0] + (np.arange(U) - c) / up
    b = s0[1] + (np.arange(U) - c) / up
    Ky = np.exp(2j * np.pi * np.outer(a, freq_grid(n0)) / n0)   # [U, N0]
    Kx = np.exp(2j * np.pi * np.outer(freq_grid(n1), b) / n1)   # [N1, U]
    return Ky @ X @ Kx, c


def register64(ref, mov, up=100, norm=0):
    """Subpixel registration (Methods, position refinement; reading R-reg).

    Returns (shift[2], peak[4]) where shift = s0 + ((u*, v*) - c)/up and
    peak = (p_y, p_x, u*, v*) are the integer argmax indices of the coarse
    correlation and of the upsampled window.
    """
    ref = np.asarray(ref, dtype=np.complex128)
    mov = np.asarray(mov, dtype=np.complex128)
    X = np.fft.fft2(ref) * np.conj(np.fft.fft2(mov))
    if norm == 1:
        m = np.abs(X)
        Xn = np.zeros_like(X)
        nz = m > 0
        Xn[nz] = X[nz] / m[nz]
        X = Xn
    sy, sx, (py, px) = _coarse_peak(X)
    C, c = upsampled_window(X, (sy, sx), up)
    q = int(np.argmax(np.abs(C)))
    u, v = divmod(q, C.shape[1])
    shift = np.array([sy + (u - c) / up, sx + (v - c) / up])
    return shift, np.array([py, px, u, v], dtype=np.int64)


def adam64(pos, state, g, t, prm: Params, bounds):
    """Alg. 1 (modified Adam) for one position; in-place on pos and state.

    state = [m_y, m_x, v_y, v_x]; g = measured shift (the gradient g_t);
    bounds = (max_y, max_x) of the box corner (reading R-adam).
    """
    b1, b2 = prm.adam_b1, prm.adam_b2
    for a in range(2):
        state[a] = b1 * state[a] + (1.0 - b1) * g[a]
        state[2 + a] = b2 * state[2 + a] + (1.0 - b2) * g[a] * g[a]
        mhat = state[a] / (1.0 - b1 ** t)
        vhat = state[2 + a] / (1.0 - b2 ** t)
        pos[a] = pos[a] + prm.adam_lr * mhat / (math.sqrt(vhat) + prm.adam_eps)
        pos[a] = min(max(pos[a], 0.0), float(bounds[a]))
    return pos, state


# ----------------------------------------------------------------------------
# The sequential sweep (Methods, M-rPIE + Adam refinement)
# ----------------------------------------------------------------------------
def rpie64(O, P, pos, I, prm: Params, adam=None, record=None):
    """Sequential M-rPIE reconstruction, optionally with XCORR_A refinement.

    O: [H, W] complex object (updated copy returned), P: [M, N, N] probe modes,
    pos: [J, 2] (y, x) box corners in pixels, I: [J, N, N] intensities in FFT
    order.  Returns dict(O, P, pos, adam, err[T]) where err[it] is the
    normalised Fourier error sum_j sum (A - sqrt(I))^2 / sum_j sum I.
    ``record`` (optional list) receives (it, j, ref, mov) for refined
    steps: (o, o + delta_o) for XCORR_A, (A, sqrt(I)) for XCORR_B.
    """
    O = np.array(O, dtype=np.complex128, copy=True)
    P = np.array(P, dtype=np.complex128, copy=True)
    pos = np.array(pos, dtype=np.float64, copy=True)
    I = np.asarray(I, dtype=np.float64)
    H, W = O.shape
    M, N, _ = P.shape
    J = pos.shape[0]
    adam = np.zeros((J, 4)) if adam is None else np.array(adam, dtype=np.float64, copy=True)
    bounds = (H - N, W - N)
    Isum = float(np.sum(np.maximum(I, 0.0)))
    err = np.zeros(prm.iterations)
    for t_i in range(prm.iterations):
        it = prm.iter_offset + t_i
        for j in range(J):
            n, f = split_position(pos[j], prm.subpixel)
            if not (0 <= n[0] <= H - N and 0 <= n[1] <= W - N):
                raise ValueError(f"position {j} outside the object")
            box = (slice(n[0], n[0] + N), slice(n[1], n[1] + N))
            o = fourier_shift(O[box], f)
            d_o, P_new, e, A, sqI = rpie_position_update(o, P, I[j], prm,
                                                         update_probe=it >= prm.probe_update_start)
            err[t_i] += e
            P = P_new
            O[box] = O[box] + fourier_shift(d_o, -f)
            if prm.refine and it >= prm.refine_start:
                # XCORR_A: the patch against its own update; XCORR_B: the
                # modelled detector amplitude against the measured one
                ref, mov = (o, o + d_o) if prm.xcorr_point == 0 else (A, sqI)
                s, _ = register64(ref, mov, prm.upsample, prm.xcorr_norm)
                if record is not None:
                    record.append((it, j, ref, mov))
                adam64(pos[j], adam[j], s, it - prm.refine_start + 1, prm, bounds)
        err[t_i] /= Isum if Isum > 0 else 1.0
    return dict(O=O, P=P, pos=pos, adam=adam, err=err)


# ----------------------------------------------------------------------------
# Loss and analytic gradient (adjoint of the Eq. 4 forward model)
# ----------------------------------------------------------------------------
def loss_grad64(O, P, pos, I, subpixel=1):
    """Amplitude loss and its gradient w.r.t. O, P and positions (R-grad).

    Positions enter through the Fourier shift of the crop (R-crop); the
    integer corner is piecewise constant and contributes nothing.
    Returns (L, gO [H, W], gP [M, N, N], gpos [J, 2]).
    """
    O = np.asarray(O, dtype=np.complex128)
    P = np.asarray(P, dtype=np.complex128)
    pos = np.asarray(pos, dtype=np.float64)
    I = np.asarray(I, dtype=np.float64)
    M, N, _ = P.shape
    J = pos.shape[0]
    k = freq_grid(N)
    L = 0.0
    gO = np.zeros_like(O)
    gP = np.zeros_like(P)
    gpos = np.zeros((J, 2))
    for j in range(J):
        n, f = split_position(pos[j], subpixel)
        box = (slice(n[0], n[0] + N), slice(n[1], n[1] + N))
        o = fourier_shift(O[box], f)
        Psi = fft2u(P * o[None])
        A = np.sqrt(np.sum(np.abs(Psi) ** 2, axis=0))
        sqI = np.sqrt(np.maximum(I[j], 0.0))
        L += float(np.sum((A - sqI) ** 2))
        w = np.zeros_like(A)
        nz = A > 0
        w[nz] = 1.0 - sqI[nz] / A[nz]
        chi = ifft2u(w[None] * Psi)
        gP += 2.0 * np.conj(o)[None] * chi
        g_o = 2.0 * np.sum(np.conj(P) * chi, axis=0)
        gO[box] += fourier_shift(g_o, -f)
        if subpixel:
            Go = fft2u(g_o)
            Fo = fft2u(o)
            ky = (2j * np.pi * k / N)[:, None]
            kx = (2j * np.pi * k / N)[None, :]
            gpos[j, 0] = np.real(np.sum(np.conj(Go) * ky * Fo))
            gpos[j, 1] = np.real(np.sum(np.conj(Go) * kx * Fo))
    return L, gO, gP, gpos


# ----------------------------------------------------------------------------
# Canvas map (Results, sparse-scan figure)
# ----------------------------------------------------------------------------
def canvas64(P, pos, H, W):
    """Canvas map (reading R-canv): sum_j sum_p |P_p|^2 placed at the box
    of position j, on an H x W grid."""
    P = np.asarray(P, dtype=np.complex128)
    pos = np.asarray(pos, dtype=np.float64)
    N = P.shape[-1]
    Pi = np.sum(np.abs(P) ** 2, axis=0)
    C = np.zeros((H, W))
    for j in range(pos.shape[0]):
        n, _ = split_position(pos[j], 0)
        if not (0 <= n[0] <= H - N and 0 <= n[1] <= W - N):
            raise ValueError(f"position {j} outside the object")
        C[n[0]:n[0] + N, n[1]:n[1] + N] += Pi
    return C
