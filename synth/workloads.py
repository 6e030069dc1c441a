"""Seeded synthetic inputs (the paper's "virtual experiment").

This module serves both the HIP path and the oracle with the same bytes.  It
holds no reconstruction arithmetic: it draws objects, probes and scans from a
seeded ``numpy.random.Generator(PCG64(seed))`` and simulates far-field
diffraction data (Methods, "Virtual experiment": a far-field setup, a scan
with random jitter, object and probe assembled from magnitude and phase).
The data simulation uses ``scipy.fft``; neither the oracle nor the GPU path
imports anything from here except the finished arrays.

Shapes follow the workloads of the paper's soft-X-ray scans (a small raster
case, a 1024^2 / 256^2 / 3-mode / 1600-point
Fermat-spiral case, its position-error variant, a gradient-check subset and a
64-job uneven batch).  All arrays handed out are complex64 / float32, the
precision the GPU path works in; the oracle upcasts them.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.fft as sfft
from scipy.ndimage import gaussian_filter
from scipy.special import erfc

GOLDEN_ANGLE = math.pi * (3.0 - math.sqrt(5.0))


@dataclass
class Workload:
    name: str
    O_true: np.ndarray          # [H, W] complex64
    P_true: np.ndarray          # [M, N, N] complex64 (photon-scaled)
    pos_true: np.ndarray        # [J, 2] float32 (y, x) box corners
    I: np.ndarray               # [J, N, N] float32, FFT order
    O0: np.ndarray              # [H, W] complex64 initial object
    P0: np.ndarray              # [M, N, N] complex64 initial probe
    pos0: np.ndarray            # [J, 2] float32 initial positions
    params: dict = field(default_factory=dict)

    @property
    def shape(self):
        M, N, _ = self.P0.shape
        H, W = self.O0.shape
        return dict(H=H, W=W, N=N, M=M, J=self.pos0.shape[0])


# ----------------------------------------------------------------------------
# Object, probe and scan recipes
# ----------------------------------------------------------------------------
def object_field(rng, H, W, sigma=4.0):
    """Amplitude U(0.8, 1); phase = white noise smoothed (sigma px, wrap),
    affinely rescaled to [-pi/2, pi/2]."""
    amp = rng.uniform(0.8, 1.0, size=(H, W))
    ph = gaussian_filter(rng.standard_normal((H, W)), sigma=sigma, mode="wrap")
    ph = (ph - ph.min()) / (ph.max() - ph.min()) * math.pi - math.pi / 2
    return amp * np.exp(1j * ph)


def disc_probe(N, R, edge=2.0, phase_edge=0.5, with_phase=True):
    """Disc of radius R centred at (N/2, N/2) with an erfc-apodised edge of
    width `edge` px and a quadratic phase of `phase_edge` rad at r = R."""
    y, x = np.mgrid[0:N, 0:N].astype(np.float64)
    r = np.hypot(y - N / 2, x - N / 2)
    amp = 0.5 * erfc((r - R) / (math.sqrt(2.0) * edge))
    ph = phase_edge * (r / R) ** 2 if with_phase else 0.0
    return amp * np.exp(1j * ph)


MODE_POWERS = (0.7, 0.2, 0.1, 0.05, 0.025, 0.0125, 0.00625, 0.003125)


def probe_modes(N, R, M, powers=None, with_phase=True):
    """M (<= 8) mutually orthogonal modes {P0, P0 x/R, P0 y/R,
    P0 (x^2-y^2)/R^2, P0 2xy/R^2, P0 (x^3-3xy^2)/R^3, P0 (3x^2y-y^3)/R^3,
    P0 (x^2+y^2)/R^2}[:M], Gram-Schmidt orthogonalised, unit total power
    split by `powers` (renormalised)."""
    base = disc_probe(N, R, with_phase=with_phase)
    y, x = np.mgrid[0:N, 0:N].astype(np.float64)
    y = (y - N / 2) / R
    x = (x - N / 2) / R
    mods = [np.ones_like(x), x, y, x * x - y * y, 2 * x * y, x ** 3 - 3 * x * y * y, 3 * x * x * y - y ** 3,
            x * x + y * y][:M]
    powers = np.asarray(powers if powers is not None else MODE_POWERS[:M], dtype=np.float64)
    powers = powers / powers.sum()
    out = []
    for m in mods:
        v = base * m
        for u in out:
            v = v - np.vdot(u, v) * u
        v = v / math.sqrt(np.vdot(v, v).real)
        out.append(v)
    return np.stack([math.sqrt(p) * v for p, v in zip(powers, out)])


def raster_scan(rng, nside, step, origin, jitter):
    """nside x nside raster (y, x) with uniform +-jitter per axis."""
    g = origin + step * np.arange(nside, dtype=np.float64)
    yy, xx = np.meshgrid(g, g, indexing="ij")
    pos = np.stack([yy.ravel(), xx.ravel()], axis=1)
    return pos + rng.uniform(-jitter, jitter, size=pos.shape)


def fermat_spiral(J, c, centre):
    """Fermat spiral r_k = c sqrt(k), golden-angle increments, (y, x)."""
    k = np.arange(J, dtype=np.float64)
    r = c * np.sqrt(k)
    th = k * GOLDEN_ANGLE
    return np.stack([centre[0] + r * np.sin(th), centre[1] + r * np.cos(th)], axis=1)


# ----------------------------------------------------------------------------
# Virtual experiment: far-field patterns
# ----------------------------------------------------------------------------
def _crop_shifted(O, p, N):
    """Patch of O at corner round-half-up(p), moved by the fractional part
    with a band-limited phase ramp (continuous stage positions)."""
    n = np.floor(p + 0.5).astype(np.int64)
    f = p - n
    c = O[n[0]:n[0] + N, n[1]:n[1] + N]
    if f[0] == 0 and f[1] == 0:
        return c
    k = sfft.fftfreq(N) * N
    ramp = np.exp(2j * math.pi * (k[:, None] * f[0] + k[None, :] * f[1]) / N)
    return sfft.ifft2(sfft.fft2(c, norm="ortho") * ramp, norm="ortho")


def _fresnel_kernel(N, fresnel):
    """Paraxial free-space transfer function of an N x N window whose Fresnel
    number (N delta)^2 / (lambda z) is `fresnel`: exp(-i pi (ky^2 + kx^2) /
    fresnel) on the integer FFT frequencies."""
    q = sfft.fftfreq(N) * N
    ph = -math.pi * (q[:, None] ** 2 + q[None, :] ** 2) / fresnel
    return np.cos(ph) + 1j * np.sin(ph)


def simulate_patterns(rng, O, P, pos, photons, noise=True, fresnel=None):
    """Mixed-state patterns at `pos` (far field, FFT order; or, with a
    Fresnel number, near field in detector-pixel order), scaled to a mean of
    `photons` counts per pattern, with Poisson noise.  Returns (I float32,
    scale)."""
    M, N, _ = P.shape
    J = pos.shape[0]
    I = np.empty((J, N, N), dtype=np.float64)
    Hk = _fresnel_kernel(N, fresnel) if fresnel else None
    for j in range(J):
        o = _crop_shifted(O, pos[j], N)
        F = sfft.fft2(P * o[None], norm="ortho", axes=(-2, -1))
        if Hk is not None:
            F = sfft.ifft2(F * Hk[None], norm="ortho", axes=(-2, -1))
        I[j] = np.sum(F.real ** 2 + F.imag ** 2, axis=0)
    scale = photons / float(I.sum(axis=(1, 2)).mean())
    I *= scale
    if noise:
        I = rng.poisson(I).astype(np.float64)
    return I.astype(np.float32), scale


INIT_PHASE = 0.2


def initial_object(seed, H, W):
    """Initial object guess: unit magnitude with a small white random phase
    U(-0.2, 0.2) rad (own generator, seed + 1000, so the data draws do not
    move).  A perfectly flat start would make the first updates depend on
    the phase of round-off: on a flat object the model spectrum of a smooth
    probe has near-zero bins where the data are non-zero, and the modulus
    step keeps the (arbitrary) phase of those bins."""
    rng = np.random.Generator(np.random.PCG64(seed + 1000))
    return np.exp(1j * rng.uniform(-INIT_PHASE, INIT_PHASE, size=(H, W)))


def _finish(name, O, P, pos_true, pos0, I, scale, R, params, seed=0):
    M, N, _ = P.shape
    P_true = (P * math.sqrt(scale)).astype(np.complex64)
    # initial guess: near-flat object, phase-free probe of the same mode
    # recipe at the data's mean power
    P0 = probe_modes(N, R, M, with_phase=False)
    mean_power = float(I.astype(np.float64).sum(axis=(1, 2)).mean())
    P0 = P0 * math.sqrt(mean_power / float(np.sum(np.abs(P0) ** 2)))
    return Workload(name=name, O_true=O.astype(np.complex64), P_true=P_true,
                    pos_true=pos_true.astype(np.float32), I=I,
                    O0=initial_object(seed, *O.shape).astype(np.complex64),
                    P0=P0.astype(np.complex64), pos0=pos0.astype(np.float32),
                    params=params)


# rPIE parameters of the small raster case, reading "alpha=0.1, beta=1.0" as
# object-denominator weight 0.1 and probe-denominator weight 1.0, unit steps.
R1_PARAMS = dict(alpha_obj=1.0, alpha_probe=1.0, beta=1.0, gamma=0.1)
# literal-symbol alternative: M-ePIE with step 0.1
R2_PARAMS = dict(alpha_obj=0.1, alpha_probe=0.1, beta=1.0, gamma=1.0)


def raster_case(seed=0, H=256, N=64, R=20.0, nside=10, step=16.0, origin=24.0,
                jitter=2.0, photons=1e6, iterations=20, noise=True, name="raster64",
                fractional=False, M=1):
    """Raster workload (64^2 probe, 256^2 object, 10x10 scan by default).
    `fractional` keeps the jittered positions unrounded (continuous stage
    positions; the patterns are simulated with the Fourier shift)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    O = object_field(rng, H, H)
    P = probe_modes(N, R, M)
    pos = raster_scan(rng, nside, step, origin, jitter)
    if not fractional:
        pos = np.floor(pos + 0.5)
    I, scale = simulate_patterns(rng, O, P, pos, photons, noise)
    return _finish(name, O, P, pos, pos, I, scale, R,
                   dict(R1_PARAMS, iterations=iterations, subpixel=int(fractional)), seed=seed)


def spiral_case(seed=1, H=1024, N=256, M=3, J=1600, R=32.0, c=9.6, photons=1e7,
                iterations=50, pos_sigma=0.0, noise=True, name="spiral256x3"):
    """Mixed-state Fermat-spiral workload (256^2 probe, 3 modes, 1600 points,
    ~70 % overlap, 1024^2 object).  With pos_sigma > 0 the true positions
    carry Gaussian errors and the reconstruction starts at the nominal
    spiral."""
    rng = np.random.Generator(np.random.PCG64(seed))
    O = object_field(rng, H, H)
    P = probe_modes(N, R, M)
    span = H - N
    nominal = np.floor(fermat_spiral(J, c, (span / 2.0, span / 2.0)) + 0.5)
    nominal = np.clip(nominal, 0, span)
    if pos_sigma > 0:
        true = np.clip(nominal + rng.normal(0.0, pos_sigma, size=nominal.shape), 0, span)
    else:
        true = nominal
    I, scale = simulate_patterns(rng, O, P, true, photons, noise)
    prm = dict(R1_PARAMS, iterations=iterations)
    if pos_sigma > 0:
        prm.update(subpixel=1, refine=1, refine_start=0, upsample=100, xcorr_norm=0,
                   adam_lr=0.5, adam_b1=0.9, adam_b2=0.999, adam_eps=1e-8)
    return _finish(name, O, P, true, nominal, I, scale, R, prm, seed=seed)


def refine_case(seed=2, **kw):
    """Spiral workload with sigma = 3 px position errors and refinement on."""
    kw.setdefault("name", "spiral256x3_refine")
    return spiral_case(seed=seed, pos_sigma=3.0, **kw)


def gradient_subset(seed=3, H=128, N=32, M=3, R=10.0, photons=1e6):
    """Gradient-check subset: 128^2 object, 32^2 probe, 3 modes, 5x5 raster
    (origin 32, step 8) with subpixel offsets U(-0.4, 0.4)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    O = object_field(rng, H, H)
    P = probe_modes(N, R, M)
    pos = raster_scan(rng, 5, 8.0, 32.0, 0.0)
    pos = pos + rng.uniform(-0.4, 0.4, size=pos.shape)
    I, scale = simulate_patterns(rng, O, P, pos, photons, True)
    return _finish("grad_subset", O, P, pos, pos, I, scale, R, dict(subpixel=1), seed=seed)


def _batch_job(seed, b, N, J, M, photons, iterations):
    """Job b of the uneven batch, drawn from its own generator (seed, b)."""
    rng = np.random.Generator(np.random.PCG64([seed, b]))
    c = 0.0394 * N
    H = int(math.ceil((2 * c * math.sqrt(J) + N + 8) / 16.0) * 16)
    R = N / 8.0
    O = object_field(rng, H, H)
    P = probe_modes(N, R, M)
    span = H - N
    pos = np.clip(np.floor(fermat_spiral(J, c, (span / 2.0, span / 2.0)) + 0.5), 0, span)
    I, scale = simulate_patterns(rng, O, P, pos, photons, True)
    return _finish(f"job{b}", O, P, pos, pos, I, scale, R,
                   dict(R1_PARAMS, iterations=iterations), seed=seed * 1000 + b)


def batch_jobs(seed=4, njobs=64, sizes=(64, 128, 192, 256), jmin=50, jmax=900,
               mmax=5, photons=1e6, iterations=20, jscale=1.0, workers=1):
    """Uneven batch: N ~ U{sizes}, J ~ U{jmin..jmax}, M ~ U{1..mmax} (all
    shapes drawn first from one generator), then each job from a generator
    of its own: probe radius N/8, spiral step 0.0394 N (~70 % overlap),
    object side ceil((2 c sqrt(J) + N + 8)/16)*16.  `jscale` < 1 shrinks J
    for tests; `workers` > 1 simulates the jobs in that many processes (the
    same bytes as one process)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    shapes = []
    for b in range(njobs):
        N = int(rng.choice(sizes))
        J = int(rng.integers(jmin, jmax + 1))
        M = int(rng.integers(1, mmax + 1))
        shapes.append((N, max(4, int(round(J * jscale))), M))
    args = [(seed, b, N, J, M, photons, iterations) for b, (N, J, M) in enumerate(shapes)]
    if workers <= 1:
        return [_batch_job(*a) for a in args]
    from concurrent.futures import ProcessPoolExecutor
    import multiprocessing as mp
    # largest jobs first, so the pool drains evenly
    order = sorted(range(njobs), key=lambda b: -shapes[b][0] ** 2 * shapes[b][1] * shapes[b][2])
    out = [None] * njobs
    with ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        futs = {b: ex.submit(_batch_job, *args[b]) for b in order}
        for b in order:
            out[b] = futs[b].result()
    return out


def nearfield_case(seed=8, H=128, N=32, M=1, R=12.0, nside=6, step=12.0, origin=16.0, jitter=2.0,
                   fresnel=40.0, diffuser_sigma=1.0, photons=1e6, noise=True, name="nearfield"):
    """Near-field raster workload: a disc probe carrying a random diffuser
    phase (white noise smoothed by `diffuser_sigma` px, 2 pi rms), as used
    in near-field ptychography to give the patterns contrast; positions
    rounded; patterns through the Fresnel transfer function of Fresnel
    number `fresnel`."""
    rng = np.random.Generator(np.random.PCG64(seed))
    O = object_field(rng, H, H)
    P = probe_modes(N, R, M)
    ph = gaussian_filter(rng.standard_normal((N, N)), diffuser_sigma, mode="wrap")
    P = P * np.exp(2j * math.pi * ph / ph.std())[None]
    pos = np.floor(raster_scan(rng, nside, step, origin, jitter) + 0.5)
    I, scale = simulate_patterns(rng, O, P, pos, photons, noise, fresnel=fresnel)
    return _finish(name, O, P, pos, pos, I, scale, R,
                   dict(R1_PARAMS, propagator=1, fresnel=float(fresnel)), seed=seed)


def small_case(seed, H, N, M, J, R=None, photons=1e6, subpixel=False, edges=True,
               name="small", W=None, fresnel=None):
    """Small workload for parity tests: Fermat spiral over the whole span,
    optionally with the first two positions pinned at the object corners
    (ragged / edge boxes) and optional fractional positions.  The object is
    H x W (W = H by default).  With a Fresnel number the patterns are
    near-field (detector-pixel order)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    W = H if W is None else W
    R = R if R is not None else N / 4.0
    O = object_field(rng, H, W)
    P = probe_modes(N, R, M)
    sy, sx = H - N, W - N
    c = min(sy, sx) / 2.0 / math.sqrt(max(J - 1, 1))
    pos = fermat_spiral(J, c, (sy / 2.0, sx / 2.0))
    if edges and J >= 3:
        pos[1] = (0.0, float(sx))
        pos[2] = (float(sy), 0.0)
    lim = np.array([sy, sx], dtype=np.float64)
    if subpixel:
        pos = pos + rng.uniform(-0.45, 0.45, size=pos.shape)
        pos = np.clip(pos, 0, lim)
    else:
        pos = np.floor(pos + 0.5)
    pos = np.clip(pos, 0, lim)
    I, scale = simulate_patterns(rng, O, P, pos, photons, True, fresnel=fresnel)
    prm = dict(R1_PARAMS, subpixel=int(subpixel))
    if fresnel:
        prm.update(propagator=1, fresnel=float(fresnel))
    return _finish(name, O, P, pos, pos, I, scale, R, prm, seed=seed)
