"""Seeded synthetic star fields and target images for the DIA kernel fit.

Input generation only: this module renders reference images, draws the
injected kernels and backgrounds, and forms noisy targets.  It is shared by
the tests, the benchmark and the smoke check, and holds none of the fit's
arithmetic: the noiseless target is formed with scipy's own correlation
routine, never with the oracle or the GPU library.

Recipe (Section 3.1 "Generating artificial images" for the scene; the sizes
of each workload are those of the config functions below):

* stars at continuous positions uniform over the frame, fluxes log-uniform
  between ``flux_min`` and ``flux_max`` (the paper's own F^(-3/2) law is
  available as ``paper_reference``);
* an analytic PSF (Gaussian or Moffat) sampled at pixel centres on a stamp of
  radius 10 FWHM, normalised analytically; a constant sky;
* the injected kernel is an (elliptical) Gaussian sampled on the m x m grid,
  centred at (h + dy, h + dx) and scaled to the requested sum (the
  photometric scale factor, eq. photometric_scale_factor);
* the noiseless target is the reference cross-correlated with that kernel
  plus B0 (eq. model_image_delta_basis) on the valid region; the border,
  which the fit never uses, comes from an edge-replicated reference;
* noise: Poisson in electrons with gain G, plus Gaussian read noise
  sigma0 (electrons), both converted to ADU, so the matching CCD noise model
  (eq. CCDNM, F = 1) has sigma0_adu = sigma0 / G.

All random draws come from ``numpy.random.default_rng`` seeded with
``SeedSequence([2104, 13715, config, epoch])``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
from scipy import signal

FWHM_PER_SIGMA = 2.0 * math.sqrt(2.0 * math.log(2.0))


def rng_for(config: int, epoch: int = 0) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([2104, 13715, int(config), int(epoch)]))


# --------------------------------------------------------------------------- PSFs
def gaussian_psf(fwhm: float):
    s = fwhm / FWHM_PER_SIGMA
    norm = 1.0 / (2.0 * math.pi * s * s)
    k = -0.5 / (s * s)

    def f(r2):
        return norm * np.exp(k * r2)

    return f


def moffat_psf(fwhm: float, beta: float = 3.0):
    alpha = fwhm / (2.0 * math.sqrt(2.0 ** (1.0 / beta) - 1.0))
    norm = (beta - 1.0) / (math.pi * alpha * alpha)
    inv_a2 = 1.0 / (alpha * alpha)

    def f(r2):
        t = 1.0 / (1.0 + r2 * inv_a2)
        if beta == 3.0:
            return norm * (t * t * t)
        return norm * t ** beta

    return f


def render_stars(shape, x, y, flux, psf, radius: int, sky: float = 0.0, chunk: int = 2048):
    """Sum of flux * psf(|p - star|^2) sampled at pixel centres (x = column, y = row), stamps of the
    given radius, plus a constant sky.  Rendered on a canvas padded by the radius, then cropped."""
    H, W = shape
    Hp, Wp = H + 2 * radius + 1, W + 2 * radius + 1
    out = np.zeros(Hp * Wp, dtype=np.float64)
    off = np.arange(-radius, radius + 1, dtype=np.float64)
    flat_off = (off[:, None] * Wp + off[None, :]).astype(np.int64).ravel()
    for s in range(0, len(x), chunk):
        xs, ys, fs = x[s:s + chunk], y[s:s + chunk], flux[s:s + chunk]
        cx = np.rint(xs)
        cy = np.rint(ys)
        fx = cx - xs
        fy = cy - ys
        ddx = off[None, :] + fx[:, None]                       # (n, 2r+1) column offsets from the star
        ddy = off[None, :] + fy[:, None]
        r2 = ddy[:, :, None] ** 2 + ddx[:, None, :] ** 2          # (n, 2r+1, 2r+1)
        val = fs[:, None] * psf(r2.reshape(len(xs), -1))
        base = (cy.astype(np.int64) + radius) * Wp + (cx.astype(np.int64) + radius)
        out += np.bincount((base[:, None] + flat_off[None, :]).ravel(), weights=val.ravel(), minlength=Hp * Wp)
    img = out.reshape(Hp, Wp)[radius:radius + H, radius:radius + W]
    return img + sky


def kernel_gaussian(m: int, fwhm_x: float, fwhm_y: float | None = None, rot_deg: float = 0.0,
                    dx: float = 0.0, dy: float = 0.0, total: float = 1.0) -> np.ndarray:
    """(Elliptical) Gaussian on the m x m grid, centred at (h + dy, h + dx), summing to ``total``."""
    if fwhm_y is None:
        fwhm_y = fwhm_x
    h = (m - 1) // 2
    sx = fwhm_x / FWHM_PER_SIGMA
    sy = fwhm_y / FWHM_PER_SIGMA
    a, b = np.meshgrid(np.arange(m), np.arange(m), indexing="ij")
    u = b - (h + dx)
    v = a - (h + dy)
    t = math.radians(rot_deg)
    ur = math.cos(t) * u + math.sin(t) * v
    vr = -math.sin(t) * u + math.cos(t) * v
    k = np.exp(-0.5 * ((ur / sx) ** 2 + (vr / sy) ** 2))
    return k * (total / k.sum())


def correlate_target(R: np.ndarray, K: np.ndarray, B0: float) -> np.ndarray:
    """Noiseless target on R's full grid: correlation with K plus B0; edge-replicated border."""
    h = (K.shape[0] - 1) // 2
    Rp = np.pad(R, h, mode="edge")
    method = "direct" if R.size * K.size < 4e7 else "fft"
    return signal.correlate(Rp, K, mode="valid", method=method) + B0


def add_ccd_noise(I_nl: np.ndarray, gain: float, sigma0_e: float, rng: np.random.Generator) -> np.ndarray:
    lam = np.clip(I_nl, 0.0, None) * gain
    e = rng.poisson(lam).astype(np.float64)
    e += rng.normal(0.0, sigma0_e, size=I_nl.shape)
    return e / gain


def equivalent_fwhm(psf, K: np.ndarray | None = None, half_extent: float = 12.0, oversample: int = 10) -> float:
    """FWHM (pixels) of the circle whose area equals the area above half maximum of a PSF profile,
    measured on a grid oversampled ``oversample`` times per pixel.  psf is a radial profile f(r^2)
    (gaussian_psf / moffat_psf); with K the profile is that PSF correlated with the pixel kernel K
    (the PSF of a target made from the reference by K), which is what a width measurement on the
    target's stars returns."""
    t = np.arange(-half_extent, half_extent + 1e-9, 1.0 / oversample)
    yy, xx = np.meshgrid(t, t, indexing="ij")
    if K is None:
        img = psf(xx * xx + yy * yy)
    else:
        h = (K.shape[0] - 1) // 2
        img = np.zeros_like(xx)
        for a in range(K.shape[0]):
            for b in range(K.shape[1]):
                if K[a, b] != 0.0:
                    dy, dx = a - h, b - h
                    img += K[a, b] * psf((xx + dx) ** 2 + (yy + dy) ** 2)
    area = np.count_nonzero(img >= 0.5 * img.max()) / (oversample * oversample)
    return 2.0 * math.sqrt(area / math.pi)


# ----------------------------------------------------------------------- workloads
@dataclass
class Pair:
    """One reference/target pair, float32 images as handed to the fit."""
    R: np.ndarray
    I: np.ndarray
    m: int
    K_true: np.ndarray
    B0_true: float
    sigma0_adu: float
    gain: float
    I_noiseless: np.ndarray | None = None
    meta: dict = field(default_factory=dict)


@dataclass
class Epoch:
    I: np.ndarray
    row0: int
    col0: int
    K_true: np.ndarray
    B0_true: float


@dataclass
class Batch:
    R: np.ndarray
    epochs: list
    m: int
    sigma0_adu: float
    gain: float
    meta: dict = field(default_factory=dict)


def star_field(rng, H, W, n_stars, flux_min, flux_max, psf_kind, fwhm, sky, beta=3.0):
    x = rng.uniform(0.0, W, n_stars)
    y = rng.uniform(0.0, H, n_stars)
    flux = 10.0 ** rng.uniform(math.log10(flux_min), math.log10(flux_max), n_stars)
    psf = gaussian_psf(fwhm) if psf_kind == "gauss" else moffat_psf(fwhm, beta)
    radius = int(math.ceil(10 * fwhm))
    return render_stars((H, W), x, y, flux, psf, radius, sky)


def smooth_background(H: int, W: int, tilt_x: float, tilt_y: float, bump: float) -> np.ndarray:
    """A smooth differential-background field on an H x W grid: a plane of the given end-to-end
    tilts (ADU across the image) plus a wide Gaussian bump of the given height off the centre."""
    r, c = np.mgrid[0:H, 0:W].astype(np.float64)
    s = 0.4 * max(H, W)
    return (tilt_x * (c / W - 0.5) + tilt_y * (r / H - 0.5)
            + bump * np.exp(-((r - 0.3 * H) ** 2 + (c - 0.6 * W) ** 2) / (2.0 * s * s)))


def make_pair(H, W, m, *, n_stars, flux_min, flux_max, psf_kind, fwhm, sky, K_true, B0,
              sigma0_e, gain, noise=True, config=0, epoch=0, background=None) -> Pair:
    """A reference star field and its target R (x) K_true + B0 (+ the field ``background`` when given),
    with CCD noise."""
    rng = rng_for(config, epoch)
    R = star_field(rng, H, W, n_stars, flux_min, flux_max, psf_kind, fwhm, sky)
    R32 = R.astype(np.float32)
    I_nl = correlate_target(R32.astype(np.float64), K_true, B0)
    if background is not None:
        I_nl = I_nl + background
    I = add_ccd_noise(I_nl, gain, sigma0_e, rng) if noise else I_nl
    return Pair(R=R32, I=I.astype(np.float32), m=m, K_true=K_true, B0_true=B0,
                sigma0_adu=sigma0_e / gain, gain=gain, I_noiseless=I_nl,
                meta=dict(H=H, W=W, n_stars=n_stars, psf=psf_kind, fwhm=fwhm, sky=sky))


def config1(noise=True) -> Pair:
    """128^2, 150 stars (1e2..1e5), Gaussian PSF FWHM 2, sky 100; 9x9 Gaussian kernel FWHM 1.5,
    offset (+0.3, +0.3), sum 1.1; B0 = 5; sigma0 = 5 e-, G = 1."""
    K = kernel_gaussian(9, 1.5, dx=0.3, dy=0.3, total=1.1)
    return make_pair(128, 128, 9, n_stars=150, flux_min=1e2, flux_max=1e5, psf_kind="gauss", fwhm=2.0,
                     sky=100.0, K_true=K, B0=5.0, sigma0_e=5.0, gain=1.0, noise=noise, config=1)


def config_varying_background(size: int = 128, m: int = 9, noise: bool = True) -> Pair:
    """A pair whose differential background varies over the field (Section 2.6's case): config 1's
    star field, PSF and kernel shape (m x m) at size^2 (150 stars per 128^2), with a tilt of 12 and
    -7 ADU across the image and a bump of 9 ADU added to the target before the noise."""
    K = kernel_gaussian(m, 1.5, dx=0.3, dy=0.3, total=1.1)
    n = int(round(150 * (size / 128) ** 2))
    return make_pair(size, size, m, n_stars=n, flux_min=1e2, flux_max=1e5, psf_kind="gauss", fwhm=2.0,
                     sky=100.0, K_true=K, B0=5.0, sigma0_e=5.0, gain=1.0, noise=noise, config=7,
                     background=smooth_background(size, size, 12.0, -7.0, 9.0))


def config2(noise=True, size=1024) -> Pair:
    """1024^2, 5000 stars (1e2..1e6), Moffat beta 3 FWHM 3, sky 500; 19x19 elliptical Gaussian
    kernel FWHM 2.2 x 1.8 rotated 30 deg, sum 0.9; B0 = -12; sigma0 = 8 e-, G = 1.5."""
    K = kernel_gaussian(19, 2.2, 1.8, rot_deg=30.0, total=0.9)
    n = int(round(5000 * (size / 1024) ** 2))
    return make_pair(size, size, 19, n_stars=n, flux_min=1e2, flux_max=1e6, psf_kind="moffat", fwhm=3.0,
                     sky=500.0, K_true=K, B0=-12.0, sigma0_e=8.0, gain=1.5, noise=noise, config=2)


def config3(noise=True, size=4096) -> Pair:
    """4096^2 CCD-sized pair, 80,000 stars, Moffat FWHM 3.5; everything else as config 2."""
    K = kernel_gaussian(19, 2.2, 1.8, rot_deg=30.0, total=0.9)
    n = int(round(80000 * (size / 4096) ** 2))
    return make_pair(size, size, 19, n_stars=n, flux_min=1e2, flux_max=1e6, psf_kind="moffat", fwhm=3.5,
                     sky=500.0, K_true=K, B0=-12.0, sigma0_e=8.0, gain=1.5, noise=noise, config=3)


def crop(pair: Pair, size: int) -> Pair:
    """Central size x size crop of a pair (the same pixels of R and I)."""
    H, W = pair.R.shape
    r0, c0 = (H - size) // 2, (W - size) // 2
    sl = (slice(r0, r0 + size), slice(c0, c0 + size))
    return Pair(R=np.ascontiguousarray(pair.R[sl]), I=np.ascontiguousarray(pair.I[sl]), m=pair.m,
                K_true=pair.K_true, B0_true=pair.B0_true, sigma0_adu=pair.sigma0_adu, gain=pair.gain,
                I_noiseless=None if pair.I_noiseless is None else pair.I_noiseless[sl],
                meta=dict(pair.meta, crop=size))


def _batched_epoch(config: int, e: int, R64: np.ndarray, m: int, ref_size: int, side_range, noise: bool,
                   gain: float, sigma0_e: float) -> Epoch:
    """Epoch e of a batch: everything it draws comes from its own stream rng_for(config, e + 1)."""
    er = rng_for(config, e + 1)
    lo, hi = side_range
    side = int(er.integers(lo, hi + 1))
    r0 = int(er.integers(0, ref_size - side + 1))
    c0 = int(er.integers(0, ref_size - side + 1))
    K = kernel_gaussian(m, er.uniform(1.2, 3.0), dx=er.uniform(-0.5, 0.5), dy=er.uniform(-0.5, 0.5),
                        total=er.uniform(0.7, 1.3))
    B0 = float(er.uniform(-50.0, 50.0))
    I_nl = correlate_target(R64[r0:r0 + side, c0:c0 + side], K, B0)
    I = add_ccd_noise(I_nl, gain, sigma0_e, er) if noise else I_nl
    return Epoch(I=I.astype(np.float32), row0=r0, col0=c0, K_true=K, B0_true=B0)


def _map_epochs(fn, n_epochs: int, workers: int):
    """[fn(0), ..., fn(n_epochs - 1)], on that many threads of this process when workers > 1 (the FFTs and
    the random draws release the GIL; no child process is started, so callers need no __main__ guard
    and a profiler attached to this process sees no extra processes)."""
    if workers > 1 and n_epochs > 1:
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(min(workers, n_epochs)) as ex:
            return list(ex.map(fn, range(n_epochs)))
    return [fn(e) for e in range(n_epochs)]


def batched(config: int, n_epochs: int, m: int, ref_size: int, n_stars: int, side_range, *,
            fwhm=3.0, noise=True, workers: int = 1) -> Batch:
    """Shared reference star field with per-epoch targets cut from it.

    Each epoch e draws a square side in ``side_range`` (inclusive), a crop offset uniform in
    [0, ref_size - side], a Gaussian kernel with FWHM ~ U(1.2, 3.0), sum ~ U(0.7, 1.3) and
    subpixel offset ~ U(-0.5, 0.5)^2, and B0 ~ U(-50, 50).  With workers > 1 the epochs are made
    on that many threads (identical result: each epoch has its own random stream)."""
    rng = rng_for(config, 0)
    R = star_field(rng, ref_size, ref_size, n_stars, 1e2, 1e6, "moffat", fwhm, 500.0).astype(np.float32)
    R64 = R.astype(np.float64)
    gain, sigma0_e = 1.5, 8.0
    tail = (m, ref_size, side_range, noise, gain, sigma0_e)
    epochs = _map_epochs(lambda e: _batched_epoch(config, e, R64, *tail), n_epochs, workers)
    return Batch(R=R, epochs=epochs, m=m, sigma0_adu=sigma0_e / gain, gain=gain,
                 meta=dict(config=config, ref_size=ref_size, n_stars=n_stars, side_range=side_range))


def config4(noise=True, n_epochs=64, ref_size=2048, side_range=(512, 2048), workers=1) -> Batch:
    """64 epochs of side U{512..2048} cut from a shared 2048^2 reference (30,000 stars), 17x17 kernels."""
    n = int(round(30000 * (ref_size / 2048) ** 2))
    return batched(4, n_epochs, 17, ref_size, n, side_range, noise=noise, workers=workers)


def config5(noise=True, n_epochs=256, ref_size=2048, workers=1) -> Batch:
    """256 epochs at 2048^2 against one shared 2048^2 reference (40,000 stars), 25x25 kernels."""
    n = int(round(40000 * (ref_size / 2048) ** 2))
    return batched(5, n_epochs, 25, ref_size, n, (ref_size, ref_size), noise=noise, workers=workers)


# ------------------------------------------------- many small aligned pairs (the EMCCD speed test)
EMCCD_PHI_R = 1.82   # reference PSF width (FWHM, pixels; Section 5.1)
EMCCD_GAIN = 1.0     # ADU per detected photon after the EM stage
EMCCD_EXCESS = 2.0   # excess noise factor E of the EM register


def _emccd_epoch(e: int, R64: np.ndarray, F: np.ndarray, m: int, noise: bool):
    """Target e: the reference broadened to a target PSF width phi_I ~ U(2.2, 4.2) px (median ~3.2;
    widths are FWHM, the usual measure of an observed PSF) by a Gaussian kernel of FWHM
    sqrt(phi_I^2 - phi_R^2) (0.5 to 1.5 px standard deviation: from under-sampled to broad), sum
    ~ U(0.8, 1.2), subpixel offset ~ U(-0.3, 0.3)^2, B0 ~ U(-20, 20); noise with the EMCCD
    variance E max(I, 0) / (G F)."""
    er = rng_for(6, e + 1)
    phi_I = float(er.uniform(2.2, 4.2))
    K = kernel_gaussian(m, math.sqrt(phi_I ** 2 - EMCCD_PHI_R ** 2), dx=er.uniform(-0.3, 0.3),
                        dy=er.uniform(-0.3, 0.3), total=er.uniform(0.8, 1.2))
    B0 = float(er.uniform(-20.0, 20.0))
    I = correlate_target(R64, K, B0)
    if noise:
        I = I + np.sqrt(EMCCD_EXCESS * np.clip(I, 0.0, None) / (EMCCD_GAIN * F)) * er.standard_normal(I.shape)
    return Epoch(I=I.astype(np.float32), row0=0, col0=0, K_true=K, B0_true=B0), phi_I


def config_emccd(n_epochs: int = 158, size: int = 482, m: int = 19, noise: bool = True, workers: int = 1) -> Batch:
    """Many small aligned pairs shaped like the EMCCD speed test (Section 5.1): a size^2 field of
    2,000 stars (fluxes log-uniform 1e2..1e5, Gaussian PSF of FWHM phi_R, sky 200) as the shared
    reference, one flat field F ~ U(0.95, 1.05) per pixel used by every target, and n_epochs
    targets of the whole field.  meta holds phi_R, each target's phi_I, the flat, gain and E."""
    n_stars = int(round(2000 * (size / 482) ** 2))
    R = star_field(rng_for(6, 0), size, size, n_stars, 1e2, 1e5, "gauss", EMCCD_PHI_R, 200.0).astype(np.float32)
    F = rng_for(6, 100000).uniform(0.95, 1.05, (size, size))
    R64 = R.astype(np.float64)
    out = _map_epochs(lambda e: _emccd_epoch(e, R64, F, m, noise), n_epochs, workers)
    return Batch(R=R, epochs=[o[0] for o in out], m=m, sigma0_adu=0.0, gain=EMCCD_GAIN,
                 meta=dict(config="emccd", size=size, n_stars=n_stars, phi_R=EMCCD_PHI_R,
                           phi_I=[o[1] for o in out], flat=F.astype(np.float32), excess=EMCCD_EXCESS))


def paper_reference(size: int = 142, seed: int = 0, phi_R: float | None = None) -> np.ndarray:
    """Noiseless reference following Section 3.1 steps (i)-(v): Gaussian PSF with standard deviation
    phi_R ~ U(0.5, 2.5), lg star density per 100x100 px ~ U(0, 3), F^(-3/2) ~ U(1e-9, 10^-4.5),
    the brightest star moved to the centre, sky ~ U(10, 1000)."""
    rng = rng_for(0, 1000 + seed)
    if phi_R is None:
        phi_R = rng.uniform(0.5, 2.5)
    lg_rho = rng.uniform(0.0, 3.0)
    n = max(1, int(round(10.0 ** lg_rho * (size / 100.0) ** 2)))
    x = rng.uniform(0.0, size, n)
    y = rng.uniform(0.0, size, n)
    f = rng.uniform(1e-9, 10 ** -4.5, n) ** (-2.0 / 3.0)
    k = int(np.argmax(f))
    x[k] = y[k] = size / 2.0
    fwhm = phi_R * FWHM_PER_SIGMA
    return render_stars((size, size), x, y, f, gaussian_psf(fwhm), int(math.ceil(10 * fwhm)),
                        rng.uniform(10.0, 1000.0))
