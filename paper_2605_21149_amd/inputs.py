"""Seeded synthetic inputs shared by the HIP path's harness and the oracle's tests.

This module only *synthesises inputs*: masks, beams, pixel windows, power
spectra, noise covariances, scan parameter points and white-noise draws.  It
holds none of the method's arithmetic (no covariance assembly, no harmonic
basis, no solves); both the CPU oracle and the HIP path receive exactly the
arrays produced here.

Everything is seeded (numpy PCG64) so that each workload is reproducible.
The workloads follow the paper's statement of the problem (masked HEALPix
maps of T and/or Q,U, a power spectrum, a beam and a pixel window, a general
SPD noise covariance; Sect. 2.1 and App. A):

* spectra: TT = 1000/(l(l+1)) uK^2, EE = 0.05 TT plus a reionisation bump of
  0.05 uK^2 below l = 10, BB = 1e-3 EE, TE = 0.3 sqrt(TT EE), TB = EB = 0;
* Gaussian beams; an equal-area top-hat disc stands in for the HEALPix pixel
  window (the tabulated window is not available);
* masks are RING-ordered keep-flags built from latitude cuts or a seeded
  hemisphere;
* noise = sigma^2 I (+ U U^T with seeded smooth large-scale modes).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

SPEC_NAMES = ("TT", "EE", "BB", "TE", "TB", "EB")
ARCMIN = math.pi / (180.0 * 60.0)


# ----------------------------------------------------------------------------
# HEALPix RING positions, used here only to decide which pixels a mask keeps
# and to shape smooth noise modes (input synthesis; not part of the method).
# ----------------------------------------------------------------------------
def _ring_positions(nside: int):
    zs, phis = [], []
    for i in range(1, 4 * nside):
        if i < nside:
            nr, z, shift = 4 * i, 1.0 - i * i / (3.0 * nside * nside), 0.5
            dphi = math.pi / (2 * i)
        elif i <= 3 * nside:
            nr, z = 4 * nside, 4.0 / 3.0 - 2.0 * i / (3.0 * nside)
            shift = 1.0 - 0.5 * ((i - nside + 1) % 2)
            dphi = math.pi / (2 * nside)
        else:
            k = 4 * nside - i
            nr, z, shift = 4 * k, -(1.0 - k * k / (3.0 * nside * nside)), 0.5
            dphi = math.pi / (2 * k)
        zs.append(np.full(nr, z))
        phis.append((np.arange(1, nr + 1) - shift) * dphi)
    return np.concatenate(zs), np.concatenate(phis)


def _ring_vectors(nside: int) -> np.ndarray:
    z, phi = _ring_positions(nside)
    r = np.sqrt(np.clip(1.0 - z * z, 0.0, None))
    return np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)


def mask_abs_z_above(nside: int, sin_cut: float) -> np.ndarray:
    """Keep-flags (uint8, RING order) for |z| > sin_cut (a symmetric latitude cut)."""
    z, _ = _ring_positions(nside)
    return (np.abs(z) > sin_cut).astype(np.uint8)


def mask_hemisphere(nside: int, seed: int) -> np.ndarray:
    """Keep-flags for the hemisphere around a seeded random direction (contiguous, ~50 %)."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(3)
    v /= np.linalg.norm(v)
    return (_ring_vectors(nside) @ v > 0.0).astype(np.uint8)


# ----------------------------------------------------------------------------
# Spectra, beams, windows
# ----------------------------------------------------------------------------
def fiducial_spectra(lmax: int, bump: bool = True) -> np.ndarray:
    """[6][lmax+1] uK^2 in TT, EE, BB, TE, TB, EB order; l = 0, 1 are zero."""
    cl = np.zeros((6, lmax + 1))
    ell = np.arange(2, lmax + 1, dtype=np.float64)
    tt = 1000.0 / (ell * (ell + 1.0))
    ee = 0.05 * tt + (0.05 * (ell < 10) if bump else 0.0)
    cl[0, 2:] = tt
    cl[1, 2:] = ee
    cl[2, 2:] = 1e-3 * ee
    cl[3, 2:] = 0.3 * np.sqrt(tt * ee)
    return cl


def gaussian_beam(lmax: int, fwhm_arcmin: float) -> np.ndarray:
    sigma = fwhm_arcmin * ARCMIN / math.sqrt(8.0 * math.log(2.0))
    ell = np.arange(lmax + 1, dtype=np.float64)
    return np.exp(-0.5 * ell * (ell + 1.0) * sigma * sigma)


def disc_pixel_window(lmax: int, nside: int) -> np.ndarray:
    """Window of a top-hat disc with the area of one HEALPix pixel.

    A normalised cap of opening angle t0 has Legendre coefficients
    [P_{l-1}(x0) - P_{l+1}(x0)] / ((2l+1)(1-x0)), x0 = cos t0, and value 1 at l=0.
    """
    x0 = 1.0 - 1.0 / (6.0 * nside * nside)  # 2 pi (1 - x0) = 4 pi / (12 nside^2)
    p = np.zeros(lmax + 2)
    p[0], p[1] = 1.0, x0
    for l in range(1, lmax + 1):
        p[l + 1] = ((2 * l + 1) * x0 * p[l] - l * p[l - 1]) / (l + 1)
    w = np.ones(lmax + 1)
    for l in range(1, lmax + 1):
        w[l] = (p[l - 1] - p[l + 1]) / ((2 * l + 1) * (1.0 - x0))
    return w


# ----------------------------------------------------------------------------
# Noise
# ----------------------------------------------------------------------------
def smooth_modes(nside: int, keep: np.ndarray, nfields: int, nmodes: int, seed: int,
                 amp: float = 1.0) -> np.ndarray:
    """[n][nmodes] seeded smooth large-scale patterns over the kept pixels.

    Each column holds, independently on every field block, a random polynomial
    of degree <= 4 in the pixel's Cartesian coordinates (the span of the l <= 4
    harmonics), scaled to an rms of ``amp`` uK over the kept pixels.
    """
    rng = np.random.default_rng(seed)
    v = _ring_vectors(nside)[keep.astype(bool)]
    x, y, z = v[:, 0], v[:, 1], v[:, 2]
    monos = []
    for a in range(5):
        for b in range(5 - a):
            for c in range(5 - a - b):
                if a + b + c >= 1:
                    monos.append(x ** a * y ** b * z ** c)
    basis = np.stack(monos, axis=1)
    npx = v.shape[0]
    U = np.zeros((nfields * npx, nmodes))
    for k in range(nmodes):
        for f in range(nfields):
            col = basis @ rng.standard_normal(basis.shape[1])
            col -= col.mean()
            col *= amp / np.sqrt(np.mean(col * col))
            U[f * npx:(f + 1) * npx, k] = col
    return U


# ----------------------------------------------------------------------------
# Problem descriptions
# ----------------------------------------------------------------------------
FIELDS_NMAPS = {"T": 1, "QU": 2, "TQU": 3}


@dataclass
class Problem:
    """One masked-map problem in the paper's terms: geometry, spectra, beam, window, noise."""
    name: str
    fields: str                      # "T", "QU" or "TQU"; data order [T | Q | U]
    lmin: int
    lmax: int
    cl: np.ndarray                   # [6][lmax+1]
    bl: np.ndarray                   # [lmax+1]
    pl: np.ndarray                   # [lmax+1]
    nside: int = 0
    mask: Optional[np.ndarray] = None    # uint8 [12 nside^2], 1 = keep
    theta: Optional[np.ndarray] = None   # explicit directions when nside == 0
    phi: Optional[np.ndarray] = None
    noise_diag: Optional[np.ndarray] = None    # [n]
    noise_U: Optional[np.ndarray] = None       # [n][rank]; N = diag + U U^T
    noise_dense: Optional[np.ndarray] = None   # [n][n]; overrides the two above
    extra: dict = field(default_factory=dict)

    @property
    def npix(self) -> int:
        if self.nside:
            return int(self.mask.sum()) if self.mask is not None else 12 * self.nside ** 2
        return int(self.theta.shape[0])

    @property
    def nmaps(self) -> int:
        return FIELDS_NMAPS[self.fields]

    @property
    def n(self) -> int:
        return self.npix * self.nmaps

    def noise_matrix(self) -> np.ndarray:
        if self.noise_dense is not None:
            return self.noise_dense
        N = np.diag(self.noise_diag)
        if self.noise_U is not None:
            N = N + self.noise_U @ self.noise_U.T
        return N


def spin0_problem_nside8() -> Problem:
    """T only, N_side = 8, |z| > sin 15 deg, l in [2, 24], 440' beam, white noise 1 + 1e-2 uK^2."""
    nside, lmax = 8, 24
    mask = mask_abs_z_above(nside, math.sin(math.radians(15.0)))
    p = Problem("spin0_nside8", "T", 2, lmax, fiducial_spectra(lmax),
                gaussian_beam(lmax, 440.0), disc_pixel_window(lmax, nside), nside, mask)
    p.noise_diag = np.full(p.n, 1.0 + 1e-2)
    return p


def tqu_problem_nside16(dense_noise: bool = True, seed_modes: int = 201) -> Problem:
    """TQU, N_side = 16, |b| > 20 deg (map in Galactic frame), l in [2, 47], 220' beam,
    noise 2 uK^2 I + U U^T with 20 seeded smooth modes."""
    nside, lmax = 16, 47
    mask = mask_abs_z_above(nside, math.sin(math.radians(20.0)))
    p = Problem("tqu_nside16", "TQU", 2, lmax, fiducial_spectra(lmax),
                gaussian_beam(lmax, 220.0), disc_pixel_window(lmax, nside), nside, mask)
    p.noise_diag = np.full(p.n, 2.0)
    p.noise_U = smooth_modes(nside, mask, 3, 20, seed_modes)
    if dense_noise:
        p.noise_dense = p.noise_matrix()
    return p


def qu_problem_nside32(seed_mask: int = 301) -> Problem:
    """QU, N_side = 32, seeded hemisphere (~50 %), l in [2, 95], 110' beam,
    white noise 0.5 + 1e-3 uK^2; EE with bump and BB = 1e-3 EE, EB = 0."""
    nside, lmax = 32, 95
    mask = mask_hemisphere(nside, seed_mask)
    cl = fiducial_spectra(lmax)
    cl[0] = 0.0
    cl[3] = 0.0
    p = Problem("qu_nside32", "QU", 2, lmax, cl, gaussian_beam(lmax, 110.0),
                disc_pixel_window(lmax, nside), nside, mask)
    p.noise_diag = np.full(p.n, 0.5 + 1e-3)
    return p


def qu_scan_problem(nside: int) -> Problem:
    """QU likelihood-scan problems: N_side 8 (the spin-0 N_side 8 problem's cut and beam, white
    noise 1 + 1e-2) or N_side 16 (the TQU N_side 16 problem's cut and beam, noise 2 I + U U^T on
    Q,U)."""
    if nside == 8:
        lmax, cut, fwhm = 24, 15.0, 440.0
    elif nside == 16:
        lmax, cut, fwhm = 47, 20.0, 220.0
    else:
        raise ValueError("scan problems exist for N_side 8 and 16")
    mask = mask_abs_z_above(nside, math.sin(math.radians(cut)))
    cl = fiducial_spectra(lmax)
    cl[0] = 0.0
    cl[3] = 0.0
    p = Problem(f"qu_scan_nside{nside}", "QU", 2, lmax, cl, gaussian_beam(lmax, fwhm),
                disc_pixel_window(lmax, nside), nside, mask)
    if nside == 8:
        p.noise_diag = np.full(p.n, 1.0 + 1e-2)
    else:
        p.noise_diag = np.full(p.n, 2.0)
        p.noise_U = smooth_modes(nside, mask, 2, 20, 201)
    return p


# ----------------------------------------------------------------------------
# Bins
# ----------------------------------------------------------------------------
@dataclass
class Bins:
    lo: np.ndarray
    hi: np.ndarray
    spectra: tuple  # subset of SPEC_NAMES, in SPEC_NAMES order

    @property
    def nbins(self) -> int:
        return int(self.lo.shape[0])

    @property
    def mask_bits(self) -> int:
        return sum(1 << SPEC_NAMES.index(s) for s in self.spectra)


def uniform_bins(lmin: int, lmax: int, delta: int, spectra) -> Bins:
    lo = np.arange(lmin, lmax + 1, delta, dtype=np.int32)
    hi = np.minimum(lo + delta - 1, lmax).astype(np.int32)
    order = tuple(s for s in SPEC_NAMES if s in spectra)
    return Bins(lo, hi, order)


def spectra_for_fields(fields: str):
    return {"T": ("TT",), "QU": ("EE", "BB", "EB"),
            "TQU": SPEC_NAMES}[fields]


# ----------------------------------------------------------------------------
# Likelihood-scan parameter points (7 parameters: 6 EE band amplitudes + bump)
# ----------------------------------------------------------------------------
EE_BANDS = ((2, 6), (7, 11), (12, 16), (17, 21), (22, 25), (26, 29))


def scan_points(npoints: int, seed: int = 401, lo: float = 0.5, hi: float = 1.5) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=(npoints, 7))


def scan_spectra(theta: np.ndarray, base_cl: np.ndarray) -> np.ndarray:
    """Per-point spectra [npoints][6][lmax+1]: EE for l <= 29 is a_b 0.05 TT + A 0.05 [l <= 9];
    every other multipole and spectrum stays at base_cl."""
    theta = np.atleast_2d(theta)
    lmax = base_cl.shape[1] - 1
    out = np.repeat(base_cl[None], theta.shape[0], axis=0).copy()
    ell = np.arange(lmax + 1, dtype=np.float64)
    tt = np.zeros(lmax + 1)
    tt[2:] = 1000.0 / (ell[2:] * (ell[2:] + 1.0))
    for b, (l0, l1) in enumerate(EE_BANDS):
        l1 = min(l1, lmax)
        if l0 > lmax:
            continue
        sl = slice(l0, l1 + 1)
        bump = 0.05 * (ell[sl] <= 9)
        out[:, 1, sl] = theta[:, b:b + 1] * 0.05 * tt[sl] + theta[:, 6:7] * bump
    return out


def white_maps(n: int, nmaps: int, seed: int, rms: float = 1.0) -> np.ndarray:
    """[nmaps][n] seeded standard-normal draws times ``rms``."""
    rng = np.random.default_rng(seed)
    return rms * rng.standard_normal((nmaps, n))
