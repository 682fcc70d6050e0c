"""Small problems for the oracle's pins (full-sky Gauss-Legendre grids, tiny HEALPix maps)."""
import numpy as np

from paper_2605_21149_amd import inputs as I


def gl_grid(lmax):
    """Gauss-Legendre nodes in cos(theta) (lmax+1) x (2 lmax + 1) equispaced phi, with the
    quadrature weight of each pixel; exact for products of harmonics up to lmax."""
    x, wx = np.polynomial.legendre.leggauss(lmax + 1)
    nphi = 2 * lmax + 1
    th = np.repeat(np.arccos(x), nphi)
    ph = np.tile(2 * np.pi * np.arange(nphi) / nphi, lmax + 1)
    w = np.repeat(wx, nphi) * (2 * np.pi / nphi)
    return th, ph, w


def random_spectra(lmax, seed, cross=True):
    rng = np.random.default_rng(seed)
    cl = np.zeros((6, lmax + 1))
    cl[0, 2:] = rng.uniform(1.0, 3.0, lmax - 1)
    cl[1, 2:] = rng.uniform(0.5, 1.5, lmax - 1)
    cl[2, 2:] = rng.uniform(0.2, 0.8, lmax - 1)
    if cross:
        # |TE|, |TB|, |EB| small enough to keep every 3x3 block positive definite
        cl[3, 2:] = rng.uniform(-0.3, 0.3, lmax - 1) * np.sqrt(cl[0, 2:] * cl[1, 2:])
        cl[4, 2:] = rng.uniform(-0.2, 0.2, lmax - 1) * np.sqrt(cl[0, 2:] * cl[2, 2:])
        cl[5, 2:] = rng.uniform(-0.2, 0.2, lmax - 1) * np.sqrt(cl[1, 2:] * cl[2, 2:])
    return cl


def gl_problem(fields, lmax, nu, seed=7, beam_fwhm=None):
    th, ph, w = gl_grid(lmax)
    cl = random_spectra(lmax, seed)
    bl = np.ones(lmax + 1) if beam_fwhm is None else I.gaussian_beam(lmax, beam_fwhm)
    p = I.Problem(f"gl_{fields}", fields, 2, lmax, cl, bl, np.ones(lmax + 1), 0, None, th, ph)
    nm = len(fields) if fields != "QU" else 2
    nm = {"T": 1, "QU": 2, "TQU": 3}[fields]
    p.noise_diag = np.tile(nu / w, nm)
    p.extra["weights"] = w
    return p


def tiny_healpix(fields, nside=2, lmax=6, cut=0.3, seed=11, noise=0.5, lowrank=0):
    mask = I.mask_abs_z_above(nside, cut)
    cl = random_spectra(lmax, seed)
    p = I.Problem(f"tiny_{fields}", fields, 2, lmax, cl, I.gaussian_beam(lmax, 1200.0),
                  I.disc_pixel_window(lmax, nside), nside, mask)
    p.noise_diag = np.full(p.n, noise)
    if lowrank:
        p.noise_U = 0.3 * I.smooth_modes(nside, mask, p.nmaps, lowrank, seed + 1)
    return p
