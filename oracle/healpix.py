"""HEALPix RING pixel centres (Gorski et al. 2005), the pixelisation of Sect. 2.1.

Oracle code: test infrastructure only (see oracle/__init__.py).
"""
import numpy as np


def ring_theta_phi(nside):
    """Colatitude and longitude of every pixel centre, RING order.

    Rings i = 1 .. 4 nside - 1.  North polar cap (i < nside): 4i pixels,
    z = 1 - i^2 / (3 nside^2), phi = pi/(2i) (j - 1/2).  Equatorial belt
    (nside <= i <= 3 nside): 4 nside pixels, z = 4/3 - 2i/(3 nside),
    phi = pi/(2 nside) (j - 1 + s/2) with s = (i - nside + 1) mod 2, so that rings with
    s = 0 start at phi = 0 (the labelling of the standard HEALPix library).  The south
    cap mirrors the north one.
    """
    thetas, phis = [], []
    for i in range(1, 4 * nside):
        if i < nside:
            npr = 4 * i
            z = 1.0 - i * i / (3.0 * nside * nside)
            ph = np.pi / (2.0 * i) * (np.arange(1, npr + 1) - 0.5)
        elif i <= 3 * nside:
            npr = 4 * nside
            z = 4.0 / 3.0 - 2.0 * i / (3.0 * nside)
            s = (i - nside + 1) % 2
            ph = np.pi / (2.0 * nside) * (np.arange(1, npr + 1) - 1.0 + 0.5 * s)
        else:
            k = 4 * nside - i
            npr = 4 * k
            z = -(1.0 - k * k / (3.0 * nside * nside))
            ph = np.pi / (2.0 * k) * (np.arange(1, npr + 1) - 0.5)
        thetas.append(np.full(npr, np.arccos(z)))
        phis.append(ph)
    return np.concatenate(thetas), np.concatenate(phis)


def unit_vectors(theta, phi):
    st = np.sin(theta)
    return np.stack([st * np.cos(phi), st * np.sin(phi), np.cos(theta)], axis=1)


def active_directions(nside, mask=None, theta=None, phi=None):
    """(theta, phi) of the retained pixels: RING centres filtered by the keep-mask,
    or explicit directions when nside == 0."""
    if nside:
        th, ph = ring_theta_phi(nside)
        if mask is not None:
            keep = np.asarray(mask).astype(bool)
            th, ph = th[keep], ph[keep]
        return th, ph
    return np.asarray(theta, dtype=np.float64), np.asarray(phi, dtype=np.float64)
