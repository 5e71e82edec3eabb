"""CPU oracle of Taylor lensing on HEALPix rings -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  It shares no code with the GPU library
and never imports it; it builds on ``oracle.taylens_oracle`` (harmonic sums,
positions, Taylor sum, rotation).

The paper simulates HEALPix maps and interpolates on them (Sec. II.A-B):
for every output pixel x the displaced position x' = x + grad phi is found,
the pixel containing x' (``ang2pix``) and its centre x0' (``pix2ang``) give
the sub-pixel offset x' - x0', and eq. 5 sums the Taylor series of T, Q, U
about x0' with the derivatives at that centre.  Here the derivatives come
from the harmonic coefficients directly (the theta part from the oracle's
recursions at the ring colatitude, the phi part as sum_m (i m)^k F_m
e^{i m phi}), and Q/U are rotated by the parallel transport R (eq. 2).

HEALPix ring geometry (RING ordering), as published by Gorski et al. (2005),
for resolution nside, npix = 12 nside^2, rings i = 1 .. 4 nside - 1:
* north polar cap, i < nside: z = 1 - i^2 / (3 nside^2), 4 i pixels at
  phi = (pi / (2 i)) (k + 1/2), first pixel 2 i (i - 1);
* equatorial belt, nside <= i <= 3 nside: z = 4/3 - 2 i / (3 nside),
  4 nside pixels at phi = (pi / (2 nside)) (k + s / 2), s = (i - nside + 1)
  mod 2, first pixel 2 nside (nside - 1) + 4 nside (i - nside);
* south polar cap, i > 3 nside: the mirror image of ring 4 nside - i.
``ang2pix`` locates the pixel containing a direction with the published
construction: in the belt (|z| <= 2/3) by the two families of pixel edge
lines phi/(pi/2) nside +- (3/4) nside z, in the caps by the same lines in
the variable nside sqrt(3 (1 - |z|)).
"""
from __future__ import annotations

import math

import numpy as np

from oracle import taylens_oracle as tor


# ------------------------------------------------------------ geometry ----

def npix(nside: int) -> int:
    return 12 * nside * nside


def ring_geometry(nside: int):
    """Per ring (index 0 .. 4 nside - 2 = HEALPix ring 1 .. 4 nside - 1):
    theta, number of pixels, phi of the first pixel, first pixel index.
    Colatitudes come from sin(theta/2) in the caps (no loss near the
    poles) and from z in the belt."""
    nr = 4 * nside - 1
    theta = np.empty(nr)
    nphi = np.empty(nr, dtype=np.int64)
    phi0 = np.empty(nr)
    start = np.empty(nr, dtype=np.int64)
    for r in range(nr):
        i = r + 1
        north = i <= 2 * nside
        ii = i if north else 4 * nside - i           # ring counted from the nearer pole
        if ii < nside:                               # polar cap
            th = 2.0 * math.asin(ii / (math.sqrt(6.0) * nside))
            n = 4 * ii
            p0 = math.pi / (4.0 * ii)
        else:                                        # belt (ring counted from the north)
            z = 4.0 / 3.0 - 2.0 * i / (3.0 * nside)
            th = math.acos(z)
            n = 4 * nside
            s = (i - nside + 1) % 2                    # 1: rings shifted by half a pixel
            p0 = math.pi * s / (4.0 * nside)
        if ii < nside and not north:
            th = math.pi - th
        theta[r] = th
        nphi[r] = n
        phi0[r] = p0
    # first pixel of each ring: cumulative counts
    start[0] = 0
    start[1:] = np.cumsum(nphi)[:-1]
    return theta, nphi, phi0, start


def pix2ang(nside: int, pix):
    """Pixel centres (theta, phi) of RING-ordered pixel indices."""
    theta, nphi, phi0, start = ring_geometry(nside)
    pix = np.asarray(pix, dtype=np.int64)
    r = np.searchsorted(start, pix, side="right") - 1
    k = pix - start[r]
    return theta[r], phi0[r] + 2.0 * math.pi * k / nphi[r]


def ang2pix(nside: int, theta, phi):
    """RING index of the pixel containing each direction (theta, phi)."""
    theta = np.asarray(theta, dtype=np.float64)
    phi = np.asarray(phi, dtype=np.float64)
    theta, phi = np.broadcast_arrays(theta, phi)
    z = np.cos(theta)
    za = np.abs(z)
    tt = np.mod(phi, 2.0 * math.pi) / (0.5 * math.pi)       # in [0, 4)
    tt = np.where(tt >= 4.0, 0.0, tt)
    out = np.empty(theta.shape, dtype=np.int64)
    belt = za <= 2.0 / 3.0
    # equatorial belt
    t1 = nside * (0.5 + tt[belt])
    t2 = nside * z[belt] * 0.75
    jp = np.floor(t1 - t2).astype(np.int64)                  # ascending edge line index
    jm = np.floor(t1 + t2).astype(np.int64)                  # descending edge line index
    ir = nside + 1 + jp - jm                                 # ring from z = 2/3, 1 .. 2 nside + 1
    kshift = 1 - (ir & 1)
    ip = (jp + jm - nside + kshift + 1) // 2
    ip = np.mod(ip, 4 * nside)
    out[belt] = 2 * nside * (nside - 1) + (ir - 1) * 4 * nside + ip
    # polar caps: nside sqrt(3 (1 - |z|)) = nside sin(theta) sqrt(3 / (1 + |z|))
    cap = ~belt
    tp = tt[cap] - np.floor(tt[cap])
    tmp = nside * np.sin(theta[cap]) * np.sqrt(3.0 / (1.0 + za[cap]))
    jp = np.floor(tp * tmp).astype(np.int64)
    jm = np.floor((1.0 - tp) * tmp).astype(np.int64)
    ir = jp + jm + 1                                         # ring from the nearer pole
    ip = np.floor(tt[cap] * ir).astype(np.int64)
    ip = np.mod(ip, 4 * ir)
    north = z[cap] > 0
    out[cap] = np.where(north, 2 * ir * (ir - 1) + ip, 12 * nside * nside - 2 * ir * (ir + 1) + ip)
    return out


def pixel_ring(nside: int, pix):
    """Ring index (0-based) of each pixel."""
    _, _, _, start = ring_geometry(nside)
    return np.searchsorted(start, np.asarray(pix, dtype=np.int64), side="right") - 1


# ------------------------------------------------------ ring synthesis ----

def ring_values(F, k: int, phis) -> np.ndarray:
    """sum_{m=-L}^{L} (i m)^k F_m e^{i m phi} (F_{-m} = conj F_m, Re F_0 only)
    at the given phi (direct sum)."""
    return tor.phi_eval(np.asarray(F), k, phis)


def derivative_pixels(lmax, order, nside, pix, alm_T, alm_E=None, alm_B=None, nthreads=0):
    """d^j_theta d^k_phi s at the centres of the given pixels:
    {field: {(j, k): [len(pix)]}}."""
    theta, nphi, phi0, start = ring_geometry(nside)
    pix = np.asarray(pix, dtype=np.int64)
    rings = pixel_ring(nside, pix)
    ur = np.unique(rings)
    F = tor.ring_coeffs(lmax, order, theta[ur], alm_T, alm_E, alm_B, nthreads)
    _, ph = pix2ang(nside, pix)
    out = {f: {jk: np.empty(pix.size) for jk in tor.jk_pairs(order)} for f in F}
    for q, r in enumerate(ur):
        sel = rings == r
        for f, arr in F.items():
            for (j, k) in tor.jk_pairs(order):
                out[f][(j, k)][sel] = ring_values(arr[q, j, :], k, ph[sel])
    return out


def deflection_pixels(lmax, alm_phi, nside, pix, nthreads=0):
    """alpha_theta = d_theta phi and alpha_phi = d_phi phi / sin theta at the
    given pixel centres (HEALPix has no pixel at a pole)."""
    theta, _, _, _ = ring_geometry(nside)
    D = derivative_pixels(lmax, 1, nside, pix, alm_phi, nthreads=nthreads)["T"]
    th = theta[pixel_ring(nside, pix)]
    return D[(1, 0)], D[(0, 1)] / np.sin(th)


# ------------------------------------------------------------- lensing ----

def lens_pixels(lmax, order, nside, pix, alm_T, alm_E=None, alm_B=None, alm_phi=None, rotate=True,
                naive=False, nthreads=0) -> dict:
    """Lensed T (and Q, U) at the given output pixels of a HEALPix map:
    positions x' = x + alpha (geodesic, or the naive rule), the pixel p'
    containing x', its centre x0', the offsets dth = theta' - theta0',
    dph = phi' - phi0' (wrapped to (-pi, pi]), the order-N sum of eq. 5 with
    the derivatives at x0', then the rotation R."""
    pix = np.asarray(pix, dtype=np.int64)
    th, ph = pix2ang(nside, pix)
    if alm_phi is None:
        a_t = np.zeros(pix.size)
        a_p = np.zeros(pix.size)
    else:
        a_t, a_p = deflection_pixels(lmax, alm_phi, nside, pix, nthreads)
    if naive:
        thp, php = tor.naive_positions(th, ph, a_t, a_p)
        xp = tor.unit_vectors(thp, php)[0]
        dist = np.hypot(a_t, a_p)
    else:
        thp, php, xp, dist, _ = tor.geodesic_positions(th, ph, a_t, a_p)
    src = ang2pix(nside, thp, php)
    th0, ph0 = pix2ang(nside, src)
    dth = thp - th0
    dph = np.angle(np.exp(1j * (php - ph0)))
    usrc, inv = np.unique(src, return_inverse=True)
    D = derivative_pixels(lmax, order, nside, usrc, alm_T, alm_E, alm_B, nthreads)
    res = {}
    for f, Df in D.items():
        res[f] = tor.taylor_sum(lambda j, k: Df[(j, k)][inv], dth, dph, order)
    if "Q" in res and rotate and not naive:
        Qr, Ur = tor.rotate_pol_3d(res["Q"], res["U"], th, ph, thp, php, xp)
        res["Q"] = np.where(dist > 0, Qr, res["Q"])
        res["U"] = np.where(dist > 0, Ur, res["U"])
    res["_src"] = src
    res["_dth"] = dth
    res["_dph"] = dph
    res["_thp"] = thp
    res["_php"] = php
    res["_alpha_theta"] = a_t
    res["_alpha_phi"] = a_p
    return res


def lens_map(lmax, order, nside, alm_T, alm_E=None, alm_B=None, alm_phi=None, rotate=True, naive=False,
             nthreads=0) -> dict:
    """Whole lensed HEALPix maps ([npix] per field, RING order)."""
    return lens_pixels(lmax, order, nside, np.arange(npix(nside)), alm_T, alm_E, alm_B, alm_phi, rotate,
                       naive, nthreads)


def ring_pixels(nside: int, rings) -> np.ndarray:
    """All pixel indices of the given rings (0-based ring indices)."""
    _, nphi, _, start = ring_geometry(nside)
    return np.concatenate([np.arange(start[r], start[r] + nphi[r]) for r in np.atleast_1d(rings)])
