"""Pins of the HEALPix oracle (geometry and lensing on HEALPix rings) against
results fixed by the published pixelization and by mathematics it does not
use:

H1  the twelve base pixels of nside = 1 (Gorski et al. 2005: three rings at
    z = 2/3, 0, -2/3; the polar ones centred on phi = pi/4 + k pi/2, the
    equatorial ones on phi = k pi/2);
H2  pix2ang then ang2pix returns every pixel, for several nside;
H3  equal area: uniform random directions fall into every pixel with the
    same probability (chi-square over 192 and 768 pixels);
H4  locality: every direction lies within the largest pixel radius of the
    centre of the pixel ang2pix gives;
H5  zero deflection: the lensed map at the pixel centres equals the brute
    force sum a_lm Y_lm there (scipy; spin 2 by Goldberg's sum), with polar
    rings of 4..12 pixels far below the band limit (the phi synthesis folds
    m into them);
H6  convergence: order by order the HEALPix Taylor result approaches the
    brute-force field at the displaced positions.
"""
import math

import numpy as np
import pytest

from oracle import healpix_oracle as hp
from paper_1307_0719_amd import skygen
from tests import pinlib


def test_h1_base_pixels():
    th, ph = hp.pix2ang(1, np.arange(12))
    z = np.cos(th)
    np.testing.assert_allclose(z, [2 / 3] * 4 + [0.0] * 4 + [-2 / 3] * 4, atol=1e-15)
    np.testing.assert_allclose(ph, [(k + 0.5) * math.pi / 2 for k in range(4)] + [k * math.pi / 2 for k in range(4)]
                               + [(k + 0.5) * math.pi / 2 for k in range(4)], atol=1e-15)
    assert np.array_equal(hp.ang2pix(1, th, ph), np.arange(12))


@pytest.mark.parametrize("nside", [1, 2, 3, 4, 7, 16, 64, 256])
def test_h2_round_trip_and_ring_structure(nside):
    p = np.arange(hp.npix(nside))
    th, ph = hp.pix2ang(nside, p)
    assert np.array_equal(hp.ang2pix(nside, th, ph), p)
    theta, nphi, phi0, start = hp.ring_geometry(nside)
    assert nphi.sum() == 12 * nside * nside
    # equal pixel counts by ring pair: the sphere is symmetric under z -> -z
    np.testing.assert_allclose(theta + theta[::-1], math.pi, atol=1e-14)
    assert np.array_equal(nphi, nphi[::-1])
    # ring z from the published closed forms
    i = np.arange(1, 4 * nside)
    ii = np.minimum(i, 4 * nside - i)
    zcap = 1 - ii ** 2 / (3.0 * nside ** 2)
    zbelt = 4.0 / 3.0 - 2.0 * i / (3.0 * nside)
    want = np.where(ii < nside, np.sign(2 * nside - i) * zcap, zbelt)
    np.testing.assert_allclose(np.cos(theta), want, atol=1e-14)


@pytest.mark.parametrize("nside", [4, 8])
def test_h3_equal_area(nside):
    rng = np.random.default_rng(7 + nside)
    n = 3_000_000
    z = rng.uniform(-1, 1, n)
    phi = rng.uniform(0, 2 * math.pi, n)
    counts = np.bincount(hp.ang2pix(nside, np.arccos(z), phi), minlength=hp.npix(nside))
    mean = n / hp.npix(nside)
    chi2 = np.sum((counts - mean) ** 2 / mean)
    dof = hp.npix(nside) - 1
    # chi-square of equal-probability cells: mean dof, sd sqrt(2 dof)
    assert abs(chi2 - dof) < 6 * math.sqrt(2 * dof), (chi2, dof)
    assert np.all(np.abs(counts - mean) < 6 * math.sqrt(mean))


@pytest.mark.parametrize("nside", [2, 16, 128])
def test_h4_locality(nside):
    rng = np.random.default_rng(11)
    n = 400_000
    z = rng.uniform(-1, 1, n)
    phi = rng.uniform(0, 2 * math.pi, n)
    th = np.arccos(z)
    p = hp.ang2pix(nside, th, phi)
    tc, pc = hp.pix2ang(nside, p)
    cosd = np.cos(th) * np.cos(tc) + np.sin(th) * np.sin(tc) * np.cos(phi - pc)
    d = np.arccos(np.clip(cosd, -1, 1))
    # every HEALPix pixel fits inside a circle of about 1.4 x the mean
    # pixel spacing sqrt(4 pi / npix) around its centre (the diamonds next
    # to the poles are the most elongated)
    spacing = math.sqrt(4 * math.pi / hp.npix(nside))
    assert np.max(d) < 1.5 * spacing, np.max(d) / spacing
    # and a direction close to a centre belongs to that centre's pixel
    q = rng.integers(0, hp.npix(nside), 2000)
    tq, pq = hp.pix2ang(nside, q)
    eps = 1e-3 * spacing
    t2 = np.clip(tq + eps * rng.uniform(-1, 1, q.size), 0, math.pi)
    p2 = pq + eps * rng.uniform(-1, 1, q.size) / np.maximum(np.sin(tq), 1e-3)
    assert np.array_equal(hp.ang2pix(nside, t2, p2), q)


def test_h5_zero_deflection_is_the_field_at_the_centres():
    lmax, nside = 16, 4          # ring 1 has 4 pixels, far below the band limit
    sky = skygen.make_sky(lmax, 3, pol=True)
    almB = skygen.random_alm(lmax, 4, lmin=2) * 0.3
    res = hp.lens_map(lmax, 3, nside, sky.alm_T, sky.alm_E, almB, None)
    th, ph = hp.pix2ang(nside, np.arange(hp.npix(nside)))
    T = pinlib.brute_T(sky.alm_T, lmax, th, ph)
    Q, U = pinlib.brute_QU(sky.alm_E, almB, lmax, th, ph)
    for got, want in ((res["T"], T), (res["Q"], Q), (res["U"], U)):
        np.testing.assert_allclose(got, want, atol=1e-12 * np.max(np.abs(want)))


def _sup_T(alm, lmax):
    """sup |T| <= sum_l sqrt((2l+1)/(4 pi) sum_{|m|<=l} |a_lm|^2) (addition theorem)."""
    return sum(math.sqrt((2 * l + 1) / (4 * math.pi) * sum(abs(pinlib.alm_get(alm, lmax, l, m)) ** 2
                                                           for m in range(-l, l + 1)))
               for l in range(lmax + 1))


def _sup_P(almE, almB, lmax):
    return sum(math.sqrt((2 * l + 1) / (4 * math.pi) * sum(abs(pinlib.alm_get(almE, lmax, l, m)
                                                               + 1j * pinlib.alm_get(almB, lmax, l, m)) ** 2
                                                           for m in range(-l, l + 1)))
               for l in range(2, lmax + 1))


def test_h6_order_by_order_convergence_to_the_displaced_field():
    """Every pixel's error stays within the Bernstein bound of a band-limited
    field, sup |f| * sum_{n > N} sigma^n / n!, sigma = lmax (|dth| + |dph|)
    (each coordinate derivative of a degree-lmax trigonometric polynomial is
    at most lmax times its sup), and the worst error falls order by order."""
    lmax, nside = 12, 16
    pix = np.arange(hp.npix(nside))
    spacing = math.sqrt(4 * math.pi / hp.npix(nside))
    sky = skygen.make_sky(lmax, 5, pol=True, rms_arcmin=1.5 * spacing / skygen.ARCMIN)
    almB = skygen.random_alm(lmax, 6, lmin=2) * 0.3
    sups = {"T": _sup_T(sky.alm_T, lmax)}
    sups["Q"] = sups["U"] = _sup_P(sky.alm_E, almB, lmax)
    exact = None
    errs = []
    for N in (0, 2, 4, 6, 8, 10, 12, 14):
        res = hp.lens_pixels(lmax, N, nside, pix, sky.alm_T, sky.alm_E, almB, sky.alm_phi, rotate=False)
        if exact is None:
            thp, php = res["_thp"], res["_php"]
            # the deflection must move many pixels into another pixel
            assert np.mean(res["_src"] != pix) > 0.5
            exact = {"T": pinlib.brute_T(sky.alm_T, lmax, thp, php)}
            exact["Q"], exact["U"] = pinlib.brute_QU(sky.alm_E, almB, lmax, thp, php)
        sigma = lmax * (np.abs(res["_dth"]) + np.abs(res["_dph"]))
        tail = np.exp(sigma) - sum(sigma ** n / math.factorial(n) for n in range(N + 1))
        for f in "TQU":
            err = np.abs(res[f] - exact[f])
            assert np.all(err <= sups[f] * tail + 1e-12 * sups[f]), (f, N)
        errs.append(max(np.max(np.abs(res[f] - exact[f])) / sups[f] for f in "TQU"))
    errs = np.array(errs)
    print("HEALPix Taylor error by order (over the sup bound)", errs)
    assert np.all(np.diff(errs) < 0)
    assert errs[-1] < 1e-7
