"""Pins of the oracle's harmonic part against mathematics it does not use.

Scalar functions: scipy's sph_harm_y, the addition theorem, Gauss-Legendre
orthonormality, finite differences, the associated Legendre ODE.
Spin-2 functions: the eth definition applied to the scalar functions,
Goldberg's explicit sum (mpmath), the spin addition theorem, orthonormality,
the spin-weighted ODE and the pole values.
"""
import math

import numpy as np
import pytest

from tests import pinlib


THETAS = [0.0, 1e-3, 0.31, 1.2, math.pi / 2, 2.2, 3.0, math.pi - 1e-3, math.pi]


@pytest.mark.parametrize("m", [0, 1, 2, 5, 17, 40, 64])
def test_scalar_lambda_matches_scipy(oracle, m):
    lmax = 64
    for th in THETAS:
        lam = oracle.spin_lambda(lmax, 0, 0, m, th)[:, 0]
        ref = np.array([pinlib.scalar_lambda(l, m, th) if l >= m else 0.0 for l in range(lmax + 1)])
        scale = max(1.0, np.max(np.abs(ref)))
        assert np.max(np.abs(lam - ref)) <= 1e-13 * scale, (m, th)


@pytest.mark.parametrize("theta", [math.pi / 4096, 0.05, 0.7, math.pi / 2])
def test_addition_theorem_to_l4096(oracle, theta):
    """sum_m |Y_lm|^2 = (2l+1)/(4 pi) for every l <= 4096 (this exercises the
    range of sin^m theta, which underflows double for large m)."""
    lmax = 4096
    acc = np.zeros(lmax + 1)
    for m in range(lmax + 1):
        lam = oracle.spin_lambda(lmax, 0, 0, m, theta)[:, 0]
        acc += (1.0 if m == 0 else 2.0) * lam * lam
    l = np.arange(lmax + 1)
    np.testing.assert_allclose(acc, (2 * l + 1) / (4 * math.pi), rtol=1e-12, atol=0)


@pytest.mark.parametrize("theta", [math.pi / 2048, 0.4, 1.9])
def test_spin2_addition_theorem(oracle, theta):
    """sum_{m=-l}^{l} |2Y_lm|^2 = (2l+1)/(4 pi), using 2lambda_{l,-m} =
    (-1)^m (-2)lambda_lm."""
    lmax = 1024
    acc = np.zeros(lmax + 1)
    for m in range(lmax + 1):
        p = oracle.spin_lambda(lmax, 0, 2, m, theta)[:, 0]
        acc += p * p
        if m > 0:
            q = oracle.spin_lambda(lmax, 0, -2, m, theta)[:, 0]
            acc += q * q
    l = np.arange(2, lmax + 1)
    np.testing.assert_allclose(acc[2:], (2 * l + 1) / (4 * math.pi), rtol=1e-12, atol=0)


@pytest.mark.parametrize("s,m", [(0, 0), (0, 3), (0, 200), (2, 0), (2, 1), (2, 7), (-2, 1), (-2, 150)])
def test_orthonormality_gauss_legendre(oracle, s, m):
    """2 pi int s_lambda_lm s_lambda_l'm sin t dt = delta_ll' (exact quadrature:
    the product is a polynomial in cos t of degree l + l')."""
    lmax = 512
    x, w = np.polynomial.legendre.leggauss(lmax + 2)
    th = np.arccos(x)
    lmin = max(abs(s), m)
    V = np.stack([oracle.spin_lambda(lmax, 0, s, m, t)[:, 0] for t in th])  # [node, l]
    G = 2 * math.pi * (V.T * w) @ V
    G = G[lmin:, lmin:]
    # 514-term double sums of weights x products up to ~(2l+1)/(4 pi): ~1e-12 rounding
    np.testing.assert_allclose(G, np.eye(G.shape[0]), atol=1e-11)


def _richardson(f, t, order, h):
    """Central-difference estimate of the order-th derivative, Richardson
    extrapolated once (error O(h^4))."""
    from math import comb

    def cd(hh):
        acc = 0.0
        for i in range(order + 1):
            acc += (-1) ** i * comb(order, i) * f(t + (order / 2 - i) * hh)
        return acc / hh ** order

    return (4 * cd(h / 2) - cd(h)) / 3


@pytest.mark.parametrize("s", [0, 2, -2])
@pytest.mark.parametrize("m", [0, 1, 4, 11])
def test_theta_derivatives_finite_difference(oracle, s, m):
    lmax = 24
    J = 4
    for t in [0.4, 1.3, 2.6]:
        ana = oracle.spin_lambda(lmax, J, s, m, t)
        for l in range(max(abs(s), m), lmax + 1):
            f = lambda tt: oracle.spin_lambda(lmax, 0, s, m, tt)[l, 0]
            for j in range(1, J + 1):
                h = {1: 1e-3, 2: 2e-3, 3: 5e-3, 4: 1e-2}[j]
                fd = _richardson(f, t, j, h)
                fmax = max(1e-3, np.max(np.abs(ana[:, 0])))
                # truncation O(h^4 l^(j+4)) (a wrong formula is off by O(l^j)), plus the
                # difference quotient rounding floor eps |f| (2/h)^j
                scale = (l + 1) ** j * fmax
                tol = scale * (1e-6 + 0.1 * (h * (l + 1)) ** 4) + 100 * 2.2e-16 * fmax * (2 / h) ** j
                assert abs(fd - ana[l, j]) <= tol, (s, m, l, j, t, fd, ana[l, j])


@pytest.mark.parametrize("s", [0, 2, -2])
def test_spin_weighted_ode_residual(oracle, s):
    """lam'' + cot t lam' + [l(l+1) - (m^2 + s^2 + 2 m s cos t)/sin^2 t] lam = 0,
    and its derivatives (checked through order 4 via the recursion's own
    higher derivatives differentiated once more)."""
    lmax = 200
    for m in [0, 1, 2, 9, 60]:
        for t in [0.2, 1.0, 2.0, 2.9]:
            d = oracle.spin_lambda(lmax, 2, s, m, t)
            l = np.arange(lmax + 1)
            ct, st = math.cos(t), math.sin(t)
            res = d[:, 2] + ct / st * d[:, 1] + (l * (l + 1) - (m * m + s * s + 2 * m * s * ct) / st ** 2) * d[:, 0]
            scale = np.max(np.abs(l * (l + 1) * d[:, 0])) + 1e-300
            lmin = max(abs(s), m)
            assert np.max(np.abs(res[lmin:])) <= 1e-11 * scale, (s, m, t)


@pytest.mark.parametrize("m", [0, 1, 2, 3, 8, 30])
def test_spin2_eth_definition(oracle, m):
    """+-2 lambda = sqrt((l-2)!/(l+2)!) [lam'' - cot lam' + m^2 csc^2 lam
    -+ 2 m csc (lam' - cot lam)] from the scalar lambda (interior theta)."""
    lmax = 60
    for t in [0.15, 0.9, 1.7, 2.8]:
        lam = oracle.spin_lambda(lmax, 2, 0, m, t)
        sp = oracle.spin_lambda(lmax, 0, 2, m, t)[:, 0]
        sm = oracle.spin_lambda(lmax, 0, -2, m, t)[:, 0]
        ct, cs = 1 / math.tan(t), 1 / math.sin(t)
        for l in range(max(2, m), lmax + 1):
            N = math.exp(0.5 * (math.lgamma(l - 1) - math.lgamma(l + 3)))
            base = lam[l, 2] - ct * lam[l, 1] + m * m * cs * cs * lam[l, 0]
            eth = 2 * m * cs * (lam[l, 1] - ct * lam[l, 0])
            sc = 1e-13 * (1 + abs(N * base))
            assert abs(N * (base - eth) - sp[l]) <= sc, (l, t)
            assert abs(N * (base + eth) - sm[l]) <= sc, (l, t)


@pytest.mark.parametrize("s", [2, -2])
def test_spin2_goldberg_closed_form(oracle, s):
    lmax = 14
    for m in range(0, lmax + 1):
        for t in [0.05, 0.8, 1.9, 3.1]:
            lam = oracle.spin_lambda(lmax, 0, s, m, t)[:, 0]
            for l in range(max(2, m), lmax + 1):
                ref = pinlib.goldberg_mp(s, l, m, t)
                assert abs(lam[l] - ref) <= 1e-14, (s, l, m, t)


def test_spin2_pole_values(oracle):
    """At theta = 0 only s = -2, m = 2 survives among m >= 0 (i.e. 2Y_{l,-2});
    at theta = pi only s = +2, m = 2 survives."""
    lmax = 40
    k = np.arange(lmax + 1)
    for m in range(0, 8):
        p0 = oracle.spin_lambda(lmax, 0, 2, m, 0.0)[:, 0]
        m0 = oracle.spin_lambda(lmax, 0, -2, m, 0.0)[:, 0]
        pp = oracle.spin_lambda(lmax, 0, 2, m, math.pi)[:, 0]
        mp_ = oracle.spin_lambda(lmax, 0, -2, m, math.pi)[:, 0]
        assert np.all(p0 == 0.0) and np.max(np.abs(mp_)) < 1e-14
        if m == 2:
            # -2 lambda_l2(0) = sqrt((2l+1)/(4 pi)) for l >= 2 (Wigner d^l_22(0) = 1)
            ref = np.where(k >= 2, np.sqrt((2 * k + 1) / (4 * math.pi)), 0.0)
            np.testing.assert_allclose(m0, ref, rtol=1e-14, atol=1e-15)
            np.testing.assert_allclose(np.abs(pp), ref, rtol=1e-13, atol=1e-15)
        else:
            assert np.max(np.abs(m0)) < 1e-15
            assert np.max(np.abs(pp)) < 1e-14


def test_ring_coeffs_match_direct_sums(oracle):
    """oracle_synth_rings == explicit sums over the pinned functions, for T
    and for the Q/U assembly from E and B (both non-zero)."""
    from paper_1307_0719_amd import skygen

    lmax, J = 20, 3
    aT = skygen.random_alm(lmax, 11)
    aE = skygen.random_alm(lmax, 12, lmin=2)
    aB = skygen.random_alm(lmax, 13, lmin=2)
    th = [0.0, 0.37, 1.4, math.pi]
    F = oracle.ring_coeffs(lmax, J, th, aT, aE, aB)
    for r, t in enumerate(th):
        for m in range(lmax + 1):
            lam = oracle.spin_lambda(lmax, J, 0, m, t)
            sp = oracle.spin_lambda(lmax, J, 2, m, t)
            sm = oracle.spin_lambda(lmax, J, -2, m, t)
            idx = [m * (2 * lmax + 1 - m) // 2 + l for l in range(lmax + 1)]
            ls = np.arange(lmax + 1)
            mask = ls >= m
            a = np.where(mask, aT[np.where(mask, idx, 0)], 0)
            e = np.where(mask & (ls >= 2), aE[np.where(mask, idx, 0)], 0)
            b = np.where(mask & (ls >= 2), aB[np.where(mask, idx, 0)], 0)
            for j in range(J + 1):
                np.testing.assert_allclose(F["T"][r, j, m], np.sum(a * lam[:, j]), atol=1e-12)
                P = -np.sum((e + 1j * b) * sp[:, j])
                M = -np.sum((e - 1j * b) * sm[:, j])
                np.testing.assert_allclose(F["Q"][r, j, m], (P + M) / 2, atol=1e-12)
                np.testing.assert_allclose(F["U"][r, j, m], (P - M) / 2j, atol=1e-12)


def test_phi_synthesis_fft_equals_direct_sum(oracle):
    rng = np.random.default_rng(5)
    L, nphi = 16, 32  # nphi = 2 L: the Nyquist term is present
    F = rng.standard_normal(L + 1) + 1j * rng.standard_normal(L + 1)
    phis = 2 * math.pi * np.arange(nphi) / nphi
    for k in range(5):
        a = oracle.phi_synth(F, k, nphi)
        b = oracle.phi_eval(F, k, phis)
        np.testing.assert_allclose(a, b, atol=1e-11 * (L ** k + 1))
    # the k-th phi-derivative of the direct sum equals finite differences
    f = lambda p: oracle.phi_eval(F, 0, np.array([p]))[0]
    for k in range(1, 4):
        fd = _richardson(f, 0.77, k, 1e-2)
        assert abs(fd - oracle.phi_eval(F, k, np.array([0.77]))[0]) < 1e-6 * L ** k * np.sum(np.abs(F))
