"""Independent reference values for pinning the oracle (tests only).

Nothing here calls the oracle: scalar harmonics come from scipy's
``sph_harm_y`` (a library routine), spin-weighted harmonics from Goldberg's
explicit finite sum (mpmath at high precision, or float64 for small l).
"""
from __future__ import annotations

import math

import mpmath as mp
import numpy as np
from scipy.special import sph_harm_y


def scalar_lambda(l, m, theta):
    """lambda_lm(theta) = Y_lm(theta, 0) (orthonormal, Condon-Shortley)."""
    return np.real(sph_harm_y(l, m, np.asarray(theta, float), 0.0))


def goldberg_mp(s, l, m, theta, dps=40):
    """s_lambda_lm(theta) by Goldberg's explicit sum, mpmath (theta in (0, pi))."""
    with mp.workdps(dps):
        th = mp.mpf(theta)
        pref = (-1) ** m * mp.sqrt(mp.factorial(l + m) * mp.factorial(l - m) * (2 * l + 1)
                                   / (4 * mp.pi * mp.factorial(l + s) * mp.factorial(l - s)))
        tot = mp.mpf(0)
        for r in range(0, l - s + 1):
            q = r + s - m
            if q < 0 or q > l + s:
                continue
            k = 2 * r + s - m
            tot += (mp.binomial(l - s, r) * mp.binomial(l + s, q) * (-1) ** (l - r - s)
                    * mp.sin(th / 2) ** (2 * l - k) * mp.cos(th / 2) ** k)
        return float(pref * tot)


def goldberg_np(s, l, m, theta):
    """Goldberg's sum in float64, vectorized over theta (valid for small l).
    Works for negative m as well."""
    th = np.asarray(theta, float)
    sh, ch = np.sin(th / 2), np.cos(th / 2)
    pref = (-1) ** (m % 2) * math.sqrt(math.factorial(l + m) * math.factorial(l - m) * (2 * l + 1)
                                      / (4 * math.pi * math.factorial(l + s) * math.factorial(l - s)))
    tot = np.zeros_like(th)
    for r in range(0, l - s + 1):
        q = r + s - m
        if q < 0 or q > l + s:
            continue
        k = 2 * r + s - m
        tot = tot + (math.comb(l - s, r) * math.comb(l + s, q) * (-1) ** ((l - r - s) % 2)
                     * sh ** (2 * l - k) * ch ** k)
    return pref * tot


def alm_get(alm, lmax, l, m):
    """a_lm for any integer m (real-field symmetry for m < 0)."""
    if m >= 0:
        return alm[m * (2 * lmax + 1 - m) // 2 + l]
    mm = -m
    return (-1) ** (mm % 2) * np.conj(alm[mm * (2 * lmax + 1 - mm) // 2 + l])


def brute_T(alm, lmax, theta, phi):
    """sum_lm a_lm Y_lm(theta, phi) by direct evaluation (real field)."""
    theta = np.asarray(theta, float)
    phi = np.asarray(phi, float)
    out = np.zeros(np.broadcast(theta, phi).shape)
    for m in range(lmax + 1):
        w = 1.0 if m == 0 else 2.0
        acc = np.zeros(out.shape, np.complex128)
        for l in range(m, lmax + 1):
            a = alm[m * (2 * lmax + 1 - m) // 2 + l]
            if a == 0:
                continue
            acc = acc + a * scalar_lambda(l, m, theta)
        out = out + w * np.real(acc * np.exp(1j * m * phi))
    return out


def brute_QU(almE, almB, lmax, theta, phi):
    """Q + iU = sum_{l>=2, |m|<=l} 2a_lm 2Y_lm, 2a_lm = -(E_lm + i B_lm), by
    Goldberg's sum over every m (negative m via the real-field symmetry)."""
    theta = np.asarray(theta, float)
    phi = np.asarray(phi, float)
    P = np.zeros(np.broadcast(theta, phi).shape, np.complex128)
    for l in range(2, lmax + 1):
        for m in range(-l, l + 1):
            E = alm_get(almE, lmax, l, m)
            B = alm_get(almB, lmax, l, m) if almB is not None else 0.0
            a2 = -(E + 1j * B)
            if a2 == 0:
                continue
            P = P + a2 * goldberg_np(2, l, m, theta) * np.exp(1j * m * phi)
    return np.real(P), np.imag(P)
