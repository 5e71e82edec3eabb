"""Pins of the oracle's lensing pipeline (remap, Taylor sum, rotation,
positions) against results fixed by mathematics it does not use:

P1  brute-force sum a_lm Y_lm(x') (scipy / Goldberg), error within the
    Bernstein bound of a band-limited function, for N = 0..14;
P2  a constant azimuthal shift, whose exact order-N result is a phase factor
    E_N(i m r) per m;
P3  a constant theta shift, exact via the doubled-circle Fourier series;
P4  alpha = 0 gives back the unlensed map bit for bit;
P8  the rotation equals the closed-form angle 2 gamma, is unitary, and obeys
    the pole-ring invariants;
P9  the positions lie at great-circle distance |alpha| in direction psi;
P10 the exact lensed field (no Taylor series) is the brute-force sum at the
    displaced positions and the limit of the Taylor remap.
"""
import math

import numpy as np
import pytest

from paper_1307_0719_amd import skygen
from tests import pinlib


def _sup_bound_T(alm, lmax):
    """sup |T| <= sum_l sqrt((2l+1)/(4 pi) sum_{|m|<=l} |a_lm|^2)."""
    tot = 0.0
    for l in range(lmax + 1):
        s = 0.0
        for m in range(0, l + 1):
            a = alm[m * (2 * lmax + 1 - m) // 2 + l]
            s += (1.0 if m == 0 else 2.0) * abs(a) ** 2
        tot += math.sqrt((2 * l + 1) / (4 * math.pi) * s)
    return tot


def _sup_bound_P(almE, almB, lmax):
    tot = 0.0
    for l in range(2, lmax + 1):
        s = 0.0
        for m in range(-l, l + 1):
            e = pinlib.alm_get(almE, lmax, l, m)
            b = pinlib.alm_get(almB, lmax, l, m)
            s += abs(e + 1j * b) ** 2
        tot += math.sqrt((2 * l + 1) / (4 * math.pi) * s)
    return tot


@pytest.fixture(scope="module")
def small_sky():
    lmax = 16
    ntheta, nphi = 4 * lmax + 1, 8 * lmax
    # deflection of ~2 pixels RMS so that the nearest pixel really moves
    pix_arcmin = (math.pi / (ntheta - 1)) / skygen.ARCMIN
    sky = skygen.make_sky(lmax, 101, pol=True, rms_arcmin=2.0 * pix_arcmin)
    almB = skygen.random_alm(lmax, 102, lmin=2) * 0.3
    return lmax, ntheta, nphi, sky, almB


def test_p1_brute_force_convergence(oracle, small_sky):
    lmax, ntheta, nphi, sky, almB = small_sky
    supT = _sup_bound_T(sky.alm_T, lmax)
    supP = _sup_bound_P(sky.alm_E, almB, lmax)
    exact = None
    errs = []
    for N in range(0, 15):
        res = oracle.lens_map(lmax, N, ntheta, nphi, sky.alm_T, sky.alm_E, almB, sky.alm_phi,
                              rotate=False)
        if exact is None:
            thp, php = res["_thp"], res["_php"]
            # the deflection must move most pixels off their own centre
            moved = np.mean(res["_i0"] != np.arange(ntheta)[:, None])
            assert moved > 0.5
            exact = {"T": pinlib.brute_T(sky.alm_T, lmax, thp, php)}
            exact["Q"], exact["U"] = pinlib.brute_QU(sky.alm_E, almB, lmax, thp, php)
        sigma = lmax * (np.abs(res["_dth"]) + np.abs(res["_dph"]))
        assert np.max(sigma) <= math.pi / 4 + 1e-12
        tail = sigma ** (N + 1) / math.factorial(N + 1)
        e = {}
        for f, sup in (("T", supT), ("Q", supP), ("U", supP)):
            err = np.abs(res[f] - exact[f])
            assert np.all(err <= sup * tail + 1e-13 * sup), (f, N)
            e[f] = np.max(err) / sup
        errs.append(max(e.values()))
    errs = np.array(errs)
    # the series converges: decreasing (to rounding level) and ~1e-13 by N = 14
    assert errs[14] < 1e-13
    assert np.all(np.diff(np.maximum(errs, 1e-14)) <= 1e-15)


@pytest.mark.parametrize("N", [0, 1, 2, 3, 5, 8])
def test_p2_constant_azimuthal_shift(oracle, N):
    lmax = 48
    ntheta, nphi = 2 * lmax + 1, 2 * lmax  # nphi = 2 lmax: Nyquist bin present
    aT = skygen.random_alm(lmax, 7)
    th = oracle.grid_theta(ntheta)
    ph = oracle.grid_phi(nphi)
    dphi = 2 * math.pi / nphi
    c = 2.37 * dphi
    q = math.floor(c / dphi + 0.5)
    r = c - q * dphi
    TH = th[:, None] * np.ones((1, nphi))
    PHp = ph[None, :] + c + 0 * TH
    res = oracle.lens_at_positions(lmax, N, ntheta, nphi, TH, PHp, aT)
    assert np.min(res["_tie"]) > 1e-6
    # exact: sum_m w_m Re[F_m(theta_i) e^{i m (phi_k + q dphi)} E_N(i m r)]
    m = np.arange(lmax + 1)
    EN = sum((1j * m * r) ** n / math.factorial(n) for n in range(N + 1))
    Fm = np.zeros((ntheta, lmax + 1), np.complex128)
    for mm in range(lmax + 1):
        for l in range(mm, lmax + 1):
            Fm[:, mm] += aT[mm * (2 * lmax + 1 - mm) // 2 + l] * pinlib.scalar_lambda(l, mm, th)
    w = np.where(m == 0, 1.0, 2.0)
    ex = np.real((w * Fm * EN)[:, None, :] * np.exp(1j * np.multiply.outer(ph + q * dphi, m))[None]).sum(-1)
    scale = np.max(np.abs(ex))
    np.testing.assert_allclose(res["T"], ex, atol=2e-13 * scale)


@pytest.mark.parametrize("N", [1, 2, 4, 7])
def test_p3_constant_theta_shift(oracle, N):
    lmax = 32
    ntheta, nphi = lmax + 3, 2 * lmax + 2
    aT = skygen.random_alm(lmax, 9)
    th = oracle.grid_theta(ntheta)
    ph = oracle.grid_phi(nphi)
    dth = math.pi / (ntheta - 1)
    c = 0.41 * dth
    rings = np.arange(1, ntheta - 1)  # interior rings (theta + c stays inside)
    TH = th[rings][:, None] + c + 0 * ph[None, :]
    PH = ph[None, :] + 0 * TH
    res = oracle.lens_at_positions(lmax, N, ntheta, nphi, TH, PH, aT)
    # F_m on the doubled circle: F_m(2 pi - t) = (-1)^m F_m(t); trig polynomial
    # of degree <= lmax in t, sampled at 2(ntheta-1) > 2 lmax points.
    nd = 2 * (ntheta - 1)
    m = np.arange(lmax + 1)
    Fm = np.zeros((ntheta, lmax + 1), np.complex128)
    for mm in range(lmax + 1):
        for l in range(mm, lmax + 1):
            Fm[:, mm] += aT[mm * (2 * lmax + 1 - mm) // 2 + l] * pinlib.scalar_lambda(l, mm, th)
    dbl = np.zeros((nd, lmax + 1), np.complex128)
    dbl[:ntheta] = Fm
    for qq in range(ntheta, nd):
        dbl[qq] = (-1.0) ** m * Fm[nd - qq]
    cq = np.fft.fft(dbl, axis=0) / nd
    p = np.fft.fftfreq(nd, d=1.0 / nd)
    assert np.max(np.abs(cq[np.abs(p) > lmax])) < 1e-12 * np.max(np.abs(cq))
    EN = sum((1j * p * c) ** n / math.factorial(n) for n in range(N + 1))
    Ft = (cq[None, :, :] * (np.exp(1j * np.multiply.outer(th[rings], p)) * EN)[:, :, None]).sum(1)
    w = np.where(m == 0, 1.0, 2.0)
    ex = np.real((w * Ft)[:, None, :] * np.exp(1j * np.multiply.outer(ph, m))[None]).sum(-1)
    scale = np.max(np.abs(ex))
    np.testing.assert_allclose(res["T"], ex, atol=1e-12 * scale)


def test_p4_zero_deflection_is_identity(oracle):
    lmax = 24
    ntheta, nphi = 2 * lmax + 1, 2 * lmax + 4
    sky = skygen.make_sky(lmax, 3)
    zero = np.zeros_like(sky.alm_phi)
    for N in (0, 3):
        res = oracle.lens_map(lmax, N, ntheta, nphi, sky.alm_T, sky.alm_E, sky.alm_B, zero)
        un = oracle.unlensed_map(lmax, ntheta, nphi, sky.alm_T, sky.alm_E, sky.alm_B)
        for f in ("T", "Q", "U"):
            assert np.array_equal(res[f], un[f]), f


def _closed_form_rotation(Q, U, theta, phi, a_t, a_p):
    x, et, ep = [np.asarray(v) for v in _uv(theta, phi)]
    d = np.hypot(a_t, a_p)
    u = (a_t[..., None] * et + a_p[..., None] * ep) / d[..., None]
    xp = np.cos(d)[..., None] * x + np.sin(d)[..., None] * u
    tp = -np.sin(d)[..., None] * x + np.cos(d)[..., None] * u
    thp = np.arctan2(np.hypot(xp[..., 0], xp[..., 1]), xp[..., 2])
    php = np.arctan2(xp[..., 1], xp[..., 0])
    _, etp, epp = _uv(thp, php)
    psi = np.arctan2(a_p, a_t)
    psip = np.arctan2(np.sum(tp * epp, -1), np.sum(tp * etp, -1))
    g = psi - psip
    P = (Q + 1j * U) * np.exp(2j * g)
    return np.real(P), np.imag(P), thp, np.mod(php, 2 * math.pi), xp


def _uv(theta, phi):
    st, ct, sp, cp = np.sin(theta), np.cos(theta), np.sin(phi), np.cos(phi)
    return (np.stack([st * cp, st * sp, ct], -1), np.stack([ct * cp, ct * sp, -st], -1),
            np.stack([-sp, cp, 0 * sp], -1))


def test_p8_rotation_closed_form_matches_3d_transport(oracle):
    rng = np.random.default_rng(0)
    n = 4000
    theta = np.concatenate([rng.uniform(0, math.pi, n - 8), [0.0] * 4, [math.pi] * 4])
    phi = rng.uniform(0, 2 * math.pi, n)
    a_t = rng.normal(0, 0.2, n)
    a_p = rng.normal(0, 0.2, n)
    Q = rng.normal(size=n)
    U = rng.normal(size=n)
    Qc, Uc, thp, php, xp = _closed_form_rotation(Q, U, theta, phi, a_t, a_p)
    Q3, U3 = oracle.rotate_pol_3d(Q, U, theta, phi, thp, php, xp)
    np.testing.assert_allclose(Q3, Qc, atol=2e-13)
    np.testing.assert_allclose(U3, Uc, atol=2e-13)
    # unitary
    np.testing.assert_allclose(np.hypot(Q3, U3), np.hypot(Q, U), rtol=1e-13)
    # the oracle's own positions agree with the construction used here
    gt, gp, gx, _, _ = oracle.geodesic_positions(theta, phi, a_t, a_p)
    np.testing.assert_allclose(gx, xp, atol=1e-15)


def test_p8_rotation_identity_at_zero_deflection(oracle):
    rng = np.random.default_rng(1)
    theta = rng.uniform(0, math.pi, 50)
    phi = rng.uniform(0, 2 * math.pi, 50)
    Q, U = rng.normal(size=50), rng.normal(size=50)
    x = _uv(theta, phi)[0]
    Q3, U3 = oracle.rotate_pol_3d(Q, U, theta, phi, theta, phi, x)
    np.testing.assert_allclose(Q3, Q, atol=1e-15)
    np.testing.assert_allclose(U3, U, atol=1e-15)


def test_p8_pole_ring_invariants(oracle):
    lmax = 32
    ntheta, nphi = 2 * lmax + 1, 2 * lmax + 2
    pix = (math.pi / (ntheta - 1)) / skygen.ARCMIN
    sky = skygen.make_sky(lmax, 21, rms_arcmin=1.5 * pix)
    res = oracle.lens_rings(lmax, 3, ntheta, nphi, [0, ntheta - 1], sky.alm_T, sky.alm_E, sky.alm_B,
                            sky.alm_phi)
    ph = oracle.grid_phi(nphi)
    T = res["T"]
    P = res["Q"] + 1j * res["U"]
    for r, sgn in ((0, 1), (1, -1)):
        assert np.ptp(T[r]) <= 1e-12 * np.max(np.abs(T))
        rot = P[r] * np.exp(2j * sgn * ph)
        assert np.max(np.abs(rot - rot[0])) <= 1e-12 * np.max(np.abs(P))


def test_p9_positions_geometry(oracle):
    rng = np.random.default_rng(2)
    n = 3000
    theta = rng.uniform(0.01, math.pi - 0.01, n)
    phi = rng.uniform(0, 2 * math.pi, n)
    a_t = rng.normal(0, 1e-3, n)
    a_p = rng.normal(0, 1e-3, n)
    thp, php, xp, d, u = oracle.geodesic_positions(theta, phi, a_t, a_p)
    x, et, ep = _uv(theta, phi)
    dist = np.arctan2(np.linalg.norm(np.cross(x, xp), axis=-1), np.sum(x * xp, -1))
    np.testing.assert_allclose(dist, np.hypot(a_t, a_p), atol=1e-15, rtol=1e-13)
    # bearing at x of the great circle through x and x'
    t0 = xp - np.sum(x * xp, -1)[:, None] * x
    bearing = np.arctan2(np.sum(t0 * ep, -1), np.sum(t0 * et, -1))
    dpsi = np.angle(np.exp(1j * (bearing - np.arctan2(a_p, a_t))))
    assert np.max(np.abs(dpsi)) < 1e-9
    # the naive rule differs at second order in alpha
    nt, npp = oracle.naive_positions(theta, phi, a_t, a_p)
    diff = np.hypot(nt - thp, np.sin(theta) * np.angle(np.exp(1j * (npp - php))))
    alpha2 = a_t ** 2 + a_p ** 2
    assert np.max(diff / (alpha2 / np.sin(theta))) < 2.0


def test_p9_pole_ring_shares_one_position(oracle):
    lmax = 40
    ntheta, nphi = 2 * lmax + 1, 2 * lmax + 2
    sky = skygen.make_sky(lmax, 5)
    a_t, a_p = oracle.deflection_rings(lmax, sky.alm_phi, ntheta, nphi, [0, ntheta - 1])
    th = oracle.grid_theta(ntheta)[[0, ntheta - 1]][:, None] + 0 * a_t
    ph = oracle.grid_phi(nphi)[None, :] + 0 * a_t
    _, _, xp, _, _ = oracle.geodesic_positions(th, ph, a_t, a_p)
    for r in range(2):
        # unit-vector components agree to a few ulp of 1
        assert np.max(np.abs(xp[r] - xp[r, 0])) < 1e-15
    # continuity: alpha_phi at a tiny colatitude tends to the pole-ring value
    eps = 1e-7
    F = oracle.ring_coeffs(lmax, 1, [eps], alm_T=sky.alm_phi)["T"]
    ap_eps = oracle.phi_synth(F[:, 0, :], 1, nphi)[0] / math.sin(eps)
    at_eps = oracle.phi_synth(F[:, 1, :], 0, nphi)[0]
    np.testing.assert_allclose(ap_eps, a_p[0], atol=1e-5 * np.max(np.abs(a_p[0])))
    np.testing.assert_allclose(at_eps, a_t[0], atol=1e-5 * np.max(np.abs(a_t[0])))


def test_p9_naive_rule_reflects_over_the_poles_like_the_meridian(oracle):
    """With alpha_phi = 0 the displacement runs along the meridian, which is
    a great circle: pushed across a pole, the naive rule (coordinate
    addition, reflected) and the geodesic rule must land on the same point,
    theta' = |theta + a_t| (or 2 pi - (theta + a_t)) on the meridian phi + pi."""
    rng = np.random.default_rng(12)
    n = 2000
    th_n = rng.uniform(0.01, 0.05, n)                 # near the north pole
    at_n = -th_n - rng.uniform(0.01, 0.05, n)         # crosses it
    th_s = math.pi - rng.uniform(0.01, 0.05, n)       # near the south pole
    at_s = (math.pi - th_s) + rng.uniform(0.01, 0.05, n)
    # and points that do not cross, either way
    th_m = rng.uniform(0.2, math.pi - 0.2, n)
    at_m = rng.normal(0, 0.05, n)
    theta = np.concatenate([th_n, th_s, th_m])
    a_t = np.concatenate([at_n, at_s, at_m])
    phi = rng.uniform(0, 2 * math.pi, theta.size)
    a_p = np.zeros_like(theta)
    nt, npp = oracle.naive_positions(theta, phi, a_t, a_p)
    gt, gp, _, _, _ = oracle.geodesic_positions(theta, phi, a_t, a_p)
    np.testing.assert_allclose(nt, gt, rtol=0, atol=4e-16 * math.pi)
    dphi = np.angle(np.exp(1j * (npp - gp)))
    assert np.max(np.abs(dphi)) < 3e-15
    # the crossing points end on the opposite meridian at the stated colatitude
    k = slice(0, n)
    np.testing.assert_allclose(nt[k], -(th_n + at_n), rtol=0, atol=1e-16)
    np.testing.assert_allclose(np.angle(np.exp(1j * (npp[k] - phi[k] - math.pi))), 0.0, atol=3e-15)
    k = slice(n, 2 * n)
    np.testing.assert_allclose(nt[k], 2 * math.pi - (th_s + at_s), rtol=0, atol=1e-15)
    np.testing.assert_allclose(np.angle(np.exp(1j * (npp[k] - phi[k] - math.pi))), 0.0, atol=3e-15)
    k = slice(2 * n, 3 * n)
    np.testing.assert_allclose(nt[k], th_m + at_m, rtol=0, atol=1e-15)


@pytest.mark.parametrize("lmax,pol", [(1024, True), (1536, False)])
def test_p3_high_l_theta_derivatives_from_the_doubled_circle(oracle, lmax, pol):
    """theta-derivatives j <= 6 of the harmonic sums at high l, against the
    spectral derivative of the oracle's own j = 0 sums (pinned by the
    addition theorem and scipy) on the doubled circle: each F_m(theta),
    continued over the poles as F_m(2 pi - t) = (-1)^m F_m(t) (spin 0 and,
    for Q/U, spin 2), is a trig polynomial of degree <= lmax, so with
    ntheta = lmax + 3 rings its Fourier series and all its derivatives are
    exact.  Rings near both poles (the exponent-scaled underflow range), at
    mid-latitude and at the equator."""
    ntheta = lmax + 3
    nd = 2 * (ntheta - 1)
    th = oracle.grid_theta(ntheta)
    aT = skygen.random_alm(lmax, 31)
    aE = skygen.random_alm(lmax, 32, lmin=2) if pol else None
    aB = skygen.random_alm(lmax, 33, lmin=2) * 0.5 if pol else None
    F0 = oracle.ring_coeffs(lmax, 0, th, aT, aE, aB)
    rings = np.array([1, 2, 3, 5, 9, 17, 40, ntheta // 4, ntheta // 2 - 1, ntheta // 2,
                      3 * ntheta // 4, ntheta - 10, ntheta - 3, ntheta - 2])
    J = 6
    Fj = oracle.ring_coeffs(lmax, J, th[rings], aT, aE, aB)
    m = np.arange(lmax + 1)
    p = np.fft.fftfreq(nd, d=1.0 / nd)
    E = np.exp(1j * np.multiply.outer(th[rings], p))           # [ring, q]
    worst = 0.0
    for f in F0:
        dbl = np.zeros((nd, lmax + 1), np.complex128)
        dbl[:ntheta] = F0[f][:, 0, :]
        dbl[ntheta:] = ((-1.0) ** m) * F0[f][nd - np.arange(ntheta, nd), 0, :]
        c = np.fft.fft(dbl, axis=0) / nd
        assert np.max(np.abs(c[np.abs(p) > lmax])) < 1e-12 * np.max(np.abs(c))
        for j in range(J + 1):
            exact = (E * (1j * p) ** j) @ c                    # [ring, m]
            got = Fj[f][:, j, :]
            scale = np.max(np.abs(exact))
            err = np.max(np.abs(got - exact)) / scale
            worst = max(worst, err)
            assert err < 5e-12, (f, j, err)
    print("worst relative derivative error", worst)


def test_p10_exact_lensing_is_the_brute_force_sum_at_the_displaced_positions(oracle, small_sky):
    """exact_lensed_pixels (the reference of the accuracy-vs-time sweep)
    against sum a_lm Y_lm(x') by scipy / Goldberg at its own positions, and
    against the order-14 Taylor remap, which P1 pins to the same sums."""
    lmax, ntheta, nphi, sky, almB = small_sky
    rng = np.random.default_rng(5)
    rings = rng.integers(0, ntheta, 60)
    cols = rng.integers(0, nphi, 60)
    ex = oracle.exact_lensed_pixels(lmax, ntheta, nphi, rings, cols, sky.alm_T, sky.alm_E, almB, sky.alm_phi,
                                    rotate=False)
    supT = _sup_bound_T(sky.alm_T, lmax)
    supP = _sup_bound_P(sky.alm_E, almB, lmax)
    bT = pinlib.brute_T(sky.alm_T, lmax, ex["_thp"], ex["_php"])
    bQ, bU = pinlib.brute_QU(sky.alm_E, almB, lmax, ex["_thp"], ex["_php"])
    assert np.max(np.abs(ex["T"] - bT)) < 1e-12 * supT
    assert np.max(np.abs(ex["Q"] - bQ)) < 1e-12 * supP
    assert np.max(np.abs(ex["U"] - bU)) < 1e-12 * supP
    # with the rotation: the converged Taylor remap on the same pixels
    exr = oracle.exact_lensed_pixels(lmax, ntheta, nphi, rings, cols, sky.alm_T, sky.alm_E, almB, sky.alm_phi)
    tay = oracle.lens_map(lmax, 14, ntheta, nphi, sky.alm_T, sky.alm_E, almB, sky.alm_phi)
    for f, sup in (("T", supT), ("Q", supP), ("U", supP)):
        assert np.max(np.abs(exr[f] - tay[f][rings, cols])) < 1e-12 * sup, f
    # no deflection: the unlensed map itself
    z = oracle.exact_lensed_pixels(lmax, ntheta, nphi, rings, cols, sky.alm_T, sky.alm_E, almB, None)
    un = oracle.unlensed_map(lmax, ntheta, nphi, sky.alm_T, sky.alm_E, almB)
    for f in "TQU":
        np.testing.assert_allclose(z[f], un[f][rings, cols], rtol=0, atol=1e-13 * supT)


def test_p11_deflection_band_limit_above_the_fields(oracle):
    """A lensing potential of higher band limit than the fields (Sec. II.A):
    lensing fields of lmax 24 with a potential of lmax 40 equals lensing the
    same fields zero-padded to lmax 40, bit for bit; the deflection takes the
    potential's own band limit, which lmax_of reads from the array (and
    refuses for a non-triangular length)."""
    L, Lp = 24, 40
    ntheta, nphi = 2 * Lp + 1, 2 * Lp + 16
    sky = skygen.make_sky(L, 61, pol=True, rms_arcmin=1.5 * (math.pi / (ntheta - 1)) / skygen.ARCMIN)
    phi = skygen.make_sky(Lp, 62, pol=False, rms_arcmin=1.5 * (math.pi / (ntheta - 1)) / skygen.ARCMIN).alm_phi

    def pad(a):
        out = np.zeros((Lp + 1) * (Lp + 2) // 2, np.complex128)
        for m in range(L + 1):
            out[m * (2 * Lp + 1 - m) // 2 + m: m * (2 * Lp + 1 - m) // 2 + L + 1] = \
                a[m * (2 * L + 1 - m) // 2 + m: m * (2 * L + 1 - m) // 2 + L + 1]
        return out

    assert oracle.lmax_of(phi) == Lp and oracle.lmax_of(sky.alm_T) == L
    with pytest.raises(ValueError):
        oracle.lmax_of(np.zeros(7))
    a = oracle.lens_map(L, 3, ntheta, nphi, sky.alm_T, sky.alm_E, None, phi)
    b = oracle.lens_map(Lp, 3, ntheta, nphi, pad(sky.alm_T), pad(sky.alm_E), None, phi)
    for f in "TQU":
        np.testing.assert_array_equal(a[f], b[f])
    # the potential's modes above the fields' band limit move pixels
    cut = phi.copy()
    for m in range(Lp + 1):
        for l in range(max(m, L + 1), Lp + 1):
            cut[m * (2 * Lp + 1 - m) // 2 + l] = 0
    c = oracle.lens_map(L, 3, ntheta, nphi, sky.alm_T, sky.alm_E, None, cut)
    assert np.max(np.abs(c["_alpha_theta"] - a["_alpha_theta"])) > 1e-3 * np.max(np.abs(a["_alpha_theta"]))


@pytest.mark.parametrize("lmax,ntheta,nphi", [(30, 33, 64), (31, 33, 66), (60, 65, 122)])
def test_p12_fft_theta_derivatives_equal_the_recursion_for_band_limited_fields(oracle, lmax, ntheta, nphi):
    """Step 8 (theta-derivatives by FFT along the great circles through both
    poles, Sec. IV) against step 1's Legendre / Wigner-d recursion: for T and
    for Q, U with E and B (components in the (e_theta, e_phi) basis), the FFT
    derivatives of every D_{0,k} equal the recursion's D_{j,k}, j + k <= 4,
    on every ring including both poles and on both meridians of each circle;
    lmax = ntheta - 2 is the largest band limit the circle of
    2 (ntheta - 1) points carries, and nphi / 2 = 33 makes one circle of
    pairs of meridians odd."""
    order = 4
    sky = skygen.make_sky(lmax, 3, pol=True)
    aB = skygen.random_alm(lmax, 1003, lmin=2) * 0.2
    D = oracle.derivative_rings(lmax, order, ntheta, nphi, np.arange(ntheta), sky.alm_T, sky.alm_E, aB)
    dth = math.pi / (ntheta - 1)
    dph = 2 * math.pi / nphi
    hp = nphi // 2
    for f in "TQU":
        for k in range(order):
            base = D[f][(0, k)] * dph ** k / math.factorial(k)
            out = oracle.theta_derivs_fft(base, order - k)
            for j in range(1, order - k + 1):
                want = D[f][(j, k)] * dth ** j * dph ** k / (math.factorial(j) * math.factorial(k))
                got = out[j - 1]
                err = max(np.max(np.abs(got[:, :hp] - want[:, :hp])), np.max(np.abs(got[:, hp:] - want[:, hp:])))
                assert err < 1e-12 * np.max(np.abs(want)), (f, j, k, err)


@pytest.mark.parametrize("q", [0, 1, 5, 15, 16])
def test_p12_fft_theta_derivatives_of_single_circle_harmonics(oracle, q):
    """Closed form: a map whose samples along every circle are cos(q tau + psi_c)
    (tau the angle along the circle from the north pole down meridian c) has
    scaled derivatives dtheta^j / j! q^j cos(q tau + psi_c + j pi / 2) on
    meridian c and (-1)^j times that on meridian c + pi, where theta runs
    against tau.  At the Nyquist degree q = P / 2 = 16 the samples are
    cos(psi_c) cos(P/2 tau): even derivatives only, odd ones zero."""
    ntheta, nphi = 17, 10
    P, hp = 2 * (ntheta - 1), nphi // 2
    th = oracle.grid_theta(ntheta)
    psi = np.random.default_rng(q).uniform(0, 2 * np.pi, hp)
    m = np.zeros((ntheta, nphi))
    for c in range(hp):
        m[:, c] = np.cos(q * th + psi[c])
        m[:, c + hp] = np.cos(q * (2 * np.pi - th) + psi[c])
    out = oracle.theta_derivs_fft(m, 5)
    dth = math.pi / (ntheta - 1)
    for j in range(1, 6):
        want = np.zeros((ntheta, nphi))
        for c in range(hp):
            amp, ph = (math.cos(psi[c]), 0.0) if q == P // 2 else (1.0, psi[c])
            if q == P // 2 and j % 2:
                continue
            want[:, c] = amp * q ** j * np.cos(q * th + ph + j * np.pi / 2)
            want[:, c + hp] = (-1) ** j * amp * q ** j * np.cos(q * (2 * np.pi - th) + ph + j * np.pi / 2)
        want *= dth ** j / math.factorial(j)
        assert np.max(np.abs(out[j - 1] - want)) < 1e-13 * max(1.0, q ** j * dth ** j), (j, q)
    # the column subset returns the same columns
    sub = oracle.theta_derivs_fft(m, 2, cols=[1, 3])
    np.testing.assert_array_equal(sub[..., [0, 1]], out[:2][..., [1, 3]])
    np.testing.assert_array_equal(sub[..., [2, 3]], out[:2][..., [1 + hp, 3 + hp]])


@pytest.mark.parametrize("ntheta", [2, 3, 4, 9, 16, 33, 41])
def test_p13_clenshaw_curtis_weights_integrate_polynomials(oracle, ntheta):
    """Step 9's ring weights: the integral of x^k over [-1, 1] for every k <= N
    (the degree the rule is exact for), symmetric weights summing to 2."""
    N = ntheta - 1
    w = oracle.cc_weights(ntheta)
    x = np.cos(math.pi * np.arange(ntheta) / N)
    np.testing.assert_allclose(w, w[::-1], rtol=0, atol=1e-15)
    for k in range(N + 1):
        exact = (1.0 + (-1.0) ** k) / (k + 1.0)
        assert abs(np.dot(w, x ** k) - exact) < 1e-14, (k, np.dot(w, x ** k), exact)


def test_p13_analysis_closed_forms_and_round_trip(oracle):
    """Step 9's analysis: T = 1 has a_00 = sqrt(4 pi) and T = cos theta has
    a_10 = sqrt(4 pi / 3), nothing else; a band-limited map synthesized by
    step 1 (lmax 24, E-independent T) comes back to its a_lm when
    L + lmax <= ntheta - 1 and misses them when the grid is too coarse."""
    lmax, ntheta, nphi = 24, 49, 50
    th = oracle.grid_theta(ntheta)
    one = oracle.analysis_T(np.ones((ntheta, nphi)), lmax)
    want = np.zeros_like(one)
    want[0] = math.sqrt(4 * math.pi)
    np.testing.assert_allclose(one, want, rtol=0, atol=1e-13)
    cz = oracle.analysis_T(np.repeat(np.cos(th)[:, None], nphi, axis=1), lmax)
    want = np.zeros_like(cz)
    want[1] = math.sqrt(4 * math.pi / 3)
    np.testing.assert_allclose(cz, want, rtol=0, atol=1e-13)
    alm = skygen.random_alm(lmax, 77)
    alm[:lmax + 1] = alm[:lmax + 1].real                      # m = 0 entries are real
    T = oracle.unlensed_map(lmax, ntheta, nphi, alm)["T"]
    back = oracle.analysis_T(T, lmax)
    assert np.max(np.abs(back - alm)) < 1e-12 * np.max(np.abs(alm))
    Tc = oracle.unlensed_map(lmax, 25, nphi, alm)["T"]       # L + lmax = 48 > 24
    assert np.max(np.abs(oracle.analysis_T(Tc, lmax) - alm)) > 1e-3 * np.max(np.abs(alm))


def test_p13_spectrum_binning_and_ell_star(oracle):
    """C_l from a_lm (one entry a_32 = 1 + i: C_3 = 2 |a_32|^2 / 7), bins of
    50 multipoles from l = 2, and the l* rule: the last bin before the first
    whose mean relative error exceeds 0.5 % by more than 4 standard errors."""
    lmax = 10
    alm = np.zeros((lmax + 1) * (lmax + 2) // 2, np.complex128)
    alm[2 * (2 * lmax + 1 - 2) // 2 + 3] = 1 + 1j
    cl = oracle.cl_from_alm(alm, lmax)
    np.testing.assert_allclose(cl, np.where(np.arange(lmax + 1) == 3, 4.0 / 7.0, 0.0), atol=1e-15)
    c, m = oracle.bin_cl(np.arange(160, dtype=float))
    np.testing.assert_array_equal(c, [26.5, 76.5, 126.5])
    np.testing.assert_allclose(m, [26.5, 76.5, 126.5])
    centres = np.array([26.5, 76.5, 126.5, 176.5])
    e = np.array([[0.001, 0.004, 0.010, 0.001], [0.001, 0.006, 0.011, 0.001], [0.001, 0.005, 0.012, 0.002]])
    assert oracle.ell_star(centres, e) == 76.5                  # bin 3 fails, bin 2 is within its error
    assert oracle.ell_star(centres, np.full((3, 4), 0.001)) == 176.5
    assert oracle.ell_star(centres, np.full((3, 4), 0.02)) is None
    assert oracle.ell_star(centres, [[0.001, 0.0051, 0.0, 0.0]]) == 26.5   # one simulation: no error bar


def test_p13_spin2_analysis_round_trip(oracle):
    """Step 9's E/B analysis: Q/U maps synthesized by step 1 from E and B of
    lmax 20 (Goldberg-pinned spin-2 functions) come back to E and B on 41
    rings of 42 pixels; an E-only sky has no B; too few rings miss them."""
    lmax, ntheta, nphi = 20, 41, 42
    aT = skygen.random_alm(lmax, 1)
    aE = skygen.random_alm(lmax, 2, lmin=2)
    aB = skygen.random_alm(lmax, 3, lmin=2)
    for a in (aE, aB):
        a[:lmax + 1] = a[:lmax + 1].real
    m = oracle.unlensed_map(lmax, ntheta, nphi, aT, aE, aB)
    E, B = oracle.analysis_EB(m["Q"], m["U"], lmax)
    assert np.max(np.abs(E - aE)) < 1e-12 * np.max(np.abs(aE))
    assert np.max(np.abs(B - aB)) < 1e-12 * np.max(np.abs(aB))
    m0 = oracle.unlensed_map(lmax, ntheta, nphi, aT, aE, None)
    E0, B0 = oracle.analysis_EB(m0["Q"], m0["U"], lmax)
    assert np.max(np.abs(E0 - aE)) < 1e-12 * np.max(np.abs(aE))
    assert np.max(np.abs(B0)) < 1e-12 * np.max(np.abs(aE))
    mc = oracle.unlensed_map(lmax, 21, nphi, aT, aE, aB)
    Ec, _ = oracle.analysis_EB(mc["Q"], mc["U"], lmax)
    assert np.max(np.abs(Ec - aE)) > 1e-3 * np.max(np.abs(aE))


@pytest.mark.parametrize("lmax,ntheta,nphi,pol", [(511, 513, 1024, False), (255, 257, 512, True)])
def test_p12_fft_theta_derivatives_at_higher_l(oracle, lmax, ntheta, nphi, pol):
    """Step 8 against step 1 at lmax 511 (T) and 255 (T, Q, U): the FFT
    derivatives (j <= 2) of the recursion's D_{0,k} equal its D_{j,k}, on
    every ring, to 1e-11 of the largest value."""
    order = 2
    aT = skygen.random_alm(lmax, 41)
    aE = skygen.random_alm(lmax, 42, lmin=2) if pol else None
    D = oracle.derivative_rings(lmax, order, ntheta, nphi, np.arange(ntheta), aT, aE, None)
    dth = math.pi / (ntheta - 1)
    for f in D:
        for k in range(order):
            out = oracle.theta_derivs_fft(D[f][(0, k)], order - k)
            hp = nphi // 2
            for j in range(1, order - k + 1):
                want = D[f][(j, k)] * dth ** j / math.factorial(j)
                got = np.concatenate([out[j - 1][:, :hp], out[j - 1][:, hp:]], axis=1)
                assert np.max(np.abs(got - want)) < 1e-11 * np.max(np.abs(want)), (f, j, k)
