"""HIP path vs the CPU oracle, through the C ABI (marked gpu).

Stage by stage (deflection, harmonic stage, derivative maps, remap) at sizes
the oracle finishes in seconds and that span several 64-ring tiles, 8-m
groups and a ragged tail; then whole-map parity on the T-only lmax=256
workload, sampled-ring parity at the lmax=2048 and lmax=4096 T+Q/U sizes in
the launch configuration the benchmark uses, and the edge cases.

Tolerances: FP64 form 1e-12 (relative RMS per field, C12 reading), 1e-11 on
max |err| / RMS; FP32 form 1e-5 relative RMS (the stated target for the plain
FP32 path) and 1e-4 max |err| / RMS.  Pixels whose displaced position lies
within 1e-9 pixel of a rounding tie are excluded (either neighbour is a valid
expansion point); their count is asserted to be tiny.
"""
import math

import numpy as np
import pytest
import torch

from paper_1307_0719_amd import skygen
from tests.gpu_util import (ORACLE_THREADS, dmap_scale, max_rel, need_gpu, oracle_scaled_derivs, rel_rms,
                            smooth_nphi, t2np)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tl():
    need_gpu()
    from paper_1307_0719_amd import taylens

    taylens.lib()
    return taylens


def _sky(lmax, seed, pol=True, with_b=False, rms_pix=None, ntheta=None):
    rms = skygen.DEFLECTION_RMS_ARCMIN
    if rms_pix is not None:
        rms = rms_pix * (math.pi / (ntheta - 1)) / skygen.ARCMIN
    sky = skygen.make_sky(lmax, seed, pol=pol, rms_arcmin=rms)
    if with_b:
        sky.alm_B = skygen.random_alm(lmax, seed + 1000, lmin=2) * 0.2
    return sky


# ------------------------------------------------------------- stages ----

@pytest.mark.parametrize("lmax,ntheta,nphi", [(40, 41, 80), (40, 70, 96), (130, 131, 270), (0, 2, 2), (1, 3, 4)])
def test_deflection_fp64(tl, oracle, lmax, ntheta, nphi):
    sky = _sky(lmax, 5, rms_pix=2.0, ntheta=ntheta)
    plan = tl.Plan(lmax, ntheta, nphi, 2, "fp64", pol=False)
    at, ap = plan.deflection(sky.alm_phi)
    ot, op = oracle.deflection_rings(lmax, sky.alm_phi, ntheta, nphi, np.arange(ntheta), ORACLE_THREADS)
    if lmax == 0:
        assert np.all(t2np(at) == 0) and np.all(t2np(ap) == 0)
        return
    assert max_rel(t2np(at), ot) < 1e-11
    assert max_rel(t2np(ap), op) < 1e-11


@pytest.mark.parametrize("precision", ["fp32", "fp16"])
@pytest.mark.parametrize("lmax,ntheta,nphi", [(40, 41, 80), (130, 131, 270), (300, 301, 600), (257, 200, 540)])
def test_deflection_other_forms(tl, oracle, precision, lmax, ntheta, nphi):
    """Plans of the FP32 and tabulated forms: the deflection entry point keeps
    the FP64 arithmetic (several ring blocks, a ragged last one).  Bars:
    relative RMS 3e-6 and max |err| / RMS 5e-5 (the FP32 harmonic-stage bars,
    far above what FP64 reaches)."""
    sky = _sky(lmax, 6, rms_pix=2.0, ntheta=ntheta)
    plan = tl.Plan(lmax, ntheta, nphi, 2, precision, pol=False)
    at, ap = plan.deflection(sky.alm_phi)
    ot, op = oracle.deflection_rings(lmax, sky.alm_phi, ntheta, nphi, np.arange(ntheta), ORACLE_THREADS)
    for g, ref in ((t2np(at), ot), (t2np(ap), op)):
        err = g - ref
        rms = np.sqrt(np.mean(ref ** 2))
        print(precision, lmax, ntheta, "rel RMS", np.sqrt(np.mean(err ** 2)) / rms, "max/RMS", np.abs(err).max() / rms)
        assert np.sqrt(np.mean(err ** 2)) / rms < 3e-6
        assert np.abs(err).max() / rms < 5e-5


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("lmax,ntheta,order,with_b", [
    (37, 38, 3, True), (37, 75, 5, False), (130, 129, 4, True), (70, 200, 8, True), (3, 5, 2, True),
    (2, 2, 1, False)])
def test_legendre_stage(tl, oracle, precision, lmax, ntheta, order, with_b):
    nphi = smooth_nphi(max(2, 2 * lmax + 2))
    sky = _sky(lmax, 7, with_b=with_b)
    plan = tl.Plan(lmax, ntheta, nphi, order, precision, pol=True)
    F = t2np(plan.legendre(sky.alm_T, sky.alm_E, sky.alm_B))
    th = oracle.grid_theta(ntheta)
    ref = oracle.ring_coeffs(lmax, order, th, sky.alm_T, sky.alm_E, sky.alm_B, ORACLE_THREADS)
    # FP64 form: 1e-11 on max |err| / RMS of each (field, j) block.  FP32 form
    # (L-power contraction on MFMA away from the polar caps): relative RMS
    # 3e-6 and max |err| / RMS 5e-5 per block -- operand rounding amplified by
    # the 1/sin theta coefficients near the caps; the maps stay within 1e-5.
    for f, name in enumerate(("T", "Q", "U")):
        for j in range(order + 1):
            got = F[f, j]
            want = ref[name][:, j, :]
            scale = np.sqrt(np.mean(np.abs(want) ** 2))
            if scale == 0:
                assert np.max(np.abs(got)) == 0
                continue
            emax = np.max(np.abs(got - want)) / scale
            erms = np.sqrt(np.mean(np.abs(got - want) ** 2)) / scale
            if precision == "fp64":
                assert emax < 1e-11, (name, j, emax)
            else:
                assert erms < 3e-6 and emax < 5e-5, (name, j, erms, emax)


@pytest.mark.parametrize("lmax,ntheta,order,with_b", [(64, 301, 4, True), (200, 201, 6, False), (96, 97, 2, True)])
def test_legendre_fp32_near_poles(tl, oracle, lmax, ntheta, order, with_b):
    """FP32 form (matrix-core contraction of the L-power form away from the
    poles): every ring, in particular the first rings past the pole-adjacent
    ones that stay on the direct kernel, against the oracle."""
    nphi = smooth_nphi(2 * lmax + 2)
    sky = _sky(lmax, 71, with_b=with_b)
    plan = tl.Plan(lmax, ntheta, nphi, order, "fp32", pol=True)
    F = t2np(plan.legendre(sky.alm_T, sky.alm_E, sky.alm_B))
    ref = oracle.ring_coeffs(lmax, order, oracle.grid_theta(ntheta), sky.alm_T, sky.alm_E, sky.alm_B,
                             ORACLE_THREADS)
    worst, rms = [], []
    for f, name in enumerate(("T", "Q", "U")):
        for j in range(order + 1):
            want = ref[name][:, j, :]
            scale = np.sqrt(np.mean(np.abs(want) ** 2))
            err_ring = np.max(np.abs(F[f, j] - want), axis=1) / scale
            worst.append((float(err_ring.max()), name, j, int(err_ring.argmax())))
            rms.append(float(np.sqrt(np.mean(np.abs(F[f, j] - want) ** 2)) / scale))
    worst.sort(reverse=True)
    assert worst[0][0] < 5e-5, worst[:5]
    assert max(rms) < 3e-6, rms


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_derivative_maps(tl, oracle, precision):
    lmax, ntheta, nphi, order = 60, 61, 120, 4   # nphi = 2 lmax: Nyquist bin present
    sky = _sky(lmax, 11, with_b=True)
    plan = tl.Plan(lmax, ntheta, nphi, order, precision, pol=True)
    D = t2np(plan.synth_derivs(sky.alm_T, sky.alm_E, sky.alm_B))
    ref = oracle_scaled_derivs(oracle, lmax, order, ntheta, nphi, np.arange(ntheta), sky.alm_T, sky.alm_E,
                               sky.alm_B)
    tol = 1e-12 if precision == "fp64" else 1e-6
    for f in range(3):
        for q in range(ref.shape[1]):
            assert max_rel(D[f, q], ref[f, q]) < 10 * tol, (f, q)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("nphi,lmax", [(1024, 511), (2048, 1023), (4096, 2047), (8192, 4095),
                                       (2048, 300), (4096, 2048)])
def test_derivative_maps_power_of_two_rings(tl, oracle, precision, nphi, lmax):
    """Every length of the power-of-two ring FFT (M = nphi/2 = 512..4096, the
    paired spectrum build; FP32 keeps the row for all of a job's outputs) in
    both FFT precisions, lmax up to the last bin below Nyquist, order 4 (up
    to five phi-derivative outputs per row): sampled rings vs the oracle;
    also a row far shorter than the ring (zeros from clamped reads) and
    lmax = nphi/2 (the Nyquist bin enters through the mirrored term).
    FP64 bar: the stage-map bar, relative RMS 1e-11 (1e-10 on the maximum)
    up to lmax 2048, growing as lmax^2 beyond: the rounding of the
    l-recursion and of the m^k-weighted sums grows with lmax (worst map
    measured 1.9e-12, 6.5e-12, 2.1e-11 at lmax 1023, 2047, 4095)."""
    ntheta, order = 25, 4
    rings = np.array([0, 1, 5, 12])
    sky = _sky(lmax, 21)
    plan = tl.Plan(lmax, ntheta, nphi, order, precision, pol=True)
    D = t2np(plan.synth_derivs(sky.alm_T, sky.alm_E, None))[:, :, rings]
    ref = oracle_scaled_derivs(oracle, lmax, order, ntheta, nphi, rings, sky.alm_T, sky.alm_E)
    grow = max(1.0, lmax / 2048.0) ** 2
    tol_rms, tol_max = (1e-11 * grow, 1e-10 * grow) if precision == "fp64" else (1e-5, 1e-4)
    errs = [(rel_rms(D[f, q], ref[f, q]), max_rel(D[f, q], ref[f, q]), f, q)
            for f in range(3) for q in range(ref.shape[1])]
    print("worst rel RMS", max(errs), "worst max", max(errs, key=lambda e: e[1]))
    for e_rms, e_max, f, q in errs:
        assert e_rms < tol_rms and e_max < tol_max, (f, q, e_rms, e_max)


@pytest.mark.parametrize("rotate", [1, 0])
def test_remap_from_oracle_inputs(tl, oracle, rotate):
    """tl_remap fed the oracle's derivative maps and deflection reproduces the
    oracle's remap + Taylor sum (+ rotation)."""
    lmax, ntheta, nphi, order = 48, 97, 192, 5
    sky = _sky(lmax, 13, with_b=True, rms_pix=1.7, ntheta=ntheta)
    plan = tl.Plan(lmax, ntheta, nphi, order, "fp64", pol=True, rotate=bool(rotate))
    D = oracle_scaled_derivs(oracle, lmax, order, ntheta, nphi, np.arange(ntheta), sky.alm_T, sky.alm_E, sky.alm_B)
    at, ap = oracle.deflection_rings(lmax, sky.alm_phi, ntheta, nphi, np.arange(ntheta), ORACLE_THREADS)
    T, Q, U = plan.remap(torch.from_numpy(D), torch.from_numpy(at), torch.from_numpy(ap))
    ref = oracle.lens_map(lmax, order, ntheta, nphi, sky.alm_T, sky.alm_E, sky.alm_B, sky.alm_phi,
                          rotate=bool(rotate), nthreads=ORACLE_THREADS)
    mask = ref["_tie"] > 1e-9
    assert np.mean(~mask) < 1e-3
    for name, got in (("T", T), ("Q", Q), ("U", U)):
        assert max_rel(t2np(got), ref[name], mask) < 1e-11, name


# --------------------------------------------------------- end to end ----

def _check_maps(got, ref, fields, tol_rms, tol_max):
    mask = ref["_tie"] > 1e-9
    assert np.mean(~mask) < 1e-3
    errs = {}
    for f, g in zip(fields, got):
        e1 = rel_rms(t2np(g), ref[f], mask)
        e2 = max_rel(t2np(g), ref[f], mask)
        errs[f] = (e1, e2)
        assert e1 < tol_rms, (f, e1)
        assert e2 < tol_max, (f, e2)
    return errs


def test_lens_T256_fp64_whole_map(tl, oracle):
    """T-only lmax=256, 513 x 1024 rings, order 3, FP64: the whole map."""
    w = skygen.WORKLOADS["T256"]
    sky = skygen.make_sky(w.lmax, w.seed, pol=False)
    plan = tl.Plan(w.lmax, w.ntheta, w.nphi, w.order, "fp64", pol=False)
    T, _, _ = plan.lens_map(sky.alm_T, None, None, sky.alm_phi)
    ref = oracle.lens_map(w.lmax, w.order, w.ntheta, w.nphi, sky.alm_T, None, None, sky.alm_phi,
                          nthreads=ORACLE_THREADS)
    _check_maps([T], ref, ["T"], 1e-12, 1e-11)


@pytest.mark.parametrize("precision,tol", [("fp64", (1e-12, 1e-11)), ("fp32", (1e-5, 1e-4))])
def test_lens_TP_whole_map(tl, oracle, precision, tol):
    lmax, ntheta, nphi, order = 128, 129, 256, 4
    sky = _sky(lmax, 17, with_b=True, rms_pix=1.2, ntheta=ntheta)
    plan = tl.Plan(lmax, ntheta, nphi, order, precision, pol=True)
    got = plan.lens_map(sky.alm_T, sky.alm_E, sky.alm_B, sky.alm_phi)
    ref = oracle.lens_map(lmax, order, ntheta, nphi, sky.alm_T, sky.alm_E, sky.alm_B, sky.alm_phi,
                          nthreads=ORACLE_THREADS)
    _check_maps(got, ref, ["T", "Q", "U"], *tol)


@pytest.mark.parametrize("order", [1, 2, 3, 4, 5])
def test_lens_TP2048_fp32_sampled_rings(tl, oracle, order):
    """T+Q/U lmax=2048 on 2049 x 4096 rings, FP32, orders 1-5, sampled output
    rings (poles, pole-adjacent, both sides of the polar-cap boundary,
    mid-latitude, equator) vs the oracle."""
    w = skygen.WORKLOADS["TP2048"]
    sky = skygen.make_sky(w.lmax, w.seed, pol=True)
    plan = tl.Plan(w.lmax, w.ntheta, w.nphi, order, "fp32", pol=True)
    got = [t2np(x) for x in plan.lens_map(sky.alm_T, sky.alm_E, sky.alm_B, sky.alm_phi)]
    rp = plan.query("rpole")
    rings = np.array([0, 1, 3, rp - 2, rp - 1, rp, rp + 1, 700, 1024, w.ntheta - 1 - rp, 2045, 2048])
    ref = oracle.lens_rings(w.lmax, order, w.ntheta, w.nphi, rings, sky.alm_T, sky.alm_E, sky.alm_B,
                            sky.alm_phi, nthreads=ORACLE_THREADS)
    _check_maps([g[rings] for g in got], ref, ["T", "Q", "U"], 1e-5, 1e-4)


def test_lens_TP4096_fp32_sampled_rings(tl, oracle):
    """Full-size T+Q/U lmax=4096, 4097 x 8192 rings, order 4, FP32 -- the
    benchmark's launch -- on sampled output rings vs the oracle."""
    w = skygen.WORKLOADS["TP4096"]
    sky = skygen.make_sky(w.lmax, w.seed, pol=True)
    plan = tl.Plan(w.lmax, w.ntheta, w.nphi, w.order, "fp32", pol=True)
    got = [t2np(x) for x in plan.lens_map(sky.alm_T, sky.alm_E, sky.alm_B, sky.alm_phi)]
    rp = plan.query("rpole")
    rings = np.array([0, 2, rp - 1, rp, rp + 1, 1500, 2048, w.ntheta - 1 - rp, 4096])
    ref = oracle.lens_rings(w.lmax, w.order, w.ntheta, w.nphi, rings, sky.alm_T, sky.alm_E, sky.alm_B,
                            sky.alm_phi, nthreads=ORACLE_THREADS)
    _check_maps([g[rings] for g in got], ref, ["T", "Q", "U"], 1e-5, 1e-4)
    # properties over the whole map: finite, pole rings constant (T) / P e^{+-2i phi} constant
    T, Q, U = got
    assert np.all(np.isfinite(T)) and np.all(np.isfinite(Q)) and np.all(np.isfinite(U))
    ph = 2 * np.pi * np.arange(w.nphi) / w.nphi
    for r, sg in ((0, 1), (w.ntheta - 1, -1)):
        assert np.ptp(T[r]) < 1e-5 * np.sqrt(np.mean(T ** 2))
        P = (Q[r] + 1j * U[r]) * np.exp(2j * sg * ph)
        assert np.max(np.abs(P - P[0])) < 1e-5 * np.sqrt(np.mean(Q ** 2 + U ** 2))


# ----------------------------------------------------------- edge cases --

def test_zero_deflection_gives_unlensed_maps(tl, oracle):
    lmax, ntheta, nphi = 33, 34, 72
    sky = _sky(lmax, 19, with_b=True)
    for precision in ("fp64", "fp32"):
        plan = tl.Plan(lmax, ntheta, nphi, 3, precision, pol=True)
        got = plan.lens_map(sky.alm_T, sky.alm_E, sky.alm_B, None)
        D = plan.synth_derivs(sky.alm_T, sky.alm_E, sky.alm_B)
        for f in range(3):
            assert torch.equal(got[f], D[f, 0]), (precision, f)
    un = oracle.unlensed_map(lmax, ntheta, nphi, sky.alm_T, sky.alm_E, sky.alm_B)
    plan = tl.Plan(lmax, ntheta, nphi, 3, "fp64", pol=True)
    got = plan.lens_map(sky.alm_T, sky.alm_E, sky.alm_B, torch.zeros(skygen.nalm(lmax), dtype=torch.complex128))
    for f, name in enumerate("TQU"):
        assert max_rel(t2np(got[f]), un[name]) < 1e-12


@pytest.mark.parametrize("lmax,ntheta,nphi", [(0, 2, 2), (1, 2, 2), (2, 3, 4), (5, 2, 10), (8, 9, 16), (6, 4, 30)])
def test_tiny_grids(tl, oracle, lmax, ntheta, nphi):
    sky = _sky(lmax, 23, with_b=True, rms_pix=0.8, ntheta=ntheta)
    plan = tl.Plan(lmax, ntheta, nphi, 3, "fp64", pol=True)
    got = plan.lens_map(sky.alm_T, sky.alm_E, sky.alm_B, sky.alm_phi)
    ref = oracle.lens_map(lmax, 3, ntheta, nphi, sky.alm_T, sky.alm_E, sky.alm_B, sky.alm_phi)
    mask = ref["_tie"] > 1e-9
    for f, name in enumerate("TQU"):
        g, r = t2np(got[f])[mask], ref[name][mask]
        scale = max(np.sqrt(np.mean(r ** 2)), 1e-300)
        assert np.max(np.abs(g - r)) <= 1e-11 * scale + 1e-14, name


def test_lens_map_pos_constant_shift(tl, oracle):
    lmax, ntheta, nphi, order = 50, 51, 100, 5
    sky = _sky(lmax, 29, with_b=True)
    th = oracle.grid_theta(ntheta)[:, None] * np.ones((1, nphi))
    ph = oracle.grid_phi(nphi)[None, :] + 1.37 * 2 * np.pi / nphi + 0 * th
    plan = tl.Plan(lmax, ntheta, nphi, order, "fp64", pol=True)
    got = plan.lens_map_pos(sky.alm_T, sky.alm_E, sky.alm_B, torch.from_numpy(th), torch.from_numpy(ph))
    ref = oracle.lens_at_positions(lmax, order, ntheta, nphi, th, ph, sky.alm_T, sky.alm_E, sky.alm_B)
    for f, name in enumerate("TQU"):
        assert max_rel(t2np(got[f]), ref[name]) < 1e-11, name


def test_naive_positions(tl, oracle):
    lmax, ntheta, nphi, order = 40, 41, 80, 3
    sky = _sky(lmax, 31, rms_pix=1.5, ntheta=ntheta)
    plan = tl.Plan(lmax, ntheta, nphi, order, "fp64", pol=True, naive_pos=True)
    got = plan.lens_map(sky.alm_T, sky.alm_E, sky.alm_B, sky.alm_phi)
    ref = oracle.lens_map(lmax, order, ntheta, nphi, sky.alm_T, sky.alm_E, sky.alm_B, sky.alm_phi, naive=True)
    mask = ref["_tie"] > 1e-9
    for f, name in enumerate("TQU"):
        assert max_rel(t2np(got[f]), ref[name], mask) < 1e-11, name


def test_convenience_entry_and_batch(tl):
    lmaxes = [24, 40, 24]
    skies = [_sky(l, 40 + i) for i, l in enumerate(lmaxes)]
    plans = [tl.Plan(l, l + 1, 2 * l, 4, "fp32") for l in lmaxes]
    single = [p.lens_map(s.alm_T, s.alm_E, s.alm_B, s.alm_phi) for p, s in zip(plans, skies)]
    outs = [tuple(torch.empty_like(x) for x in o) for o in single]
    tl.lens_map_batch(plans, [(s.alm_T, s.alm_E, s.alm_B, s.alm_phi) for s in skies], outs)
    torch.cuda.synchronize()
    for a, b in zip(single, outs):
        for x, y in zip(a, b):
            assert torch.equal(x, y)
    s = skies[1]
    T, Q, U = tl.lens_map(s.alm_T, s.alm_E, s.alm_B, s.alm_phi, 40, 4, 41, 80)
    for x, y in zip((T, Q, U), single[1]):
        assert torch.equal(x, y)


def test_invalid_arguments_report_errors(tl):
    with pytest.raises(tl.TaylensError) as e:
        tl.Plan(10, 11, 18, 3, "fp32")  # nphi < 2 lmax
    assert e.value.code == tl.TL_ERR_INVALID
    with pytest.raises(tl.TaylensError) as e:
        tl.Plan(10, 11, 22, 3, "fp32")  # nphi/2 = 11
    assert e.value.code == tl.TL_ERR_UNSUPPORTED
    with pytest.raises(tl.TaylensError) as e:
        tl.Plan(64, 65, 128, 3, "fp32", workspace_cap=1000)
    assert e.value.code == tl.TL_ERR_NOMEM


@pytest.mark.parametrize("precision,batch,nphi", [("fp64", 1, 192), ("fp32", 1, 192), ("fp16x2", 2, 192),
                                                  ("fp32", 1, 1024), ("fp16x2", 3, 1024)])
def test_deflection_band_limit_above_the_fields(tl, oracle, precision, batch, nphi):
    """A lensing potential of lmax_phi = 80 beside fields of lmax 48 (Sec.
    II.A): the deflection (the direct FP64 recursion at the potential's own
    band limit on every ring, also for the tabulated forms) and the lensed
    maps against the oracle, on ring lengths of the mixed-radix and the
    radix-16 FFTs; realizations of one table pass agree with single calls."""
    lmax, lmax_phi, ntheta, order = 48, 80, 49, 3
    rms = 1.5 * (math.pi / (ntheta - 1)) / skygen.ARCMIN
    skies = [skygen.make_sky(lmax, 70 + i, pol=True, rms_arcmin=rms) for i in range(batch)]
    phis = [skygen.make_sky(lmax_phi, 80 + i, pol=False, rms_arcmin=rms).alm_phi for i in range(batch)]
    plan = tl.Plan(lmax, ntheta, nphi, order, precision, pol=True, batch=batch, lmax_phi=lmax_phi)
    at, ap = plan.deflection(phis[0])
    ot, op = oracle.deflection_rings(lmax, phis[0], ntheta, nphi, np.arange(ntheta), ORACLE_THREADS)
    assert max_rel(t2np(at), ot) < 1e-11 and max_rel(t2np(ap), op) < 1e-11
    alms = [(s.alm_T, s.alm_E, None, ph) for s, ph in zip(skies, phis)]
    got = plan.lens_map_many(alms) if batch > 1 else [plan.lens_map(*alms[0])]
    tol = {"fp64": 1e-11, "fp32": 1e-5, "fp16x2": 1e-5}[precision]
    for i in (0, batch - 1):
        ref = oracle.lens_map(lmax, order, ntheta, nphi, skies[i].alm_T, skies[i].alm_E, None, phis[i],
                              nthreads=ORACLE_THREADS)
        mask = ref["_tie"] > 1e-9
        for f, g in zip("TQU", got[i]):
            e = rel_rms(t2np(g), ref[f], mask)
            assert e < tol, (precision, i, f, e)
    if batch > 1:
        for a, s in zip(got, alms):
            for x, y in zip(a, plan.lens_map(*s)):
                assert torch.equal(x, y)
    plan.close()


def test_rings_too_long_for_the_fp64_fft_in_lds(tl, oracle):
    """Rings of 16384 pixels: the FP64 ring transform (two buffers of 8192
    complex) does not fit in a workgroup's LDS, so FP32-map plans take the
    deflection's ring FFTs in FP32 too (FP64 rows and result); the FP64 form
    is refused.  Deflection (potential of lmax_phi 300) and lensed rings of
    the FP32 and split FP16 forms against the oracle."""
    lmax, lmax_phi, ntheta, nphi, order = 64, 300, 65, 16384, 3
    with pytest.raises(tl.TaylensError) as e:
        tl.Plan(lmax, ntheta, nphi, order, "fp64")
    assert e.value.code == tl.TL_ERR_UNSUPPORTED
    rms = 1.5 * (math.pi / (ntheta - 1)) / skygen.ARCMIN
    sky = skygen.make_sky(lmax, 91, pol=True, rms_arcmin=rms)
    phi = skygen.make_sky(lmax_phi, 92, pol=False, rms_arcmin=rms).alm_phi
    rings = np.array([0, 1, 17, 32, 63, 64])
    ref = oracle.lens_rings(lmax, order, ntheta, nphi, rings, sky.alm_T, sky.alm_E, None, phi, nthreads=ORACLE_THREADS)
    mask = ref["_tie"] > 1e-9
    for precision in ("fp32", "fp16x2"):
        plan = tl.Plan(lmax, ntheta, nphi, order, precision, pol=True, lmax_phi=lmax_phi)
        at, ap = plan.deflection(phi)
        assert max_rel(t2np(at)[rings], ref["_alpha_theta"]) < 5e-6
        assert max_rel(t2np(ap)[rings], ref["_alpha_phi"]) < 5e-6
        got = plan.lens_map(sky.alm_T, sky.alm_E, None, phi)
        for f, g in zip("TQU", got):
            e = rel_rms(t2np(g)[rings], ref[f], mask)
            assert e < 1e-5, (precision, f, e)
        plan.close()
