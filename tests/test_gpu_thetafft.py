"""Theta-derivatives by FFT along the great circles through both poles
(tl_theta_derivs, Sec. IV's FFT route on the equal-theta grid) against the
oracle, through the C ABI (marked gpu).

* Method parity: for band-limited fields (lmax <= ntheta - 2) the FFT
  derivatives of the derivative maps D_{0,k} that the library synthesizes
  equal the oracle's recursion maps D_{j,k} (T, Q, U with E and B), and the
  library's own recursion maps; FP64 form, bar 1e-11 of the largest value
  (FP64 rounding of the synthesis, which the transform carries over with a
  gain of at most pi^j / j!).
* Kernel parity: on arbitrary (not band-limited) maps the output equals the
  oracle's definition of the transform (step 8) applied to the same input
  values: FP64 to 1e-12 of the largest input; FP32 to the rounding of each
  output (2^-24 relative) plus 1e-12 of the largest input.
* Sizes: tiny (3 rings), odd counts of circle pairs (nphi / 2 odd: the last
  workgroup takes one circle), several workgroups per map, and the
  4097 x 8192 grid of the lmax 4095 workload (all maps of one field,
  sampled circles and rings).
* The FP64 form with theta_fft (rows j = 0 from the recursion, the rest by
  FFT): derivative maps and lensed maps against the oracle at the FP64 bars
  and against the same plan without the option, batches bit-identical to
  single calls, and T+Q/U order 4 at lmax 4095 on 4097 x 8192 rings.
"""
import ctypes
import math

import numpy as np
import pytest
import torch

from paper_1307_0719_amd import skygen
from tests.gpu_util import ORACLE_THREADS, max_rel, need_gpu, oracle_scaled_derivs, rel_rms, t2np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tl():
    need_gpu()
    from paper_1307_0719_amd import taylens

    taylens.lib()
    return taylens


def _jk(order):
    return [(j, k) for j in range(order + 1) for k in range(order + 1 - j)]


@pytest.mark.parametrize("lmax,ntheta,nphi", [(60, 65, 150), (63, 65, 150), (100, 129, 256)])
def test_fft_theta_derivatives_equal_the_recursion(tl, oracle, lmax, ntheta, nphi):
    order = 4
    sky = skygen.make_sky(lmax, 17, pol=True)
    aB = skygen.random_alm(lmax, 1017, lmin=2) * 0.2
    plan = tl.Plan(lmax, ntheta, nphi, order, "fp64", pol=True)
    D = plan.synth_derivs(sky.alm_T, sky.alm_E, aB)          # [3][15][ntheta][nphi]
    print("theta fft: method parity", lmax, ntheta, nphi, flush=True)
    out = t2np(plan.theta_derivs(D[:, :order], order))        # [3][k][j-1][ntheta][nphi]
    Dh = t2np(D)
    ref = oracle_scaled_derivs(oracle, lmax, order, ntheta, nphi, np.arange(ntheta), sky.alm_T, sky.alm_E, aB)
    pairs = _jk(order)
    for f in range(3):
        for k in range(order):
            for j in range(1, order - k + 1):
                q = pairs.index((j, k))
                got = out[f, k, j - 1]
                scale = np.max(np.abs(ref[f, q]))
                assert np.max(np.abs(got - ref[f, q])) < 1e-11 * scale, (f, j, k)
                assert np.max(np.abs(got - Dh[f, q])) < 1e-11 * scale, (f, j, k)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("ntheta,nphi,lmax,nmaps,jmax", [(3, 4, 1, 2, 3), (9, 10, 5, 3, 5), (65, 150, 60, 3, 4),
                                                         (257, 30, 15, 2, 8), (513, 1024, 500, 2, 4)])
def test_fft_theta_derivatives_match_the_definition(tl, oracle, precision, ntheta, nphi, lmax, nmaps, jmax):
    plan = tl.Plan(lmax, ntheta, nphi, 1, precision, pol=False)
    dt = torch.float64 if precision == "fp64" else torch.float32
    g = torch.Generator().manual_seed(ntheta * 7 + nphi)
    maps = torch.randn((nmaps, ntheta, nphi), generator=g, dtype=torch.float64).to(dt)
    print("theta fft: definition", precision, ntheta, nphi, nmaps, jmax, flush=True)
    out = t2np(plan.theta_derivs(maps.cuda(), jmax))
    m64 = maps.double().numpy()
    want = oracle.theta_derivs_fft(m64, jmax)                 # [nmaps][jmax][ntheta][c..., c+hp...]
    hp = nphi // 2
    want = np.concatenate([want[..., :hp], want[..., hp:]], axis=-1)
    amax = np.max(np.abs(m64))
    if precision == "fp64":
        assert np.max(np.abs(out - want)) < 1e-12 * amax
    else:
        assert np.all(np.abs(out - want) <= 2.0 ** -24 * np.abs(want) + 1e-12 * amax)


def test_fft_theta_derivatives_at_the_lmax4095_grid(tl, oracle):
    """lmax 4095 on 4097 x 8192 rings (the largest circle, 8192 points): T
    derivative maps of the FP64 form, theta-derivatives of D_{0,k}, k <= 3,
    against the library's recursion maps everywhere and the oracle's on
    sampled rings (poles, near-pole rings, the 0.15 cap edge, equator); then
    the FP32 form's maps against the definition on sampled circles."""
    lmax, ntheta, nphi, order = 4095, 4097, 8192, 4
    sky = skygen.make_sky(lmax, 23, pol=False)
    plan = tl.Plan(lmax, ntheta, nphi, order, "fp64", pol=False)
    print("theta fft: lmax 4095 fp64 synthesis", flush=True)
    D = plan.synth_derivs(sky.alm_T)                          # [1][15][4097][8192]
    print("theta fft: lmax 4095 fp64 transform", flush=True)
    out = plan.theta_derivs(D[0, :order], order)              # [4][4][4097][8192]
    torch.cuda.synchronize()
    pairs = _jk(order)
    rings = np.array([0, 1, 5, 197, 1024, 2048, 3899, 4095, 4096])
    ref = oracle_scaled_derivs(oracle, lmax, order, ntheta, nphi, rings, sky.alm_T)
    for k in range(order):
        for j in range(1, order - k + 1):
            q = pairs.index((j, k))
            scale = float(D[0, q].abs().max())
            d = float((out[k, j - 1] - D[0, q]).abs().max())
            assert d < 1e-10 * scale, (j, k, d / scale)
            got = t2np(out[k, j - 1][torch.as_tensor(rings, device=out.device)])
            assert np.max(np.abs(got - ref[0, q])) < 1e-10 * np.max(np.abs(ref[0, q])), (j, k)
    del D, out, plan
    torch.cuda.empty_cache()

    plan32 = tl.Plan(lmax, ntheta, nphi, 1, "fp32", pol=False)
    g = torch.Generator().manual_seed(4097)
    maps = torch.randn((2, ntheta, nphi), generator=g, dtype=torch.float32)
    print("theta fft: lmax 4095 fp32 transform", flush=True)
    out32 = t2np(plan32.theta_derivs(maps.cuda(), 4))
    cols = [0, 1, 2, 1023, 2047, 4094, 4095]
    m64 = maps.double().numpy()
    want = oracle.theta_derivs_fft(m64, 4, cols=cols)
    got = np.concatenate([out32[..., cols], out32[..., [c + nphi // 2 for c in cols]]], axis=-1)
    amax = np.max(np.abs(m64))
    assert np.all(np.abs(got - want) <= 2.0 ** -24 * np.abs(want) + 1e-12 * amax)


def test_theta_derivs_argument_errors(tl):
    L = tl.lib()
    x = torch.zeros((2, 65, 150), dtype=torch.float32, device="cuda")
    y = torch.zeros((2, 4, 65, 150), dtype=torch.float32, device="cuda")
    good = tl.Plan(60, 65, 150, 1, "fp32", pol=False)
    vp = ctypes.c_void_p
    call = lambda plan, a, n, j, b: L.tl_theta_derivs(plan._h, vp(a), n, j, vp(b))
    assert call(good, x.data_ptr(), 0, 4, y.data_ptr()) == 0
    assert call(good, x.data_ptr(), 2, 0, y.data_ptr()) == -1
    assert call(good, x.data_ptr(), 2, 9, y.data_ptr()) == -1
    assert call(good, x.data_ptr(), -1, 4, y.data_ptr()) == -1
    assert call(good, None, 2, 4, y.data_ptr()) == -1
    assert call(good, x.data_ptr() + 4, 2, 4, y.data_ptr()) == -1   # not aligned to two values
    assert L.tl_theta_derivs(None, vp(x.data_ptr()), 2, 4, vp(y.data_ptr())) == -1
    odd = tl.Plan(60, 66, 150, 1, "fp32", pol=False)                # ntheta - 1 = 65
    assert call(odd, x.data_ptr(), 1, 1, y.data_ptr()) == -2
    high = tl.Plan(64, 65, 150, 1, "fp32", pol=False)               # lmax > ntheta - 2
    assert call(high, x.data_ptr(), 1, 1, y.data_ptr()) == -2
    hpx = tl.Plan(16, 0, 0, 1, "fp32", pol=False, nside=8)
    assert call(hpx, x.data_ptr(), 1, 1, y.data_ptr()) == -2
    torch.cuda.synchronize()
    assert float(y.abs().max()) == 0.0                               # nothing ran


def _sky_b(lmax, seed, ntheta, rms_pix=1.2):
    sky = skygen.make_sky(lmax, seed, pol=True, rms_arcmin=rms_pix * (math.pi / (ntheta - 1)) / skygen.ARCMIN)
    sky.alm_B = skygen.random_alm(lmax, seed + 1000, lmin=2) * 0.2
    return sky


def _check_lens(got, ref, tol_rms, tol_max):
    mask = ref["_tie"] > 1e-9
    assert np.mean(~mask) < 1e-3
    for f, g in zip("TQU", got):
        assert rel_rms(t2np(g), ref[f], mask) < tol_rms, f
        assert max_rel(t2np(g), ref[f], mask) < tol_max, f


@pytest.mark.parametrize("lmax,ntheta,nphi,order", [(60, 65, 150, 4), (127, 129, 256, 4), (100, 129, 256, 1),
                                                    (100, 129, 256, 6)])
def test_theta_fft_plan_against_the_oracle_and_the_recursion(tl, oracle, lmax, ntheta, nphi, order):
    sky = _sky_b(lmax, 31, ntheta)
    a = (sky.alm_T, sky.alm_E, sky.alm_B)
    pt = tl.Plan(lmax, ntheta, nphi, order, "fp64", pol=True, theta_fft=True)
    pr = tl.Plan(lmax, ntheta, nphi, order, "fp64", pol=True)
    print("theta_fft plan", lmax, ntheta, nphi, order, flush=True)
    Dt, Dr = t2np(pt.synth_derivs(*a)), t2np(pr.synth_derivs(*a))
    ref = oracle_scaled_derivs(oracle, lmax, order, ntheta, nphi, np.arange(ntheta), *a)
    for f in range(3):
        for q in range(ref.shape[1]):
            s = np.max(np.abs(ref[f, q]))
            assert np.max(np.abs(Dt[f, q] - ref[f, q])) < 1e-11 * s, (f, q)
            assert np.max(np.abs(Dt[f, q] - Dr[f, q])) < 1e-11 * s, (f, q)
    mt = pt.lens_map(*a, sky.alm_phi)
    mr = pr.lens_map(*a, sky.alm_phi)
    for x, y in zip(mt, mr):
        assert rel_rms(t2np(x), t2np(y)) < 1e-12 and max_rel(t2np(x), t2np(y)) < 1e-11
    if (lmax, order) == (127, 4):
        ref = oracle.lens_map(lmax, order, ntheta, nphi, *a, sky.alm_phi, nthreads=ORACLE_THREADS)
        _check_lens(mt, ref, 1e-12, 1e-11)
    # several realizations: bit-identical to single calls
    sky2 = _sky_b(lmax, 32, ntheta)
    many = pt.lens_map_many([(*a, sky.alm_phi), (sky2.alm_T, sky2.alm_E, sky2.alm_B, sky2.alm_phi)])
    single2 = pt.lens_map(sky2.alm_T, sky2.alm_E, sky2.alm_B, sky2.alm_phi)
    for x, y in zip(many[0], mt):
        assert torch.equal(x, y)
    for x, y in zip(many[1], single2):
        assert torch.equal(x, y)


def test_theta_fft_plan_at_the_lmax4095_grid(tl, oracle):
    """T+Q/U lmax 4095 on 4097 x 8192 rings (the largest circle), order 4,
    FP64 with theta_fft: the whole lensed maps against the plan without the
    option, sampled rings (poles, cap edge, belt) against the oracle."""
    lmax, ntheta, nphi, order = 4095, 4097, 8192, 4
    sky = skygen.make_sky(lmax, 41, pol=True)
    a = (sky.alm_T, sky.alm_E, sky.alm_B, sky.alm_phi)
    print("theta_fft plan lmax 4095", flush=True)
    pt = tl.Plan(lmax, ntheta, nphi, order, "fp64", pol=True, theta_fft=True)
    mt = pt.lens_map(*a)
    del pt
    pr = tl.Plan(lmax, ntheta, nphi, order, "fp64", pol=True)
    mr = pr.lens_map(*a)
    del pr
    for x, y in zip(mt, mr):
        d = float(torch.sqrt(torch.mean((x - y) ** 2)) / torch.sqrt(torch.mean(y ** 2)))
        assert d < 1e-11, d
    # the FP64 bar of the derivative maps above lmax 2048, 1e-11 (lmax / 2048)^2
    rings = np.array([0, 2, 197, 1500, 2048, 3899, 4096])
    ref = oracle.lens_rings(lmax, order, ntheta, nphi, rings, *a, nthreads=ORACLE_THREADS)
    _check_lens([t2np(g)[rings] for g in mt], ref, 4e-11, 4e-10)
