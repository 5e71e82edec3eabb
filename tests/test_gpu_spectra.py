"""Analysis of temperature maps (tl_analysis_T) and the lensed-spectrum
accuracy measure of Sec. III.A-B against the oracle (step 9), through the C
ABI (marked gpu).

* Kernel parity: a_lm of arbitrary maps equal the oracle's quadrature on the
  same values to 1e-11 of the largest coefficient (FP64 recursions of
  different order of summation; the scaled start values near the poles
  agree to ~1e-13 relative), on grids with even and odd ring counts, the
  smallest grids (2 and 3 rings) and plans of several forms.
* Round trip: the library's own unlensed maps of band limit L analysed at
  lmax = L with L + lmax <= ntheta - 1 and L + lmax < nphi give back their
  a_lm (lmax 1024 on 2049 x 4096 rings and lmax 2048 on 4097 x 8192 rings).
* Spectrum measure: for lensed maps of the FP32 form at orders 0 and 2
  against an FP64 order-8 reference, the binned relative errors and l* from
  the library's a_lm equal those from the oracle's analysis of the same maps.
"""
import ctypes
import math

import numpy as np
import pytest
import torch

from paper_1307_0719_amd import skygen
from tests.gpu_util import need_gpu, t2np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tl():
    need_gpu()
    from paper_1307_0719_amd import taylens

    taylens.lib()
    return taylens


@pytest.mark.parametrize("lmax,ntheta,nphi,precision,order,pol", [
    (16, 33, 32, "fp64", 1, False), (10, 12, 32, "fp32", 1, True), (8, 2, 16, "fp64", 0, False),
    (5, 3, 16, "fp64", 0, False), (64, 129, 128, "fp64", 2, False), (100, 97, 256, "fp64", 1, False),
    (200, 401, 512, "fp32", 4, False)])
def test_analysis_matches_the_oracle(tl, oracle, lmax, ntheta, nphi, precision, order, pol):
    plan = tl.Plan(lmax, ntheta, nphi, order, precision, pol=pol)
    T = np.random.default_rng(lmax * 1000 + ntheta).standard_normal((ntheta, nphi))
    print("analysis", lmax, ntheta, nphi, precision, flush=True)
    got = t2np(plan.analysis_T(torch.from_numpy(T).cuda()))
    want = oracle.analysis_T(T, lmax)
    assert np.max(np.abs(got - want)) < 1e-11 * np.max(np.abs(want))


@pytest.mark.parametrize("lmax,ntheta,nphi", [(1024, 2049, 4096), (2048, 4097, 8192)])
def test_analysis_round_trip(tl, lmax, ntheta, nphi):
    sky = skygen.make_sky(lmax, 5, pol=False)
    plan = tl.Plan(lmax, ntheta, nphi, 1, "fp64", pol=False)
    print("analysis round trip", lmax, ntheta, nphi, flush=True)
    T, _, _ = plan.lens_map(sky.alm_T, None, None, None)
    got = t2np(plan.analysis_T(T))
    want = sky.alm_T.copy()
    want[:lmax + 1] = want[:lmax + 1].real
    assert np.max(np.abs(got - want)) < 1e-11 * np.max(np.abs(want))


def test_analysis_argument_errors(tl):
    L = tl.lib()
    vp = ctypes.c_void_p
    m = torch.zeros((33, 32), dtype=torch.float64, device="cuda")
    a = torch.zeros(17 * 18 // 2 + 1, dtype=torch.complex128, device="cuda")
    good = tl.Plan(16, 33, 32, 1, "fp64", pol=False)
    assert L.tl_analysis_T(good._h, None, vp(a.data_ptr())) == -1
    assert L.tl_analysis_T(good._h, vp(m.data_ptr()), None) == -1
    assert L.tl_analysis_T(good._h, vp(m.data_ptr()), vp(a.data_ptr() + 8)) == -1
    assert L.tl_analysis_T(None, vp(m.data_ptr()), vp(a.data_ptr())) == -1
    assert L.tl_analysis_T(tl.Plan(16, 33, 48, 1, "fp64", pol=False)._h, vp(m.data_ptr()), vp(a.data_ptr())) == -2
    assert L.tl_analysis_T(tl.Plan(16, 33, 32, 0, "fp32", pol=False)._h, vp(m.data_ptr()), vp(a.data_ptr())) == -2
    assert L.tl_analysis_T(tl.Plan(16, 0, 0, 1, "fp64", pol=False, nside=8)._h, vp(m.data_ptr()),
                           vp(a.data_ptr())) == -2
    torch.cuda.synchronize()
    assert float(a.abs().max()) == 0.0


def test_spectrum_accuracy_measure_matches_the_oracle(tl, oracle):
    lmax, ntheta, nphi = 150, 301, 512
    ana = tl.Plan(lmax, ntheta, nphi, 1, "fp64", pol=False)
    ref_plan = tl.Plan(lmax, ntheta, nphi, 8, "fp64", pol=False)
    plans = {N: tl.Plan(lmax, ntheta, nphi, N, "fp32", pol=False) for N in (0, 2)}
    errs_gpu = {N: [] for N in plans}
    errs_cpu = {N: [] for N in plans}
    for seed in (3, 4):
        sky = skygen.make_sky(lmax, seed, pol=False, rms_arcmin=2.0 * (math.pi / (ntheta - 1)) / skygen.ARCMIN)
        ref = ref_plan.lens_map(sky.alm_T, None, None, sky.alm_phi)[0]
        c_ref = oracle.cl_from_alm(t2np(ana.analysis_T(ref)), lmax)
        c_ref_o = oracle.cl_from_alm(oracle.analysis_T(t2np(ref), lmax), lmax)
        _, b_ref = oracle.bin_cl(c_ref)
        _, b_ref_o = oracle.bin_cl(c_ref_o)
        for N, p in plans.items():
            T = p.lens_map(sky.alm_T, None, None, sky.alm_phi)[0].double()
            cen, b = oracle.bin_cl(oracle.cl_from_alm(t2np(ana.analysis_T(T)), lmax))
            _, bo = oracle.bin_cl(oracle.cl_from_alm(oracle.analysis_T(t2np(T), lmax), lmax))
            errs_gpu[N].append(b / b_ref - 1)
            errs_cpu[N].append(bo / b_ref_o - 1)
    for N in plans:
        np.testing.assert_allclose(errs_gpu[N], errs_cpu[N], rtol=0, atol=1e-10)
        assert oracle.ell_star(cen, errs_gpu[N]) == oracle.ell_star(cen, errs_cpu[N])
    # order 2 is more accurate than order 0 overall and in the last bin
    e0, e2 = np.abs(np.mean(errs_gpu[0], axis=0)), np.abs(np.mean(errs_gpu[2], axis=0))
    assert e2.sum() < e0.sum() and e2[-1] < e0[-1]
