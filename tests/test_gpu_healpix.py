"""Lensing on HEALPix rings (marked gpu): the HIP path against the HEALPix
oracle (the paper's own pixelization, Sec. II.A-B).

Stages: the deflection at the pixel centres and the scaled derivative maps
(ring syntheses that fold the band limit onto each ring's pixel count and
phase) in FP64; then whole maps (positions, the pixel containing x', the
Taylor series about its centre, rotation) in every precision form at small
nside, with lmax from nside to 3 nside (polar rings of 4, 8, ... pixels far
below the band limit), with B modes, naive positions, zero deflection and
caller positions; then nside 2048 at full size on sampled rings (lmax 4096,
order 3 in the FP32 form; lmax 3072, order 2 on split FP16 tables, six
realizations per pass).
Bars as on the equal-theta grid: FP64 1e-11 (1e-10 on the maximum),
FP32 and split FP16 1e-5, FP16 1e-3 (relative RMS per field)."""
import math

import numpy as np
import pytest
import torch

from oracle import healpix_oracle as hp
from paper_1307_0719_amd import skygen
from tests.gpu_util import ORACLE_THREADS, max_rel, need_gpu, rel_rms, t2np

pytestmark = pytest.mark.gpu

TOL = {"fp64": (1e-11, 1e-10), "fp32": (1e-5, 1e-4), "fp16x2": (1e-5, 1e-4), "fp16": (1e-3, 1e-2)}


@pytest.fixture(scope="module")
def tl():
    need_gpu()
    from paper_1307_0719_amd import taylens

    taylens.lib()
    return taylens


def _sky(lmax, nside, seed, rms_pix=1.3, with_b=True):
    spacing = math.sqrt(4 * math.pi / hp.npix(nside))
    sky = skygen.make_sky(lmax, seed, pol=True, rms_arcmin=rms_pix * spacing / skygen.ARCMIN)
    if with_b:
        sky.alm_B = skygen.random_alm(lmax, seed + 1000, lmin=2) * 0.2
    return sky


@pytest.mark.parametrize("nside,lmax", [(1, 4), (2, 6), (8, 24), (32, 64), (64, 128)])
def test_healpix_deflection_and_derivative_maps(tl, nside, lmax):
    order = 4
    sky = _sky(lmax, nside, 11)
    plan = tl.Plan(lmax, 0, 0, order, "fp64", pol=True, nside=nside)
    at, ap = plan.deflection(sky.alm_phi)
    pix = np.arange(hp.npix(nside))
    ot, op = hp.deflection_pixels(lmax, sky.alm_phi, nside, pix, ORACLE_THREADS)
    assert max_rel(t2np(at), ot) < 1e-11 and max_rel(t2np(ap), op) < 1e-11
    D = t2np(plan.synth_derivs(sky.alm_T, sky.alm_E, sky.alm_B))
    ref = hp.derivative_pixels(lmax, order, nside, pix, sky.alm_T, sky.alm_E, sky.alm_B, ORACLE_THREADS)
    delta = math.pi / (4 * nside)
    for f, name in enumerate("TQU"):
        for q, (j, k) in enumerate([(j, k) for j in range(order + 1) for k in range(order + 1 - j)]):
            want = ref[name][(j, k)] * delta ** (j + k) / (math.factorial(j) * math.factorial(k))
            if np.max(np.abs(want)) == 0:
                assert np.max(np.abs(D[f, q])) == 0
                continue
            assert max_rel(D[f, q], want) < 1e-10, (name, j, k)


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16x2", "fp16"])
@pytest.mark.parametrize("nside,lmax,order", [(16, 32, 3), (32, 96, 4), (48, 96, 5)])
def test_healpix_lens_map_whole(tl, precision, nside, lmax, order):
    sky = _sky(lmax, nside, 21 + nside)
    plan = tl.Plan(lmax, 0, 0, order, precision, pol=True, nside=nside)
    got = plan.lens_map(sky.alm_T, sky.alm_E, sky.alm_B, sky.alm_phi)
    ref = hp.lens_map(lmax, order, nside, sky.alm_T, sky.alm_E, sky.alm_B, sky.alm_phi, nthreads=ORACLE_THREADS)
    # the pixel containing x' is ambiguous within rounding of a pixel edge:
    # skip pixels whose source pixel differs under a 1e-12 nudge of x'
    nudged = hp.ang2pix(nside, ref["_thp"] + 1e-12, ref["_php"] + 1e-12)
    ok = nudged == ref["_src"]
    assert np.mean(~ok) < 1e-3
    tr, tm = TOL[precision]
    for name, g in zip("TQU", got):
        e1, e2 = rel_rms(t2np(g), ref[name], ok), max_rel(t2np(g), ref[name], ok)
        print(precision, nside, lmax, order, name, f"{e1:.2e} {e2:.2e}")
        assert e1 < tr and e2 < tm, (name, e1, e2)


def test_healpix_options_and_edge_cases(tl):
    nside, lmax, order = 8, 24, 3
    sky = _sky(lmax, nside, 31)
    pix = np.arange(hp.npix(nside))
    # zero deflection: the field at the centres
    plan = tl.Plan(lmax, 0, 0, order, "fp64", pol=True, nside=nside)
    got = plan.lens_map(sky.alm_T, sky.alm_E, sky.alm_B, None)
    ref = hp.lens_map(lmax, order, nside, sky.alm_T, sky.alm_E, sky.alm_B, None)
    for name, g in zip("TQU", got):
        assert max_rel(t2np(g), ref[name]) < 1e-12, name
    # naive positions, rotation off
    for naive, rotate in ((True, False), (False, False)):
        p2 = tl.Plan(lmax, 0, 0, order, "fp64", pol=True, nside=nside, naive_pos=naive, rotate=rotate)
        got = p2.lens_map(sky.alm_T, sky.alm_E, sky.alm_B, sky.alm_phi)
        ref = hp.lens_map(lmax, order, nside, sky.alm_T, sky.alm_E, sky.alm_B, sky.alm_phi, rotate=rotate,
                          naive=naive)
        for name, g in zip("TQU", got):
            assert max_rel(t2np(g), ref[name]) < 1e-10, (naive, rotate, name)
    # caller positions: a constant shift of every centre
    th, ph = hp.pix2ang(nside, pix)
    thp = np.clip(th + 0.3 * math.pi / (4 * nside), 0, math.pi)
    php = ph + 0.7 * math.pi / (4 * nside)
    got = plan.lens_map_pos(sky.alm_T, sky.alm_E, sky.alm_B, torch.from_numpy(thp), torch.from_numpy(php))
    src = hp.ang2pix(nside, thp, php)
    th0, ph0 = hp.pix2ang(nside, src)
    D = hp.derivative_pixels(lmax, order, nside, src, sky.alm_T, sky.alm_E, sky.alm_B)
    from oracle import taylens_oracle as tor
    dth, dph = thp - th0, np.angle(np.exp(1j * (php - ph0)))
    for name, g in zip("TQU", got):
        want = tor.taylor_sum(lambda j, k: D[name][(j, k)], dth, dph, order)
        assert max_rel(t2np(g), want) < 1e-10, name
    # T only
    pT = tl.Plan(lmax, 0, 0, order, "fp32", pol=False, nside=nside)
    T, _, _ = pT.lens_map(sky.alm_T, None, None, sky.alm_phi)
    ref = hp.lens_map(lmax, order, nside, sky.alm_T, None, None, sky.alm_phi)
    assert rel_rms(t2np(T), ref["T"]) < 1e-5


def test_healpix_refusals(tl):
    with pytest.raises(tl.TaylensError) as e:
        tl.Plan(16, 0, 0, 3, "fp32", nside=0 - 1)
    assert e.value.code == tl.TL_ERR_INVALID
    with pytest.raises(tl.TaylensError) as e:
        tl.Plan(16, 0, 0, 3, "fp32", nside=4096)
    assert e.value.code == tl.TL_ERR_UNSUPPORTED
    p = tl.Plan(16, 0, 0, 4, "fp32", nside=4)
    with pytest.raises(tl.TaylensError) as e:
        tl.Batch([p, p])
    assert e.value.code == tl.TL_ERR_UNSUPPORTED


@pytest.mark.parametrize("nside,lmax,precision", [(256, 400, "fp64"), (256, 600, "fp64"), (256, 1100, "fp64"),
                                                   (512, 1536, "fp32"), (128, 300, "fp16x2")])
def test_healpix_ring_fft_classes(tl, nside, lmax, precision):
    """Every ring FFT class on sampled rings against the oracle: the belt of
    nside 256 and 512 (power-of-two length N = 4 nside; lmax below N / 2, up
    to N - 1 with the mirror term c_{N - m}, and lmax >= N, which folds more
    and takes the mixed-radix kernel), cap rings of smooth length (mixed
    radix) and of lengths with a large prime factor (Bluestein: 4 i pixels
    with i = 17, 37, 101, 127, 251, 509)."""
    order = 3
    dev = torch.device("cuda", 0)
    sky = _sky(lmax, nside, 41 + nside + lmax)
    plan = tl.Plan(lmax, 0, 0, order, precision, pol=True, nside=nside)
    got = plan.lens_map(*(torch.from_numpy(a).to(dev) if a is not None else None
                          for a in (sky.alm_T, sky.alm_E, sky.alm_B, sky.alm_phi)))
    torch.cuda.synchronize()
    caps = [i for i in (1, 2, 16, 17, 24, 37, 101, 127, 251, 509) if i < nside]
    rings = np.array(sorted(set([i - 1 for i in caps] + [4 * nside - 1 - i for i in caps[:4]]
                                + [nside - 1, nside, nside + 1, 2 * nside - 1, 3 * nside - 1])))
    pix = hp.ring_pixels(nside, rings)
    rows = [t2np(x[torch.from_numpy(pix).to(dev)]) for x in got]
    plan.close()
    ref = hp.lens_pixels(lmax, order, nside, pix, sky.alm_T, sky.alm_E, sky.alm_B, sky.alm_phi,
                         nthreads=ORACLE_THREADS)
    ok = hp.ang2pix(nside, ref["_thp"] + 1e-12, ref["_php"] + 1e-12) == ref["_src"]
    tr, tm = TOL[precision]
    for name, g in zip("TQU", rows):
        e1, e2 = rel_rms(g, ref[name], ok), max_rel(g, ref[name], ok)
        print(precision, nside, lmax, name, f"{e1:.2e} {e2:.2e}")
        assert e1 < tr and e2 < tm, (name, e1, e2)


@pytest.mark.parametrize("precision,lmax,order,batch", [("fp32", 4096, 3, 1), ("fp16x2", 3072, 2, 6)])
def test_healpix_nside2048_sampled_rings(tl, precision, lmax, order, batch):
    """nside 2048 at lmax 4096, order 3 (FP32 form) and at lmax 3072, order 2
    on split FP16 tables with six realizations per table pass (the launch the
    benchmark times; the first and last realization of the pass checked): rows of the paper's
    fastest-settings table at full size.  The split tables of lmax 4096 on
    8191 HEALPix rings take 258 GiB, too much beside six realizations' work
    buffers."""
    nside = 2048
    dev = torch.device("cuda", 0)
    skies = [skygen.make_sky(lmax, 2 + i, pol=True) for i in range(batch)]
    plan = tl.Plan(lmax, 0, 0, order, precision, pol=True, nside=nside, batch=batch if batch > 1 else 0)
    alms = [tuple(torch.from_numpy(a).to(dev) if a is not None else None
                  for a in (s.alm_T, s.alm_E, None, s.alm_phi)) for s in skies]
    outs = plan.lens_map_many(alms) if batch > 1 else [plan.lens_map(*alms[0])]
    torch.cuda.synchronize()
    # polar rings of 4 and 8 pixels, the cap rows next to the belt, the first
    # belt ring, mid-latitude, equator, the southmost ring
    rings = np.array([0, 1, 200, nside - 2, nside - 1, nside, 3 * nside // 2, 2 * nside - 1, 4 * nside - 2])
    pix = hp.ring_pixels(nside, rings)
    idx = torch.from_numpy(pix).to(dev)
    rows = [[t2np(x[idx]) for x in o] for o in outs]
    del outs, alms
    plan.close()
    torch.cuda.empty_cache()
    tr, tm = TOL[precision]
    for q in sorted({0, batch - 1}):
        s = skies[q]
        ref = hp.lens_pixels(lmax, order, nside, pix, s.alm_T, s.alm_E, s.alm_B, s.alm_phi,
                             nthreads=ORACLE_THREADS)
        ok = hp.ang2pix(nside, ref["_thp"] + 1e-12, ref["_php"] + 1e-12) == ref["_src"]
        for name, g in zip("TQU", rows[q]):
            e1, e2 = rel_rms(g, ref[name], ok), max_rel(g, ref[name], ok)
            print(precision, "nside 2048 realization", q, name, f"{e1:.2e} {e2:.2e}")
            assert e1 < tr and e2 < tm, (q, name, e1, e2)
