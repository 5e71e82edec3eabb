"""Reduced-precision forms of the harmonic stage (tabulated lambda/lambda' on
MFMA) and the many-realization entry point, against the oracle (marked gpu).

Each form is checked at the harmonic stage (relative RMS per (field, j)
block) and on whole maps (relative RMS per field); the tolerances are the
ones each form is stated to meet (maps; harmonic-stage blocks in brackets):
    fp16x2 (hi + lo FP16, 22-bit operands)   1e-5   [1e-4]
    bf16x3 (hi + lo BF16, 16-bit operands)   3e-5   [1.5e-4]
    fp16 (power-of-two scaled)               1e-3   [1e-2]
    bf16                                     1e-2   [5e-2]
Only fp16 and the split forms meet the 1e-3 bar of the fastest form; bf16
does not (about 5e-3 on maps).
"""
import math

import numpy as np
import pytest
import torch

from paper_1307_0719_amd import skygen
from tests.gpu_util import ORACLE_THREADS, need_gpu, rel_rms, smooth_nphi, t2np

pytestmark = pytest.mark.gpu

MAP_TOL = {"fp32": 1e-5, "bf16x3": 3e-5, "fp16x2": 1e-5, "fp16": 1e-3, "bf16": 1e-2}
STAGE_TOL = {"bf16x3": 1.5e-4, "fp16x2": 1e-4, "fp16": 1e-2, "bf16": 5e-2}


@pytest.fixture(scope="module")
def tl():
    need_gpu()
    from paper_1307_0719_amd import taylens

    taylens.lib()
    return taylens


def _sky(lmax, seed, with_b=False, rms_pix=None, ntheta=None):
    rms = skygen.DEFLECTION_RMS_ARCMIN
    if rms_pix is not None:
        rms = rms_pix * (math.pi / (ntheta - 1)) / skygen.ARCMIN
    sky = skygen.make_sky(lmax, seed, rms_arcmin=rms)
    if with_b:
        sky.alm_B = skygen.random_alm(lmax, seed + 1000, lmin=2) * 0.2
    return sky


@pytest.mark.parametrize("precision", ["bf16x3", "fp16x2", "fp16", "bf16"])
@pytest.mark.parametrize("lmax,ntheta,order,with_b", [(130, 131, 4, True), (300, 301, 2, False), (64, 97, 6, False)])
def test_tab_legendre_stage(tl, oracle, precision, lmax, ntheta, order, with_b):
    nphi = smooth_nphi(2 * lmax + 2)
    sky = _sky(lmax, 81, with_b=with_b)
    plan = tl.Plan(lmax, ntheta, nphi, order, precision, pol=True)
    F = t2np(plan.legendre(sky.alm_T, sky.alm_E, sky.alm_B))
    ref = oracle.ring_coeffs(lmax, order, oracle.grid_theta(ntheta), sky.alm_T, sky.alm_E, sky.alm_B,
                             ORACLE_THREADS)
    errs = []
    for f, name in enumerate(("T", "Q", "U")):
        for j in range(order + 1):
            want = ref[name][:, j, :]
            scale = np.sqrt(np.mean(np.abs(want) ** 2))
            errs.append((float(np.sqrt(np.mean(np.abs(F[f, j] - want) ** 2)) / scale), name, j))
    errs.sort(reverse=True)
    print(precision, lmax, order, "worst stage rel RMS", errs[:3])
    assert errs[0][0] < STAGE_TOL[precision], errs[:4]


@pytest.mark.parametrize("precision", ["bf16x3", "fp16x2", "fp16", "bf16"])
def test_tab_lens_map(tl, oracle, precision):
    lmax, ntheta, nphi, order = 160, 161, 320, 4
    sky = _sky(lmax, 83, with_b=True, rms_pix=1.3, ntheta=ntheta)
    plan = tl.Plan(lmax, ntheta, nphi, order, precision, pol=True)
    got = plan.lens_map(sky.alm_T, sky.alm_E, sky.alm_B, sky.alm_phi)
    ref = oracle.lens_map(lmax, order, ntheta, nphi, sky.alm_T, sky.alm_E, sky.alm_B, sky.alm_phi,
                          nthreads=ORACLE_THREADS)
    mask = ref["_tie"] > 1e-9
    errs = {f: rel_rms(t2np(g), ref[f], mask) for f, g in zip("TQU", got)}
    print(precision, "map rel RMS", errs)
    for f, e in errs.items():
        assert e < MAP_TOL[precision], (f, e)


@pytest.mark.parametrize("precision,batch", [("fp16", 3), ("bf16x3", 2), ("fp16", 4), ("bf16", 4), ("fp16x2", 6),
                                             ("bf16x3", 6), ("fp16", 6), ("bf16", 5)])
def test_lens_map_many_equals_single_calls(tl, precision, batch):
    """Realizations in one table pass give what single calls give, bit for
    bit; one more realization than the batch makes a second, smaller pass."""
    lmax, ntheta, nphi, order = 96, 97, 192, 4
    skies = [_sky(lmax, 90 + i) for i in range(batch + 1)]
    single = tl.Plan(lmax, ntheta, nphi, order, precision, pol=True)
    ref = [tuple(x.clone() for x in single.lens_map(s.alm_T, s.alm_E, None, s.alm_phi)) for s in skies]
    many = tl.Plan(lmax, ntheta, nphi, order, precision, pol=True, batch=batch)
    got = many.lens_map_many([(s.alm_T, s.alm_E, None, s.alm_phi) for s in skies])
    torch.cuda.synchronize()
    for a, b in zip(ref, got):
        for x, y in zip(a, b):
            assert torch.equal(x, y)


def test_tab_TP4096_fp16_sampled(tl, oracle):
    """The lmax=4096 T+Q/U order-4 workload in the FP16 form: sampled rings."""
    w = skygen.WORKLOADS["TP4096"]
    sky = skygen.make_sky(w.lmax, w.seed, pol=True)
    plan = tl.Plan(w.lmax, w.ntheta, w.nphi, w.order, "fp16", pol=True)
    got = [t2np(x) for x in plan.lens_map(sky.alm_T, sky.alm_E, None, sky.alm_phi)]
    rp = plan.query("rpole")
    rings = np.array([0, 3, rp - 1, rp, rp + 1, 400, 1500, 2048])
    ref = oracle.lens_rings(w.lmax, w.order, w.ntheta, w.nphi, rings, sky.alm_T, sky.alm_E, sky.alm_B,
                            sky.alm_phi, nthreads=ORACLE_THREADS)
    mask = ref["_tie"] > 1e-9
    errs = {f: rel_rms(g[rings], ref[f], mask) for f, g in zip("TQU", got)}
    print("fp16 lmax 4096 sampled rel RMS", errs)
    for f, e in errs.items():
        assert e < MAP_TOL["fp16"], (f, e)


@pytest.mark.parametrize("precision,batch", [("fp16", 1), ("bf16x3", 2), ("fp16", 4)])
def test_onthefly_engine_matches_oracle(tl, oracle, precision, batch, monkeypatch):
    """TAYLENS_ONTHEFLY=1: the same forms without tables, against the oracle
    (same bars) and against single calls (bit-exact)."""
    monkeypatch.setenv("TAYLENS_ONTHEFLY", "1")
    lmax, ntheta, nphi, order = 160, 161, 320, 4
    skies = [_sky(lmax, 130 + i, rms_pix=1.3, ntheta=ntheta) for i in range(batch)]
    plan = tl.Plan(lmax, ntheta, nphi, order, precision, pol=True, batch=batch)
    got = plan.lens_map_many([(s.alm_T, s.alm_E, None, s.alm_phi) for s in skies])
    torch.cuda.synchronize()
    s0 = skies[0]
    ref = oracle.lens_map(lmax, order, ntheta, nphi, s0.alm_T, s0.alm_E, None, s0.alm_phi, nthreads=ORACLE_THREADS)
    mask = ref["_tie"] > 1e-9
    errs = {f: rel_rms(t2np(g), ref[f], mask) for f, g in zip("TQU", got[0])}
    print(precision, batch, "on the fly, map rel RMS", errs)
    for f, e in errs.items():
        assert e < MAP_TOL[precision], (f, e)
    single = tl.Plan(lmax, ntheta, nphi, order, precision, pol=True)
    for s, g in zip(skies, got):
        one = single.lens_map(s.alm_T, s.alm_E, None, s.alm_phi)
        torch.cuda.synchronize()
        for x, y in zip(one, g):
            assert torch.equal(x, y)


def test_deflection_fold_policy(tl):
    """The split table forms carry the lensing potential in their table pass;
    the single-table forms and the FP32 form keep the FP64 deflection."""
    for prec, want in [("bf16x3", 1), ("fp16x2", 1), ("fp16", 0), ("bf16", 0), ("fp32", 0)]:
        plan = tl.Plan(96, 97, 192, 4, prec, pol=True)
        assert plan.query("defl_folded") == want, prec
        plan.close()



def test_polar_cap_policy(tl):
    """Ring pairs kept on the direct FP64 kernels: sin theta < 0.15 in every
    form and order but the split FP16 one, sin theta < 0.05 there; caps of 48
    ring pairs or more rounded to whole 64-lane waves (down when that gives
    up at most 1/16 of the cap, else up)."""
    def rpole(prec, order, lmax=160):
        plan = tl.Plan(lmax, lmax + 1, 2 * lmax, order, prec, pol=True)
        r = plan.query("rpole")
        plan.close()
        return r

    # sin(pi r / 160) < 0.15 for r < 8, < 0.05 for r < 3
    for prec in ("fp32", "fp16", "bf16", "bf16x3"):
        for order in (2, 4, 6):
            assert rpole(prec, order) == 8, (prec, order)
    for order in (2, 4, 6):
        assert rpole("fp16x2", order) == 3, order
    # lmax 4096 on 4097 rings: sin(pi r / 4096) < 0.05 for r < 66 -> 64;
    # < 0.15 for r < 197 -> 192; lmax 3000: < 0.15 for r < 144 -> 192
    assert rpole("fp16x2", 4, 4096) == 64
    assert rpole("fp16", 4, 4096) == 192
    assert rpole("fp32", 4, 3000) == 192


@pytest.mark.parametrize("precision,batch", [("fp16x2", 3), ("fp16", 2), ("fp16x2", 5)])
def test_lens_map_many_with_b(tl, oracle, precision, batch):
    """B modes present: the table pass carries T, E, B (and, split forms, the
    lensing potential) columns, the direct spin kernel two right-hand sides
    per realization.  Many vs single calls bit-identical; the first
    realization against the oracle at the form's map bar."""
    lmax, ntheta, nphi, order = 96, 97, 192, 4
    skies = [_sky(lmax, 140 + i, with_b=True, rms_pix=1.0, ntheta=ntheta) for i in range(batch)]
    single = tl.Plan(lmax, ntheta, nphi, order, precision, pol=True)
    ref = [tuple(x.clone() for x in single.lens_map(s.alm_T, s.alm_E, s.alm_B, s.alm_phi)) for s in skies]
    many = tl.Plan(lmax, ntheta, nphi, order, precision, pol=True, batch=batch)
    got = many.lens_map_many([(s.alm_T, s.alm_E, s.alm_B, s.alm_phi) for s in skies])
    torch.cuda.synchronize()
    for a, b in zip(ref, got):
        for x, y in zip(a, b):
            assert torch.equal(x, y)
    s0 = skies[0]
    o = oracle.lens_map(lmax, order, ntheta, nphi, s0.alm_T, s0.alm_E, s0.alm_B, s0.alm_phi, nthreads=ORACLE_THREADS)
    mask = o["_tie"] > 1e-9
    errs = {f: rel_rms(t2np(g), o[f], mask) for f, g in zip("TQU", got[0])}
    print(precision, batch, "with B, map rel RMS", errs)
    for f, e in errs.items():
        assert e < MAP_TOL[precision], (f, e)


# ------------------------------------------------ FP16 derivative maps --

def test_maps16_on_a_damped_sky(tl, oracle):
    """maps16 (D_jk with j + k >= 3 in FP16) on the lmax 2048 workload, whose
    power falls off well before the band limit: sampled rings at the FP32
    form's bar, in the FP32 and split FP16 forms, orders 3 and 5."""
    w = skygen.WORKLOADS["TP2048"]
    sky = skygen.make_sky(w.lmax, w.seed, pol=True)
    rings = np.array([0, 2, 40, 700, 1024, 2046])
    for order in (3, 5):
        ref = oracle.lens_rings(w.lmax, order, w.ntheta, w.nphi, rings, sky.alm_T, sky.alm_E, sky.alm_B,
                                sky.alm_phi, nthreads=ORACLE_THREADS)
        mask = ref["_tie"] > 1e-9
        for prec in ("fp32", "fp16x2"):
            plan = tl.Plan(w.lmax, w.ntheta, w.nphi, order, prec, pol=True, maps16=True)
            got = [t2np(x)[rings] for x in plan.lens_map(sky.alm_T, sky.alm_E, None, sky.alm_phi)]
            plan.close()
            for f, g in zip("TQU", got):
                e = rel_rms(g, ref[f], mask)
                print("maps16", prec, order, f, f"{e:.2e}")
                assert e < MAP_TOL[prec], (prec, order, f, e)


def test_maps16_with_power_at_the_band_limit(tl, oracle):
    """The documented limit of maps16: a sky with its power up to the grid's
    band limit (lmax 128 on 129 x 256 rings, deflection 1.2 pixels RMS) makes
    the third-order Taylor terms a sizable part of the field, and their FP16
    rounding shows (the plain form stays at its bar)."""
    lmax, ntheta, nphi, order = 128, 129, 256, 4
    spacing = math.pi / (ntheta - 1)
    sky = skygen.make_sky(lmax, 17, pol=True, rms_arcmin=1.2 * spacing / skygen.ARCMIN)
    ref = oracle.lens_map(lmax, order, ntheta, nphi, sky.alm_T, sky.alm_E, None, sky.alm_phi,
                          nthreads=ORACLE_THREADS)
    mask = ref["_tie"] > 1e-9
    errs = {}
    for m16 in (False, True):
        plan = tl.Plan(lmax, ntheta, nphi, order, "fp32", pol=True, maps16=m16)
        got = plan.lens_map(sky.alm_T, sky.alm_E, None, sky.alm_phi)
        errs[m16] = max(rel_rms(t2np(g), ref[f], mask) for f, g in zip("TQU", got))
        plan.close()
    print("band-limit sky, worst field rel RMS: plain %.2e, maps16 %.2e" % (errs[False], errs[True]))
    assert errs[False] < 1e-5
    assert errs[False] < errs[True] < 1e-3


def test_maps16_is_ignored_where_it_does_not_apply(tl):
    """FP64 plans, orders below 3 and HEALPix plans keep FP32/FP64 maps:
    maps16 changes nothing there (bit for bit)."""
    sky = skygen.make_sky(32, 5, pol=True)
    cases = [dict(lmax=32, ntheta=33, nphi=64, order=4, precision="fp64"),
             dict(lmax=32, ntheta=33, nphi=64, order=2, precision="fp32"),
             dict(lmax=32, ntheta=0, nphi=0, order=4, precision="fp32", nside=16)]
    for c in cases:
        outs = []
        for m16 in (False, True):
            plan = tl.Plan(c["lmax"], c["ntheta"], c["nphi"], c["order"], c["precision"], pol=True,
                           nside=c.get("nside", 0), maps16=m16)
            outs.append([x.clone() for x in plan.lens_map(sky.alm_T, sky.alm_E, None, sky.alm_phi)])
            plan.close()
        for x, y in zip(*outs):
            assert torch.equal(x, y), c


def test_paired_fp16_maps_across_table_passes(tl, oracle):
    """maps16 on rings of 1024 points (paired FP16 planes, the radix-16
    FFT at M = 512) with seven realizations on a plan of six per pass: the
    second set of maps and the second stream alternate across the two passes.
    Every realization equals a single call on the same plan bit for bit, and
    the first and last match the oracle within 3e-5 (storing the maps of
    order >= 3 in FP16 costs 5-6e-6 on this sky, one-pixel deflections, by a
    CPU estimate with the oracle's maps rounded to FP16)."""
    lmax, ntheta, nphi, order = 300, 301, 1024, 4
    skies = [_sky(lmax, 300 + i, rms_pix=1.0, ntheta=ntheta) for i in range(7)]
    plan = tl.Plan(lmax, ntheta, nphi, order, "fp16x2", pol=True, batch=6, maps16=True)
    got = [tuple(x.clone() for x in o) for o in plan.lens_map_many([(s.alm_T, s.alm_E, None, s.alm_phi)
                                                                    for s in skies])]
    single = [tuple(x.clone() for x in plan.lens_map(s.alm_T, s.alm_E, None, s.alm_phi)) for s in skies]
    torch.cuda.synchronize()
    for a, b in zip(got, single):
        for x, y in zip(a, b):
            assert torch.equal(x, y)
    for i in (0, 6):
        s = skies[i]
        ref = oracle.lens_map(lmax, order, ntheta, nphi, s.alm_T, s.alm_E, None, s.alm_phi, nthreads=ORACLE_THREADS)
        mask = ref["_tie"] > 1e-9
        for f, g in zip("TQU", got[i]):
            e = rel_rms(t2np(g), ref[f], mask)
            print("paired maps16", i, f, f"{e:.2e}")
            assert e < 3e-5, (i, f, e)
    plan.close()


def test_lens_map_many_replays_from_a_hip_graph(tl):
    """tl_lens_map_many captured in a HIP graph on the plan's stream (its
    second stream joins the capture through the call's events) and replayed
    three times, with eager calls and synchronizations between the replays:
    every replay reproduces the eager result bit for bit.  Four realizations
    on a plan of three per pass (two passes), paired FP16 planes."""
    dev = torch.device("cuda", 0)
    lmax, ntheta, nphi, order = 96, 97, 1024, 4
    skies = [_sky(lmax, 500 + i) for i in range(5)]
    to = lambda a: None if a is None else torch.from_numpy(a).to(dev)
    alms = [(to(s.alm_T), to(s.alm_E), None, to(s.alm_phi)) for s in skies[:4]]
    other = (to(skies[4].alm_T), to(skies[4].alm_E), None, to(skies[4].alm_phi))
    st = torch.cuda.Stream(dev)
    plan = tl.Plan(lmax, ntheta, nphi, order, "fp16x2", pol=True, batch=3, maps16=True, stream=st)
    mk = lambda: [tuple(torch.empty((ntheta, nphi), dtype=torch.float32, device=dev) for _ in range(3))
                  for _ in alms]
    eager, outs = mk(), mk()
    with torch.cuda.stream(st):
        plan.lens_map_many(alms, eager)
        plan.lens_map_many(alms, outs)  # warm-up before the capture
    st.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=st):
        plan.lens_map_many(alms, outs)
    for rep in range(3):
        for o in outs:
            for t in o:
                t.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for a, b in zip(eager, outs):
            for x, y in zip(a, b):
                assert torch.equal(x, y), rep
        with torch.cuda.stream(st):  # eager work of the same plan between the replays
            plan.lens_map(*other)
        st.synchronize()
    plan.close()
