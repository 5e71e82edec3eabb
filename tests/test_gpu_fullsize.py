"""Parity at the full sizes of the named workloads, in the launch
configurations the benchmark times (marked gpu).

* T+Q/U, lmax 4096 on 4097 x 8192 rings, order 4, the split FP16 form with
  six realizations per table pass and FP16 derivative maps of order >= 3
  (tl_lens_map_many, seeds 2..7: the benchmark's headline step): every
  realization against the oracle;
* the same workload in the BF16 split and single BF16 forms;
* the uneven-lmax batch (persistent launch, graph, autotuner): one
  realization of every lmax, including lmax 3000 on 3001 x 6000 rings (a
  mixed-radix ring length), against the oracle.

The oracle computes sampled output rings one by one; the sample holds four
bands: both polar-cap boundaries (the four rings on each side of the first
ring pair the reduced forms take off the direct FP64 kernels), mid-latitude
and the equator.  Every band must meet the form's bar on its own (relative
RMS per field, pixels within 1e-9 pixel of a rounding tie excluded)."""
import math
import os

import numpy as np
import pytest
import torch

from paper_1307_0719_amd import skygen
from tests.gpu_util import ORACLE_THREADS, need_gpu, rel_rms, t2np

pytestmark = pytest.mark.gpu

MAP_TOL = {"fp32": 1e-5, "fp16x2": 1e-5, "bf16x3": 3e-5, "fp16": 1e-3, "bf16": 1e-2}
HEADLINE_BATCH = 6


@pytest.fixture(scope="module")
def tl():
    need_gpu()
    from paper_1307_0719_amd import taylens

    taylens.lib()
    return taylens


def sample_bands(ntheta, rpole):
    """Ring bands of the sample: north and south cap boundary, mid-latitude,
    equator."""
    north = np.arange(max(0, rpole - 4), min(ntheta, rpole + 4))
    return {"cap_edge_north": north, "cap_edge_south": np.sort(ntheta - 1 - north),
            "mid_latitude": np.array([ntheta // 4, ntheta // 4 + 1]),
            "equator": np.array([ntheta // 2 - 1, ntheta // 2])}


def check_bands(got_rows, ref, rings, bands, tol, label):
    """got_rows: [field][len(rings)][nphi] host arrays for the sampled rings."""
    mask = ref["_tie"] > 1e-9
    assert np.mean(~mask) < 1e-3
    worst = {}
    for bname, br in bands.items():
        sel = np.isin(rings, br)
        for f, g in zip("TQU", got_rows):
            e = rel_rms(g[sel][mask[sel]], ref[f][sel][mask[sel]])
            worst[(bname, f)] = e
    print(label, {f"{b}/{f}": f"{e:.2e}" for (b, f), e in worst.items()})
    bad = {k: v for k, v in worst.items() if not v < tol}
    assert not bad, (label, bad)
    return worst


def _to_dev(s, dev):
    return tuple(None if a is None else torch.from_numpy(a).to(dev) for a in (s.alm_T, s.alm_E, None, s.alm_phi))


@pytest.fixture(scope="module")
def headline(tl):
    """The benchmark's headline step: split FP16 tables, six realizations of
    the lmax 4096 workload per table pass, derivative maps of order >= 3 in
    FP16."""
    w = skygen.WORKLOADS["TP4096"]
    dev = torch.device("cuda", 0)
    skies = [skygen.make_sky(w.lmax, w.seed + i, pol=True) for i in range(HEADLINE_BATCH)]
    plan = tl.Plan(w.lmax, w.ntheta, w.nphi, w.order, "fp16x2", pol=True, batch=HEADLINE_BATCH, maps16=True)
    rpole = plan.query("rpole")
    bands = sample_bands(w.ntheta, rpole)
    rings = np.unique(np.concatenate(list(bands.values())))
    outs = plan.lens_map_many([_to_dev(s, dev) for s in skies])
    torch.cuda.synchronize()
    idx = torch.from_numpy(rings).to(dev)
    rows = [[t2np(x[idx]) for x in o] for o in outs]
    del outs
    plan.close()
    torch.cuda.empty_cache()
    return w, skies, rings, bands, rows


@pytest.mark.parametrize("q", range(HEADLINE_BATCH))
def test_headline_fp16x2_every_realization_of_the_pass(oracle, headline, q):
    w, skies, rings, bands, rows = headline
    s = skies[q]
    ref = oracle.lens_rings(w.lmax, w.order, w.ntheta, w.nphi, rings, s.alm_T, s.alm_E, s.alm_B, s.alm_phi,
                            nthreads=ORACLE_THREADS)
    check_bands(rows[q], ref, rings, bands, MAP_TOL["fp16x2"], f"fp16x2 x{HEADLINE_BATCH} realization {q}")


@pytest.mark.parametrize("precision", ["bf16x3", "bf16"])
def test_TP4096_bf16_forms(tl, oracle, precision):
    w = skygen.WORKLOADS["TP4096"]
    dev = torch.device("cuda", 0)
    s = skygen.make_sky(w.lmax, w.seed, pol=True)
    plan = tl.Plan(w.lmax, w.ntheta, w.nphi, w.order, precision, pol=True)
    bands = sample_bands(w.ntheta, plan.query("rpole"))
    rings = np.unique(np.concatenate(list(bands.values())))
    got = plan.lens_map(*_to_dev(s, dev))
    torch.cuda.synchronize()
    rows = [t2np(x[torch.from_numpy(rings).to(dev)]) for x in got]
    del got
    plan.close()
    torch.cuda.empty_cache()
    ref = oracle.lens_rings(w.lmax, w.order, w.ntheta, w.nphi, rings, s.alm_T, s.alm_E, s.alm_B, s.alm_phi,
                            nthreads=ORACLE_THREADS)
    check_bands(rows, ref, rings, bands, MAP_TOL[precision], f"{precision} lmax 4096")


def test_uneven_batch_against_the_oracle(tl, oracle, tmp_path):
    """One realization of every lmax of the uneven batch (FP32 form, one
    persistent harmonic launch, graph capture and replay, autotuned work
    items), sampled rings against the oracle; the replay must reproduce the
    captured run bit for bit."""
    os.environ["TAYLENS_TUNE_CACHE"] = str(tmp_path / "tune.txt")
    try:
        lmaxes = [512, 1024, 2048, 3000]
        dev = torch.device("cuda", 0)
        plans = [tl.Plan(L, L + 1, 2 * L, 4, "fp32", pol=True) for L in lmaxes]
        skies = [skygen.make_sky(L, 3000 + i, pol=True) for i, L in enumerate(lmaxes)]
        alms = [_to_dev(s, dev) for s in skies]
        b = tl.Batch(plans, autotune=True, use_graph=True)
        outs = b.outputs()
        b.run(alms, outs)
        torch.cuda.synchronize()
        first = [[x.clone() for x in o] for o in outs]
        b.run(alms, outs)     # graph replay
        torch.cuda.synchronize()
        assert b.info()["graph_replays"] == 1
        for o, f in zip(outs, first):
            for x, y in zip(o, f):
                assert torch.equal(x, y)
        for L, p, s, o in zip(lmaxes, plans, skies, outs):
            bands = sample_bands(L + 1, p.query("rpole"))
            bands["pole"] = np.array([0, 1, L - 1, L])
            rings = np.unique(np.concatenate(list(bands.values())))
            rows = [t2np(x[torch.from_numpy(rings).to(dev)]) for x in o]
            ref = oracle.lens_rings(L, 4, L + 1, 2 * L, rings, s.alm_T, s.alm_E, s.alm_B, s.alm_phi,
                                    nthreads=ORACLE_THREADS)
            check_bands(rows, ref, rings, bands, MAP_TOL["fp32"], f"batch lmax {L} on {L + 1}x{2 * L}")
        b.close()
    finally:
        del os.environ["TAYLENS_TUNE_CACHE"]
