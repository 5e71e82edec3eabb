"""The allocation-free entry point (marked gpu): tl_lens_map_simple_noalloc
must give what tl_lens_map_simple gives (same kernels, so bit for bit; both
also within the FP32 form's 1e-5 bar of the oracle), on two calls in a row,
the second with a smaller input, with its workspace in the library's static
device array; a size beyond that array fails before any device work."""
import math

import numpy as np
import pytest
import torch

from paper_1307_0719_amd import skygen
from tests.gpu_util import ORACLE_THREADS, need_gpu, rel_rms, t2np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tl():
    need_gpu()
    from paper_1307_0719_amd import taylens

    taylens.lib()
    return taylens


def _case(lmax, ntheta, nphi, seed):
    pix = math.pi / (ntheta - 1) / skygen.ARCMIN
    sky = skygen.make_sky(lmax, seed, pol=True, rms_arcmin=1.3 * pix)
    sky.alm_B = skygen.random_alm(lmax, seed + 1, lmin=2) * 0.2
    return sky


def test_noalloc_matches_the_allocating_entry_point(tl, oracle):
    order = 4
    cases = [(128, 129, 256, 91), (40, 41, 80, 92)]   # second call smaller
    outs = [None, None]
    for i, (lmax, ntheta, nphi, seed) in enumerate(cases):
        s = _case(lmax, ntheta, nphi, seed)
        print(f"no-alloc call {i}: lmax {lmax}, {ntheta}x{nphi}, order {order}", flush=True)
        ref = tl.lens_map(s.alm_T, s.alm_E, s.alm_B, s.alm_phi, lmax, order, ntheta, nphi)
        out = tuple(torch.full((ntheta, nphi), float("nan"), device="cuda") for _ in range(3))
        got = tl.lens_map(s.alm_T, s.alm_E, s.alm_B, s.alm_phi, lmax, order, ntheta, nphi, out=out, noalloc=True)
        for g, r in zip(got, ref):
            assert torch.equal(g, r)
        o = oracle.lens_map(lmax, order, ntheta, nphi, s.alm_T, s.alm_E, s.alm_B, s.alm_phi,
                            nthreads=ORACLE_THREADS)
        mask = o["_tie"] > 1e-9
        for f, g in zip("TQU", got):
            assert rel_rms(t2np(g), o[f], mask) < 1e-5, f
        outs[i] = got
    # T only, after the polarized calls, through the same array
    s = _case(64, 65, 128, 93)
    ref = tl.lens_map(s.alm_T, None, None, s.alm_phi, 64, 3, 65, 128)
    got = tl.lens_map(s.alm_T, None, None, s.alm_phi, 64, 3, 65, 128, noalloc=True)
    assert torch.equal(got[0], ref[0])


def test_noalloc_rejects_a_workspace_beyond_its_array(tl):
    s = _case(1024, 1025, 2048, 94)
    with pytest.raises(tl.TaylensError) as e:
        tl.lens_map(s.alm_T, s.alm_E, None, s.alm_phi, 1024, 4, 1025, 2048, noalloc=True)
    assert e.value.code == tl.TL_ERR_NOMEM
    assert "static" in str(e.value)
