"""The accuracy-vs-time sweep's measurement (marked gpu): the GPU's lensed
maps against the exact lensed field (the unlensed field synthesized at each
displaced position, rotated; oracle step 7), on two grid oversamplings and
orders 1..5.  The error falls with the order and with the oversampling, and
equals the Taylor oracle's own error against the exact field: what the sweep
reports is the truncation of the method, not a defect of the kernels."""
import math

import numpy as np
import pytest
import torch

from paper_1307_0719_amd import skygen
from tests.gpu_util import ORACLE_THREADS, need_gpu, t2np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tl():
    need_gpu()
    from paper_1307_0719_amd import taylens

    taylens.lib()
    return taylens


def _err(x, y):
    return float(np.sqrt(np.mean((x - y) ** 2)) / np.sqrt(np.mean(y ** 2)))


def test_errors_against_the_exact_lensed_field(tl, oracle):
    lmax = 96
    # deflection of one pixel RMS on the oversampling-1 grid: the orders separate
    sky = skygen.make_sky(lmax, 41, pol=True, rms_arcmin=(math.pi / lmax) / skygen.ARCMIN)
    rings = np.array([1, 9, 30, 48, 70, 94])
    cols = np.arange(0, 2 * lmax, 3)
    R, C = (a.ravel() for a in np.meshgrid(rings, cols, indexing="ij"))
    ex = oracle.exact_lensed_pixels(lmax, lmax + 1, 2 * lmax, R, C, sky.alm_T, sky.alm_E, None, sky.alm_phi,
                                    nthreads=ORACLE_THREADS)
    errs = {}
    for g in (1, 2):
        nt, nph = g * lmax + 1, 2 * g * lmax
        for order in range(1, 6):
            plan = tl.Plan(lmax, nt, nph, order, "fp32", pol=True)
            got = [t2np(x) for x in plan.lens_map(sky.alm_T, sky.alm_E, None, sky.alm_phi)]
            plan.close()
            e_gpu = max(_err(m[g * R, g * C], ex[f]) for f, m in zip("TQU", got))
            tay = oracle.lens_rings(lmax, order, nt, nph, g * rings, sky.alm_T, sky.alm_E, None, sky.alm_phi,
                                    nthreads=ORACLE_THREADS)
            pos = np.searchsorted(g * rings, g * R)
            e_tay = max(_err(tay[f][pos, g * C], ex[f]) for f in "TQU")
            print(f"g {g} order {order}: GPU {e_gpu:.3e}  Taylor oracle {e_tay:.3e}")
            assert abs(e_gpu - e_tay) <= 0.02 * e_tay + 2e-6, (g, order, e_gpu, e_tay)
            errs[(g, order)] = e_gpu
    for g in (1, 2):
        seq = [errs[(g, o)] for o in range(1, 6)]
        assert all(b < a for a, b in zip(seq, seq[1:])), (g, seq)
        assert seq[-1] < 0.02 * seq[0]
    for order in range(1, 6):
        assert errs[(2, order)] < errs[(1, order)]
