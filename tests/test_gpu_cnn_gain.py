"""What the trained correction gains over the plain order-2 Taylor sum
(marked gpu).  Both are measured against the method itself at order 6: the RMS of
(order 2 + correction - order 6) against that of (order 2 - order 6), over
every pixel of held-out skies (seeds 20000+, never used in training).

cnn_weights.npy was written by ``python -m paper_1307_0719_amd.train_cnn``
(200 realizations at lmax 2048, 20 Adam steps of 32768 pixels each); that
run measured a gain of about 7 at lmax 2048 and about 6 at lmax 4096.  The
thresholds below leave room for the non-deterministic order of the FP32
gradient sums of a retraining.  A second test trains from scratch on a
smaller grid to show the training itself works."""
import os

import numpy as np
import pytest

from tests.gpu_util import need_gpu

pytestmark = pytest.mark.gpu

WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1307_0719_amd",
                       "cnn_weights.npy")


@pytest.fixture(scope="module")
def tc():
    need_gpu()
    from paper_1307_0719_amd import train_cnn

    return train_cnn


@pytest.mark.parametrize("lmax,min_gain,seeds,precision", [(2048, 4.0, [20000, 20001, 20002], "fp32"),
                                                            (4096, 3.5, [20000, 20001], "fp32"),
                                                            (4096, 3.5, [20002], "fp16x2")])
def test_trained_network_gains_over_order2(tc, lmax, min_gain, seeds, precision):
    """Gain over plain order 2 on held-out seeds, in the FP32 form and on the
    split FP16 tables; plain orders 3 and 4 are reported beside it (their
    error against order 6 is what the correction competes with)."""
    params = np.load(WEIGHTS)
    res = tc.evaluate(params, lmax, lmax + 1, 2 * lmax, seeds, precision=precision, plain_orders=(3, 4))
    print(lmax, precision, res)
    for f, g in zip("TQU", res["gain"]):
        assert g > min_gain, (f, g, res)
    # the plain series converges: order 4 is closer to order 6 than order 2
    for f in range(3):
        assert res["rms_err_order4"][f] < res["rms_err_order2"][f]


def test_training_from_scratch_reduces_the_remainder(tc):
    """12 realizations x 20 steps of the stated configuration (the full run
    reached a loss of 0.16 after 10 realizations, from about 1)."""
    lmax = 2048
    params, info = tc.train(lmax, lmax + 1, 2 * lmax, list(range(10000, 10012)), steps_per_real=20,
                            batch_pixels=32768, lr=2e-3, lr_end=2e-3)
    h = info["loss_per_realization"]
    assert np.mean(h[-3:]) < 0.4 * h[0], h
    res = tc.evaluate(params, lmax, lmax + 1, 2 * lmax, [20001])
    print(res)
    for f, g in zip("TQU", res["gain"]):
        assert g > 1.5, (f, g, res)
