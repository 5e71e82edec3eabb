"""Pins of the CPU oracle of the learned remainder correction (not gpu).

The network, its gradient and the optimizer step are checked against library
routines that compute the same definitions independently (torch's conv2d,
autograd and Adam, all float64 on the CPU) and against central finite
differences; the patch gather against hand-built maps whose values encode
their own (map, ring, column)."""
import math

import numpy as np
import pytest
import torch

from oracle import cnn_oracle as co
from oracle import taylens_oracle as tlo
from paper_1307_0719_amd import skygen


def _params(seed=5):
    p = skygen.cnn_init(seed).astype(np.float64)
    p[-3:] = [0.7, 1.3, 2.0]
    return p


def _x(P=7, seed=9):
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal((P, co.NIN, 5, 5))


def _torch_forward(p, x):
    d = {k: torch.tensor(v) for k, v in co.unpack(p).items()}
    for k in d:
        d[k].requires_grad_(k != "scale")
    xt = torch.tensor(x)
    h1 = torch.tanh(torch.nn.functional.conv2d(xt, d["W1"], d["b1"]))
    h2 = torch.tanh(torch.nn.functional.conv2d(h1, d["W2"], d["b2"]))[:, :, 0, 0]
    y = torch.nn.functional.linear(h2, d["W3"], d["b3"])
    return y, d


def test_conv_is_library_cross_correlation():
    rng = np.random.Generator(np.random.PCG64(1))
    x = rng.standard_normal((3, 4, 6, 5))
    W = rng.standard_normal((2, 4, 3, 3))
    b = rng.standard_normal(2)
    ref = torch.nn.functional.conv2d(torch.tensor(x), torch.tensor(W), torch.tensor(b)).numpy()
    np.testing.assert_allclose(co.conv3_valid(x, W, b), ref, rtol=1e-13, atol=1e-13)


def test_forward_matches_torch():
    p, x = _params(), _x()
    y, _ = co.forward(p, x)
    yt, _ = _torch_forward(p, x)
    np.testing.assert_allclose(y, yt.detach().numpy(), rtol=1e-13, atol=1e-14)


def test_gradient_matches_autograd():
    p, x = _params(), _x()
    t = np.random.Generator(np.random.PCG64(3)).standard_normal((x.shape[0], 3))
    loss, g = co.loss_and_grad(p, x, t)
    yt, d = _torch_forward(p, x)
    lt = torch.mean((yt - torch.tensor(t)) ** 2)
    lt.backward()
    gt = np.concatenate([d[k].grad.numpy().ravel() for k, _ in co.SIZES])
    assert abs(loss - lt.item()) < 1e-14 * max(1.0, abs(loss))
    np.testing.assert_allclose(g, gt, rtol=1e-11, atol=1e-15)


def test_gradient_matches_finite_differences():
    p, x = _params(7), _x(5, 11)
    t = np.random.Generator(np.random.PCG64(4)).standard_normal((5, 3))
    _, g = co.loss_and_grad(p, x, t)
    rng = np.random.Generator(np.random.PCG64(8))
    idx = rng.choice(co.NTRAIN, 24, replace=False)
    h = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (co.loss_and_grad(pp, x, t)[0] - co.loss_and_grad(pm, x, t)[0]) / (2 * h)
        assert abs(fd - g[i]) < 1e-7 + 1e-5 * abs(g[i]), (i, fd, g[i])


def test_adam_matches_torch():
    p = _params()
    rng = np.random.Generator(np.random.PCG64(2))
    w = torch.tensor(p[:co.NTRAIN].copy(), requires_grad=True)
    opt = torch.optim.Adam([w], lr=3e-3, betas=(0.9, 0.999), eps=1e-8)
    m = np.zeros(co.NTRAIN)
    v = np.zeros(co.NTRAIN)
    cur = p.copy()
    for step in range(1, 5):
        g = rng.standard_normal(co.NTRAIN)
        opt.zero_grad()
        w.grad = torch.tensor(g)
        opt.step()
        cur, m, v = co.adam_step(cur, g, m, v, step, 3e-3)
    np.testing.assert_allclose(cur[:co.NTRAIN], w.detach().numpy(), rtol=1e-12, atol=1e-15)
    np.testing.assert_array_equal(cur[co.NTRAIN:], p[co.NTRAIN:])


def test_patch_gather_clamps_rows_and_wraps_columns():
    ntheta, nphi = 9, 12
    r, c = np.meshgrid(np.arange(ntheta), np.arange(nphi), indexing="ij")
    Dt = {f: np.stack([1000.0 * (6 * fi + q + 1) + 20.0 * r + c for q in range(6)])
          for fi, f in enumerate("TQU")}
    i0 = np.array([0, 4, 8, 1])
    k0 = np.array([0, 11, 5, 1])
    u = np.array([0.1, -0.2, 0.5, -0.5])
    v = np.array([0.3, 0.0, -0.4, 0.25])
    x, sig = co.features(Dt, "TQU", i0, k0, u, v)
    for p in range(4):
        for a in range(5):
            for b in range(5):
                rr = min(max(i0[p] + a - 2, 0), ntheta - 1)
                cc = (k0[p] + b - 2) % nphi
                for ch in range(18):
                    raw = 1000.0 * (ch + 1) + 20.0 * rr + cc
                    assert x[p, ch, a, b] * sig[p, ch // 6] == pytest.approx(raw, rel=1e-14)
        assert np.all(x[p, 18] == u[p]) and np.all(x[p, 19] == v[p])
        for f in range(3):
            assert np.sqrt(np.mean(x[p, 6 * f:6 * f + 6] ** 2)) == pytest.approx(1.0, rel=1e-13)


def test_locate_agrees_with_the_remap_of_the_lensing_oracle():
    lmax, ntheta, nphi = 24, 25, 48
    sky = skygen.make_sky(lmax, 17, rms_arcmin=400.0)
    pix = skygen.sample_pixels(ntheta * nphi, 60, 3)
    i0, k0, u, v, _ = co.locate(lmax, ntheta, nphi, sky.alm_phi, pix)
    ref = tlo.lens_rings(lmax, 1, ntheta, nphi, np.arange(ntheta), sky.alm_T, None, None, sky.alm_phi)
    r, c = pix // nphi, pix % nphi
    np.testing.assert_array_equal(i0, ref["_i0"][r, c])
    np.testing.assert_array_equal(k0, ref["_k0"][r, c])
    np.testing.assert_allclose(u * math.pi / (ntheta - 1), ref["_dth"][r, c], rtol=0, atol=1e-15)
    np.testing.assert_allclose(v * 2 * math.pi / nphi, ref["_dph"][r, c], rtol=0, atol=1e-15)
    assert np.all(np.abs(u) <= 0.5 + 1e-12) and np.all(np.abs(v) <= 0.5 + 1e-12)


def test_scaled_derivative_maps_are_the_taylor_terms():
    """A first-order Taylor step built from the scaled maps reproduces the
    field half a pixel away to O(dtheta^2) (finite-difference consistency
    of the scaling dtheta^j dphi^k / (j! k!))."""
    lmax, ntheta, nphi = 16, 129, 256
    sky = skygen.make_sky(lmax, 2)
    Dt = co.scaled_derivative_maps(lmax, ntheta, nphi, sky.alm_T, sky.alm_E)
    T = Dt["T"]
    # central difference in phi over one pixel ~ 2 * Dt_01, in theta ~ 2 * Dt_10
    dphi_fd = (np.roll(T[0], -1, axis=1) - np.roll(T[0], 1, axis=1)) / 2
    np.testing.assert_allclose(dphi_fd[1:-1], T[1][1:-1], atol=2e-3 * np.abs(T[0]).max())
    dth_fd = (T[0][2:] - T[0][:-2]) / 2
    np.testing.assert_allclose(dth_fd, T[3][1:-1], atol=2e-3 * np.abs(T[0]).max())
    # second derivatives: Dt_02 = dphi^2/2 d2, central second difference = 2 Dt_02
    d2 = np.roll(T[0], -1, axis=1) - 2 * T[0] + np.roll(T[0], 1, axis=1)
    np.testing.assert_allclose(d2[1:-1] / 2, T[2][1:-1], atol=2e-3 * np.abs(T[0]).max())


def test_zero_output_layer_gives_zero_correction():
    p = _params()
    d = co.unpack(p.copy())
    d["W3"][:] = 0
    d["b3"][:] = 0
    r = co.correction(co.pack(d), _x(), np.ones((7, 3)))
    assert np.all(r == 0)
