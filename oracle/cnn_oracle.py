"""CPU oracle of the learned Taylor-remainder correction -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  It shares no code with the GPU library
(``paper_1307_0719_amd``) and never imports it.

The paper's method stops the Taylor series of eq. 5 at a fixed order N; the
terms it drops (the remainder beyond N, Sec. II.B) are what this small
network predicts from the order <= 2 derivative maps around the nearest
pixel.  The network is not part of the paper; its definition here is the
reference the GPU kernels are checked against:

* Input of one output pixel x (nearest source pixel (i0, k0), scaled residuals
  u = dth/dtheta, v = dph/dphi): the 5 x 5 patch of source pixels
  (i0 + a, k0 + b), a, b in -2..2, rows clamped to the grid, columns wrapped
  in phi, of the 18 pre-scaled derivative maps
  Dt_{jk} = dtheta^j dphi^k / (j! k!) d^j_theta d^k_phi s, j + k <= 2, of
  s = T, Q, U (channel 6 f + index(j, k), index (0,0) (0,1) (0,2) (1,0) (1,1)
  (2,0)), each field divided by its patch RMS sigma_f over those 6 x 25
  values; channels 18 and 19 hold u and v on all 25 positions.
* conv 3x3 (valid) 20 -> 32, tanh; conv 3x3 (valid) 32 -> 32, tanh (one
  position left); 1x1 32 -> 3: y.
* Correction of field f: r_f = sigma_f * scale_f * y_f, added to the order-2
  Taylor sum before the polarization rotation.
* Training loss: mean over pixels and fields of (y_f - t_f / (sigma_f
  scale_f))^2 with t the target remainder (order-6 minus order-2 sums).
* Adam (Kingma & Ba 2015, Algorithm 1) with bias correction.

Parameter vector (float): W1[32][20][3][3], b1[32], W2[32][32][3][3], b2[32],
W3[3][32], b3[3], then scale[3] (fixed, not trained).
Everything here is float64 and written from those definitions.
"""
from __future__ import annotations

import math

import numpy as np

from oracle import taylens_oracle as tlo

NIN, NH, NOUT = 20, 32, 3
SIZES = [("W1", (NH, NIN, 3, 3)), ("b1", (NH,)), ("W2", (NH, NH, 3, 3)), ("b2", (NH,)),
         ("W3", (NOUT, NH)), ("b3", (NOUT,))]
NTRAIN = sum(int(np.prod(s)) for _, s in SIZES)   # trainable parameters
NPARAM = NTRAIN + NOUT                             # + output scales
DMAP_ORDER = [(0, 0), (0, 1), (0, 2), (1, 0), (1, 1), (2, 0)]


def unpack(vec):
    """Parameter vector -> dict of views (W1, b1, W2, b2, W3, b3, scale)."""
    vec = np.asarray(vec, dtype=np.float64)
    out, o = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = vec[o:o + n].reshape(shape)
        o += n
    out["scale"] = vec[o:o + NOUT]
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], np.float64).ravel() for name, _ in SIZES]
                          + [np.asarray(d.get("scale", np.ones(NOUT)), np.float64)])


# ------------------------------------------------------------ inputs ----

def scaled_derivative_maps(lmax, ntheta, nphi, alm_T, alm_E, alm_B=None, nthreads=0):
    """Dt_{jk} = dtheta^j dphi^k/(j! k!) d^j_theta d^k_phi s on every ring,
    j + k <= 2: {field: [6, ntheta, nphi]} in DMAP_ORDER."""
    D = tlo.derivative_rings(lmax, 2, ntheta, nphi, np.arange(ntheta), alm_T, alm_E, alm_B, nthreads)
    dth = math.pi / (ntheta - 1)
    dph = 2 * math.pi / nphi
    out = {}
    for f in D:
        out[f] = np.stack([D[f][(j, k)] * dth ** j * dph ** k / (math.factorial(j) * math.factorial(k))
                           for (j, k) in DMAP_ORDER])
    return out


def locate(lmax, ntheta, nphi, alm_phi, pix, nthreads=0):
    """Nearest source pixel and scaled residuals of output pixels pix (flat
    ring-major indices), geodesic positions: (i0, k0, u, v, tie)."""
    pix = np.asarray(pix, dtype=np.int64)
    rings = pix // nphi
    cols = pix % nphi
    ur = np.unique(rings)
    a_t, a_p = tlo.deflection_rings(lmax, alm_phi, ntheta, nphi, ur, nthreads)
    rpos = np.searchsorted(ur, rings)
    at = a_t[rpos, cols]
    ap = a_p[rpos, cols]
    th = tlo.grid_theta(ntheta)[rings]
    ph = tlo.grid_phi(nphi)[cols]
    thp, php, _, _, _ = tlo.geodesic_positions(th, ph, at, ap)
    i0, k0, dth, dph, tie = tlo.nearest_pixel(thp, php, ntheta, nphi)
    u = dth / (math.pi / (ntheta - 1))
    v = dph / (2 * math.pi / nphi)
    return i0, k0, u, v, tie


def features(Dt, fields, i0, k0, u, v):
    """Network input [P, 20, 5, 5] and patch RMS sigma [P, 3] (module doc)."""
    f0 = Dt[fields[0]]
    ntheta, nphi = f0.shape[1], f0.shape[2]
    P = len(i0)
    x = np.zeros((P, NIN, 5, 5))
    sig = np.ones((P, NOUT))
    a = np.arange(-2, 3)
    rows = np.clip(i0[:, None] + a[None, :], 0, ntheta - 1)       # [P, 5]
    cols = np.mod(k0[:, None] + a[None, :], nphi)                 # [P, 5]
    for fi, f in enumerate(("T", "Q", "U")):
        if f not in Dt:
            continue
        patch = Dt[f][:, rows[:, :, None], cols[:, None, :]]     # [6, P, 5, 5]
        patch = np.moveaxis(patch, 0, 1)                          # [P, 6, 5, 5]
        s = np.sqrt(np.mean(patch.reshape(P, -1) ** 2, axis=1))
        s = np.where(s > 0, s, 1.0)
        sig[:, fi] = s
        x[:, 6 * fi:6 * fi + 6] = patch / s[:, None, None, None]
    x[:, 18] = np.asarray(u)[:, None, None]
    x[:, 19] = np.asarray(v)[:, None, None]
    return x, sig


# ----------------------------------------------------------- network ----

def conv3_valid(x, W, b):
    """Plain 'valid' 3x3 cross-correlation: out[p, o, i, j] = b[o] +
    sum_{c, a, e} W[o, c, a, e] x[p, c, i + a, j + e]."""
    P, C, H, Wd = x.shape
    Ho, Wo = H - 2, Wd - 2
    out = np.empty((P, W.shape[0], Ho, Wo))
    for i in range(Ho):
        for j in range(Wo):
            out[:, :, i, j] = np.einsum("pcae,ocae->po", x[:, :, i:i + 3, j:j + 3], W) + b
    return out


def forward(params, x):
    """y [P, 3] and the activations needed by backward."""
    p = unpack(params)
    h1 = np.tanh(conv3_valid(x, p["W1"], p["b1"]))        # [P, 32, 3, 3]
    h2 = np.tanh(conv3_valid(h1, p["W2"], p["b2"]))[:, :, 0, 0]   # [P, 32]
    y = h2 @ p["W3"].T + p["b3"]
    return y, (h1, h2)


def loss_and_grad(params, x, t_norm):
    """MSE loss (mean over P x 3) and its gradient w.r.t. the trainable
    parameters (chain rule through the layers above), as a vector of
    length NTRAIN."""
    p = unpack(params)
    P = x.shape[0]
    y, (h1, h2) = forward(params, x)
    diff = y - t_norm
    loss = float(np.mean(diff ** 2))
    gy = 2.0 * diff / (P * NOUT)                       # dL/dy
    gW3 = gy.T @ h2
    gb3 = gy.sum(axis=0)
    gh2 = gy @ p["W3"]                                 # [P, 32]
    gz2 = gh2 * (1.0 - h2 ** 2)
    gW2 = np.einsum("po,pcae->ocae", gz2, h1)
    gb2 = gz2.sum(axis=0)
    gh1 = np.einsum("po,ocae->pcae", gz2, p["W2"])     # [P, 32, 3, 3]
    gz1 = gh1 * (1.0 - h1 ** 2)
    gW1 = np.zeros_like(p["W1"])
    for i in range(3):
        for j in range(3):
            gW1 += np.einsum("po,pcae->ocae", gz1[:, :, i, j], x[:, :, i:i + 3, j:j + 3])
    gb1 = gz1.sum(axis=(0, 2, 3))
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
    return loss, g


def normalized_target(t, sig, scale):
    """t_f / (sigma_f scale_f) for targets t [P, 3]."""
    return t / (sig * np.asarray(scale)[None, :])


def correction(params, x, sig):
    """r_f = sigma_f scale_f y_f  [P, 3]."""
    y, _ = forward(params, x)
    return y * sig * unpack(params)["scale"][None, :]


def adam_step(params, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update of the trainable part (step counts from 1); returns
    new (params, m, v)."""
    params = np.array(params, dtype=np.float64)
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad ** 2
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    params[:NTRAIN] -= lr * mh / (np.sqrt(vh) + eps)
    return params, m, v
