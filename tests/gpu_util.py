"""Helpers for the GPU parity tests (HIP path vs the CPU oracle)."""
from __future__ import annotations

import math
import os

import numpy as np
import pytest
import torch

ORACLE_THREADS = int(os.environ.get("TAYLENS_ORACLE_THREADS", "0"))


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def rel_rms(x, ref, mask=None):
    x = np.asarray(x, float)
    ref = np.asarray(ref, float)
    if mask is not None:
        x, ref = x[mask], ref[mask]
    return float(np.sqrt(np.mean((x - ref) ** 2)) / max(np.sqrt(np.mean(ref ** 2)), 1e-300))


def max_rel(x, ref, mask=None):
    """max |x - ref| over the RMS of ref."""
    x = np.asarray(x, float)
    ref = np.asarray(ref, float)
    if mask is not None:
        x, ref = x[mask], ref[mask]
    return float(np.max(np.abs(x - ref)) / max(np.sqrt(np.mean(ref ** 2)), 1e-300))


def dmap_scale(j, k, ntheta, nphi):
    dth = math.pi / (ntheta - 1)
    dph = 2 * math.pi / nphi
    return dth ** j * dph ** k / (math.factorial(j) * math.factorial(k))


def oracle_scaled_derivs(oracle, lmax, order, ntheta, nphi, rings, aT, aE=None, aB=None):
    """Oracle derivative maps in the library's layout and scaling:
    [field][jk][len(rings)][nphi]."""
    D = oracle.derivative_rings(lmax, order, ntheta, nphi, rings, aT, aE, aB, ORACLE_THREADS)
    fields = ["T"] + (["Q", "U"] if aE is not None else [])
    pairs = oracle.jk_pairs(order)
    out = np.zeros((len(fields), len(pairs), len(np.atleast_1d(rings)), nphi))
    for f, name in enumerate(fields):
        for q, (j, k) in enumerate(pairs):
            out[f, q] = D[name][(j, k)] * dmap_scale(j, k, ntheta, nphi)
    return out


def t2np(t):
    if t is None or isinstance(t, np.ndarray):
        return t
    return t.detach().cpu().numpy()


def smooth_nphi(n):
    """Smallest even nphi >= n with nphi/2 a product of 2, 3, 5."""
    m = max(1, (n + 1) // 2)
    while True:
        k = m
        for r in (2, 3, 5):
            while k % r == 0:
                k //= r
        if k == 1:
            return 2 * m
        m += 1
