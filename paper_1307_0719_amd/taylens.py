"""Python binding of libtaylens (ctypes).  Argument marshalling only: every
step of the lensing path runs in the library's HIP kernels.  PyTorch supplies
device memory and the stream.

The library must have been built (``python -m paper_1307_0719_amd.build``);
importing this module raises if ``libtaylens.so`` is missing -- there is no
fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtaylens.so")

TL_OK = 0
TL_ERR_INVALID = -1
TL_ERR_UNSUPPORTED = -2
TL_ERR_HIP = -3
TL_ERR_NOMEM = -4
MAX_ORDER = 8

PRECISIONS = {"fp64": 0, "fp32": 1, "bf16x3": 2, "fp16x2": 3, "fp16": 4, "bf16": 5}

# every symbol include/taylens.h declares
EXPORTS = [
    "tl_plan_create", "tl_plan_destroy", "tl_plan_workspace_bytes", "tl_plan_query", "tl_lens_map", "tl_lens_map_pos",
    "tl_deflection", "tl_legendre", "tl_synth_derivs", "tl_theta_derivs", "tl_analysis_T", "tl_remap", "tl_lens_map_batch",
    "tl_lens_map_simple", "tl_lens_map_many", "tl_plan_profile", "tl_plan_stage_times", "tl_last_error", "tl_version",
    "tl_cnn_create", "tl_cnn_destroy", "tl_cnn_get_params", "tl_cnn_set_params", "tl_cnn_forward", "tl_cnn_grad",
    "tl_cnn_train_step", "tl_lens_map_cnn", "tl_batch_create", "tl_batch_destroy", "tl_batch_run", "tl_batch_info",
    "tl_lens_map_simple_noalloc", "tl_plan_create_healpix",
]
CNN_NTRAIN = 15139
CNN_NPARAM = 15142
STAGES = ["defl_legendre", "defl_fft", "legendre_T", "legendre_QU", "legendre_mfma", "tab_rhs", "legendre_tab",
          "ring_fft", "remap", "cnn", "tab_epi", "legendre_caps"]
QUERY_KEYS = {"rpole": 0, "elems": 1, "elems_caps": 2, "tab_chunks": 3, "tab_chunk_bytes": 4, "defl_folded": 5}
# kernel each stage launches
STAGE_KERNELS = {"defl_legendre": "k_legendre_scalar", "defl_fft": "k_ring_fft", "legendre_T": "k_legendre_scalar",
                 "legendre_QU": "k_legendre_spin", "legendre_mfma": "k_legendre_mfma", "tab_rhs": "k_tab_rhs",
                 "legendre_tab": "k_legendre_tab", "ring_fft": "k_ring_fft", "remap": "k_remap",
                 "cnn": "k_cnn_forward", "tab_epi": "k_tab_epi", "legendre_caps": "k_legendre_caps"}


class TaylensError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"taylens error {code}: {msg}")
        self.code = code


class Grid(ctypes.Structure):
    _fields_ = [("ntheta", ctypes.c_int32), ("nphi", ctypes.c_int32)]


class Options(ctypes.Structure):
    _fields_ = [("order", ctypes.c_int32), ("precision", ctypes.c_int32), ("pol", ctypes.c_int32),
                ("rotate", ctypes.c_int32), ("naive_pos", ctypes.c_int32), ("batch", ctypes.c_int32),
                ("workspace_cap", ctypes.c_int64), ("maps16", ctypes.c_int32), ("lmax_phi", ctypes.c_int32),
                ("theta_fft", ctypes.c_int32)]


class BatchOptions(ctypes.Structure):
    _fields_ = [("autotune", ctypes.c_int32), ("use_graph", ctypes.c_int32), ("m_groups", ctypes.c_int32),
                ("groups_per_cu", ctypes.c_int32)]


_lib = None


def lib():
    """The loaded library (raises ImportError if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libtaylens.so not built at {LIB_PATH}; run python -m paper_1307_0719_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        L.tl_plan_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int32, Grid, ctypes.POINTER(Options), vp]
        L.tl_plan_create_healpix.argtypes = [ctypes.POINTER(vp), ctypes.c_int32, ctypes.c_int32,
                                             ctypes.POINTER(Options), vp]
        L.tl_plan_destroy.argtypes = [vp]
        L.tl_plan_workspace_bytes.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
        L.tl_plan_query.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)]
        L.tl_lens_map.argtypes = [vp] * 8
        L.tl_lens_map_pos.argtypes = [vp] * 9
        L.tl_deflection.argtypes = [vp] * 4
        L.tl_legendre.argtypes = [vp] * 5
        L.tl_synth_derivs.argtypes = [vp] * 5
        L.tl_remap.argtypes = [vp] * 7
        L.tl_theta_derivs.argtypes = [vp, vp, ctypes.c_int32, ctypes.c_int32, vp]
        L.tl_analysis_T.argtypes = [vp, vp, vp]
        L.tl_lens_map_batch.argtypes = [ctypes.c_int32, vp, vp, vp]
        L.tl_lens_map_simple.argtypes = [vp, vp, vp, vp, ctypes.c_int32, ctypes.c_int32, Grid, vp, vp, vp]
        L.tl_lens_map_simple_noalloc.argtypes = [vp, vp, vp, vp, ctypes.c_int32, ctypes.c_int32, Grid, vp, vp, vp]
        L.tl_lens_map_many.argtypes = [vp, ctypes.c_int32, vp, vp]
        L.tl_plan_profile.argtypes = [vp, ctypes.c_int32]
        L.tl_plan_stage_times.argtypes = [vp, vp, vp]
        L.tl_cnn_create.argtypes = [ctypes.POINTER(vp), vp]
        L.tl_cnn_destroy.argtypes = [vp]
        L.tl_cnn_get_params.argtypes = [vp, vp]
        L.tl_cnn_set_params.argtypes = [vp, vp]
        L.tl_cnn_forward.argtypes = [vp, vp, vp, vp, vp, vp, ctypes.c_int64, vp]
        L.tl_cnn_grad.argtypes = [vp, vp, vp, vp, vp, vp, ctypes.c_int64, vp, vp]
        L.tl_cnn_train_step.argtypes = [vp, vp, vp, vp, vp, vp, ctypes.c_int64, vp, ctypes.c_float, vp]
        L.tl_lens_map_cnn.argtypes = [vp] * 9
        L.tl_batch_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int32, vp, ctypes.POINTER(BatchOptions)]
        L.tl_batch_destroy.argtypes = [vp]
        L.tl_batch_run.argtypes = [vp, vp, vp]
        L.tl_batch_info.argtypes = [vp, vp, vp, vp, vp]
        L.tl_last_error.restype = ctypes.c_char_p
        L.tl_last_error.argtypes = []
        L.tl_version.restype = ctypes.c_int
        for name in EXPORTS:
            getattr(L, name).restype = ctypes.c_int if name != "tl_last_error" else ctypes.c_char_p
        _lib = L
    return _lib


def _check(rc: int):
    if rc != TL_OK:
        raise TaylensError(rc, lib().tl_last_error().decode())


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def _alm(a, name, device, lmax):
    """complex128 contiguous device tensor of the expected length (or None)."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        a = torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex128))
    if a.dtype != torch.complex128:
        raise TypeError(f"{name} must be complex128")
    n = (lmax + 1) * (lmax + 2) // 2
    if a.numel() != n:
        raise ValueError(f"{name} has {a.numel()} coefficients, lmax={lmax} needs {n}")
    return a.to(device).contiguous()


class Plan:
    """A lensing plan: band limit, ring grid, Taylor order, precision form."""

    def __init__(self, lmax: int, ntheta: int, nphi: int, order: int, precision: str = "fp32",
                 pol: bool = True, rotate: bool = True, naive_pos: bool = False, workspace_cap: int = 0,
                 device: Optional[torch.device] = None, stream: Optional[torch.cuda.Stream] = None,
                 batch: int = 1, nside: int = 0, maps16: bool = False, lmax_phi: int = 0,
                 theta_fft: bool = False):
        """ntheta x nphi equal-theta grid, or with nside > 0 HEALPix rings
        (ntheta, nphi ignored; maps are [12 nside^2] in RING order).  maps16:
        internal derivative maps of order j + k >= 3 in FP16; lmax_phi: band
        limit of the lensing potential, 0 = lmax; theta_fft: FP64 plans take
        the theta-derivatives by FFT along great circles (see tl_options)."""
        self.nside = int(nside)
        if self.nside:
            ntheta, nphi = 4 * self.nside - 1, 4 * self.nside
        self.lmax, self.ntheta, self.nphi, self.order = int(lmax), int(ntheta), int(nphi), int(order)
        self.lmax_phi = int(lmax_phi) if lmax_phi else self.lmax
        self.npix = 12 * self.nside ** 2 if self.nside else self.ntheta * self.nphi
        self.precision = precision
        self.pol = bool(pol)
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        if precision not in PRECISIONS:
            raise ValueError(f"unknown precision {precision}")
        opt = Options(order, PRECISIONS[precision], int(pol), int(rotate), int(naive_pos), int(batch),
                      int(workspace_cap), int(maps16), int(lmax_phi), int(theta_fft))
        self.batch = int(batch)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            if self.nside:
                _check(lib().tl_plan_create_healpix(ctypes.byref(h), self.lmax, self.nside, ctypes.byref(opt),
                                                    ctypes.c_void_p(self.stream.cuda_stream)))
            else:
                _check(lib().tl_plan_create(ctypes.byref(h), self.lmax, Grid(self.ntheta, self.nphi),
                                            ctypes.byref(opt), ctypes.c_void_p(self.stream.cuda_stream)))
        self._h = h
        self.real_dtype = torch.float64 if precision == "fp64" else torch.float32
        self.cplx_dtype = torch.complex128 if precision == "fp64" else torch.complex64

    # ---------------------------------------------------------------- utils
    @property
    def handle(self):
        return self._h

    @property
    def nfield(self):
        return 3 if self.pol else 1

    @property
    def ndmap(self):
        return (self.order + 1) * (self.order + 2) // 2

    def workspace_bytes(self) -> int:
        b = ctypes.c_int64()
        _check(lib().tl_plan_workspace_bytes(self._h, ctypes.byref(b)))
        return int(b.value)

    def query(self, key: str) -> int:
        """Work counts fixed at plan creation: rpole, elems, elems_caps,
        tab_chunks, tab_chunk_bytes."""
        b = ctypes.c_int64()
        _check(lib().tl_plan_query(self._h, QUERY_KEYS[key], ctypes.byref(b)))
        return b.value

    def profile(self, enable: bool = True):
        """Start (or stop) per-stage HIP-event timing on the plan's stream."""
        _check(lib().tl_plan_profile(self._h, int(enable)))

    def stage_times(self):
        """{stage: (total_ms, launches)} since profile() (synchronizes)."""
        ms = (ctypes.c_double * len(STAGES))()
        n = (ctypes.c_int64 * len(STAGES))()
        _check(lib().tl_plan_stage_times(self._h, ctypes.cast(ms, ctypes.c_void_p), ctypes.cast(n, ctypes.c_void_p)))
        return {s: (ms[i], n[i]) for i, s in enumerate(STAGES)}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().tl_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def map_shape(self):
        return (self.npix,) if self.nside else (self.ntheta, self.nphi)

    def _maps(self, n=None):
        shape = self.map_shape if n is None else (n, *self.map_shape)
        return torch.empty(shape, dtype=self.real_dtype, device=self.device)

    def _inputs(self, alm_T, alm_E, alm_B):
        T = _alm(alm_T, "alm_T", self.device, self.lmax)
        E = _alm(alm_E, "alm_E", self.device, self.lmax) if self.pol else None
        B = _alm(alm_B, "alm_B", self.device, self.lmax) if self.pol else None
        return T, E, B

    # ------------------------------------------------------------- calls
    def lens_map(self, alm_T, alm_E=None, alm_B=None, alm_phi=None, out=None):
        """Lensed (T, Q, U) maps; Q/U are None for a T-only plan."""
        T, E, B = self._inputs(alm_T, alm_E, alm_B)
        P = _alm(alm_phi, "alm_phi", self.device, self.lmax_phi)
        if out is None:
            out = (self._maps(), self._maps() if self.pol else None, self._maps() if self.pol else None)
        _check(lib().tl_lens_map(self._h, _ptr(T), _ptr(E), _ptr(B), _ptr(P), _ptr(out[0]), _ptr(out[1]),
                                 _ptr(out[2])))
        self._keep = (T, E, B, P)
        return out

    def lens_map_many(self, alms, outs=None):
        """alms: list of (T, E, B, phi) tuples; returns list of (T, Q, U)."""
        n = len(alms)
        keep = []
        aarr = (ctypes.c_void_p * (4 * n))()
        oarr = (ctypes.c_void_p * (3 * n))()
        if outs is None:
            outs = [(self._maps(), self._maps() if self.pol else None, self._maps() if self.pol else None)
                    for _ in range(n)]
        for i, a in enumerate(alms):
            T, E, B = self._inputs(a[0], a[1], a[2])
            P = _alm(a[3], "alm_phi", self.device, self.lmax_phi)
            keep.append((T, E, B, P))
            for q, t in enumerate((T, E, B, P)):
                aarr[4 * i + q] = t.data_ptr() if t is not None else None
            for q, t in enumerate(outs[i]):
                oarr[3 * i + q] = t.data_ptr() if t is not None else None
        _check(lib().tl_lens_map_many(self._h, n, ctypes.cast(aarr, ctypes.c_void_p),
                                      ctypes.cast(oarr, ctypes.c_void_p)))
        self._keep = keep
        return outs

    def lens_map_pos(self, alm_T, alm_E, alm_B, theta_src: torch.Tensor, phi_src: torch.Tensor):
        T, E, B = self._inputs(alm_T, alm_E, alm_B)
        th = theta_src.to(self.device, torch.float64).contiguous()
        ph = phi_src.to(self.device, torch.float64).contiguous()
        out = (self._maps(), self._maps() if self.pol else None, self._maps() if self.pol else None)
        _check(lib().tl_lens_map_pos(self._h, _ptr(T), _ptr(E), _ptr(B), _ptr(th), _ptr(ph), _ptr(out[0]),
                                     _ptr(out[1]), _ptr(out[2])))
        self._keep = (T, E, B, th, ph)
        return out

    def deflection(self, alm_phi):
        P = _alm(alm_phi, "alm_phi", self.device, self.lmax_phi)
        at = torch.empty(self.map_shape, dtype=torch.float64, device=self.device)
        ap = torch.empty_like(at)
        _check(lib().tl_deflection(self._h, _ptr(P), _ptr(at), _ptr(ap)))
        self._keep = (P,)
        return at, ap

    def legendre(self, alm_T, alm_E=None, alm_B=None):
        """F[field][j][ring][m] complex."""
        T, E, B = self._inputs(alm_T, alm_E, alm_B)
        F = torch.empty((self.nfield, self.order + 1, self.ntheta, self.lmax + 1), dtype=self.cplx_dtype,
                        device=self.device)
        _check(lib().tl_legendre(self._h, _ptr(T), _ptr(E), _ptr(B), _ptr(F)))
        self._keep = (T, E, B)
        return F

    def synth_derivs(self, alm_T, alm_E=None, alm_B=None):
        """Scaled derivative maps D[field][jk][ring][pix]."""
        T, E, B = self._inputs(alm_T, alm_E, alm_B)
        D = torch.empty((self.nfield, self.ndmap, *self.map_shape), dtype=self.real_dtype, device=self.device)
        _check(lib().tl_synth_derivs(self._h, _ptr(T), _ptr(E), _ptr(B), _ptr(D)))
        self._keep = (T, E, B)
        return D

    def analysis_T(self, Tmap: torch.Tensor):
        """a_lm (complex128, triangular) of a temperature map [ntheta, nphi]
        by Clenshaw-Curtis quadrature over the rings and ring FFTs."""
        Tmap = Tmap.to(self.device, torch.float64).contiguous()
        if tuple(Tmap.shape) != tuple(self.map_shape):
            raise ValueError("map must be (ntheta, nphi)")
        alm = torch.empty((self.lmax + 1) * (self.lmax + 2) // 2, dtype=torch.complex128, device=self.device)
        _check(lib().tl_analysis_T(self._h, _ptr(Tmap), _ptr(alm)))
        self._keep = (Tmap,)
        return alm

    def theta_derivs(self, maps: torch.Tensor, jmax: int):
        """dtheta^j / j! d^j_theta of maps [..., ntheta, nphi] by FFT along the
        great circles through both poles: [..., jmax, ntheta, nphi]."""
        maps = maps.to(self.device, self.real_dtype).contiguous()
        if tuple(maps.shape[-2:]) != tuple(self.map_shape):
            raise ValueError("maps must end in (ntheta, nphi)")
        lead = tuple(maps.shape[:-2])
        nmaps = int(np.prod(lead)) if lead else 1
        out = torch.empty(lead + (int(jmax), *self.map_shape), dtype=self.real_dtype, device=self.device)
        _check(lib().tl_theta_derivs(self._h, _ptr(maps), nmaps, int(jmax), _ptr(out)))
        self._keep = (maps,)
        return out

    def remap(self, D: torch.Tensor, alpha_theta: torch.Tensor, alpha_phi: torch.Tensor):
        D = D.to(self.device, self.real_dtype).contiguous()
        at = alpha_theta.to(self.device, torch.float64).contiguous()
        ap = alpha_phi.to(self.device, torch.float64).contiguous()
        if D.numel() != self.nfield * self.ndmap * self.npix:
            raise ValueError("D has the wrong size for this plan")
        out = (self._maps(), self._maps() if self.pol else None, self._maps() if self.pol else None)
        _check(lib().tl_remap(self._h, _ptr(D), _ptr(at), _ptr(ap), _ptr(out[0]), _ptr(out[1]), _ptr(out[2])))
        self._keep = (D, at, ap)
        return out


class Cnn:
    """The learned remainder correction (weights on the device, Adam state).

    Parameter vector layout: W1[32][20][3][3], b1[32], W2[32][32][3][3],
    b2[32], W3[3][32], b3[3], scale[3] (float32, CNN_NPARAM values)."""

    def __init__(self, params):
        p = np.ascontiguousarray(np.asarray(params, dtype=np.float32))
        if p.size != CNN_NPARAM:
            raise ValueError(f"expected {CNN_NPARAM} parameters, got {p.size}")
        h = ctypes.c_void_p()
        _check(lib().tl_cnn_create(ctypes.byref(h), p.ctypes.data_as(ctypes.c_void_p)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().tl_cnn_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def params(self) -> np.ndarray:
        out = np.empty(CNN_NPARAM, dtype=np.float32)
        _check(lib().tl_cnn_get_params(self._h, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def set_params(self, params):
        p = np.ascontiguousarray(np.asarray(params, dtype=np.float32))
        if p.size != CNN_NPARAM:
            raise ValueError(f"expected {CNN_NPARAM} parameters")
        _check(lib().tl_cnn_set_params(self._h, p.ctypes.data_as(ctypes.c_void_p)))

    @staticmethod
    def _args(plan, D, at, ap, pix):
        D = D.to(plan.device, torch.float32).contiguous()
        at = at.to(plan.device, torch.float64).contiguous()
        ap = ap.to(plan.device, torch.float64).contiguous()
        if pix is not None:
            pix = torch.as_tensor(pix, dtype=torch.int64).to(plan.device).contiguous()
        return D, at, ap, pix

    def forward(self, plan: Plan, D, alpha_theta, alpha_phi, pix=None, n=None):
        """Corrections [3][n] of the pixels pix (or of pixels 0..n-1)."""
        D, at, ap, pix = self._args(plan, D, alpha_theta, alpha_phi, pix)
        n = int(pix.numel()) if pix is not None else int(n if n is not None else plan.ntheta * plan.nphi)
        out = torch.empty((3, n), dtype=torch.float32, device=plan.device)
        _check(lib().tl_cnn_forward(self._h, plan.handle, _ptr(D), _ptr(at), _ptr(ap), _ptr(pix), n, _ptr(out)))
        self._keep = (D, at, ap, pix)
        return out

    def grad(self, plan: Plan, D, alpha_theta, alpha_phi, pix, target):
        """[CNN_NTRAIN + 1]: gradient of the loss, then the loss."""
        D, at, ap, pix = self._args(plan, D, alpha_theta, alpha_phi, pix)
        t = target.to(plan.device, torch.float32).contiguous()
        n = int(t.shape[-1])
        out = torch.empty(CNN_NTRAIN + 1, dtype=torch.float32, device=plan.device)
        _check(lib().tl_cnn_grad(self._h, plan.handle, _ptr(D), _ptr(at), _ptr(ap), _ptr(pix), n, _ptr(t),
                                 _ptr(out)))
        self._keep = (D, at, ap, pix, t)
        return out

    def train_step(self, plan: Plan, D, alpha_theta, alpha_phi, pix, target, lr: float):
        """One Adam step; returns the loss before it (device scalar tensor)."""
        D, at, ap, pix = self._args(plan, D, alpha_theta, alpha_phi, pix)
        t = target.to(plan.device, torch.float32).contiguous()
        n = int(t.shape[-1])
        loss = torch.empty(1, dtype=torch.float32, device=plan.device)
        _check(lib().tl_cnn_train_step(self._h, plan.handle, _ptr(D), _ptr(at), _ptr(ap), _ptr(pix), n, _ptr(t),
                                       ctypes.c_float(lr), _ptr(loss)))
        self._keep = (D, at, ap, pix, t)
        return loss

    def lens_map(self, plan: Plan, alm_T, alm_E, alm_B, alm_phi, out=None):
        """Order-2 lensing of plan with the network's correction."""
        T, E, B = plan._inputs(alm_T, alm_E, alm_B)
        P = _alm(alm_phi, "alm_phi", plan.device, plan.lmax_phi)
        if out is None:
            out = (plan._maps(), plan._maps(), plan._maps())
        _check(lib().tl_lens_map_cnn(plan.handle, self._h, _ptr(T), _ptr(E), _ptr(B), _ptr(P), _ptr(out[0]),
                                     _ptr(out[1]), _ptr(out[2])))
        self._keep = (T, E, B, P)
        return out


class Batch:
    """Realizations of uneven lmax lensed in one pass (one persistent
    harmonic launch with a longest-first queue, optional HIP-graph replay,
    autotuned work-item shape).  plans[i] is realization i's plan (FP32 form;
    plans may repeat)."""

    def __init__(self, plans: Sequence[Plan], autotune: bool = True, use_graph: bool = True, m_groups: int = 0,
                 groups_per_cu: int = 0):
        self.plans = list(plans)
        harr = (ctypes.c_void_p * len(self.plans))(*[p.handle.value for p in self.plans])
        opt = BatchOptions(int(autotune), int(use_graph), int(m_groups), int(groups_per_cu))
        h = ctypes.c_void_p()
        _check(lib().tl_batch_create(ctypes.byref(h), len(self.plans), ctypes.cast(harr, ctypes.c_void_p),
                                     ctypes.byref(opt)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().tl_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def outputs(self):
        return [(p._maps(), p._maps() if p.pol else None, p._maps() if p.pol else None) for p in self.plans]

    def run(self, alms: Sequence[tuple], outs=None):
        """alms[i] = (T, E, B, phi) device tensors (kept at the same addresses
        for graph replay); returns outs[i] = (T, Q, U)."""
        n = len(self.plans)
        if outs is None:
            outs = self.outputs()
        keep = []
        aarr = (ctypes.c_void_p * (4 * n))()
        oarr = (ctypes.c_void_p * (3 * n))()
        for i, (p, a) in enumerate(zip(self.plans, alms)):
            for q, t in enumerate(a):
                if t is not None and (t.device != p.device or not t.is_contiguous() or t.dtype != torch.complex128):
                    raise ValueError("batch inputs must be contiguous complex128 tensors on the plan's device")
                aarr[4 * i + q] = t.data_ptr() if t is not None else None
            for q, t in enumerate(outs[i]):
                oarr[3 * i + q] = t.data_ptr() if t is not None else None
            keep.append(a)
        _check(lib().tl_batch_run(self._h, ctypes.cast(aarr, ctypes.c_void_p), ctypes.cast(oarr, ctypes.c_void_p)))
        self._keep = keep
        return outs

    def info(self):
        mg, gc = ctypes.c_int32(), ctypes.c_int32()
        ms, rp = ctypes.c_double(), ctypes.c_int64()
        _check(lib().tl_batch_info(self._h, ctypes.byref(mg), ctypes.byref(gc), ctypes.byref(ms), ctypes.byref(rp)))
        return {"m_groups": mg.value, "groups_per_cu": gc.value, "tuned_ms": ms.value, "graph_replays": rp.value}


def lens_map_batch(plans: Sequence[Plan], alms: Sequence[tuple], outs: Sequence[tuple]):
    """Lens len(plans) realizations in one call (alms[i] = (T, E, B, phi),
    outs[i] = (T, Q, U) preallocated)."""
    n = len(plans)
    keep = []
    harr = (ctypes.c_void_p * n)(*[p.handle.value for p in plans])
    aarr = (ctypes.c_void_p * (4 * n))()
    oarr = (ctypes.c_void_p * (3 * n))()
    for i, (p, a, o) in enumerate(zip(plans, alms, outs)):
        T, E, B = p._inputs(a[0], a[1], a[2])
        P = _alm(a[3], "alm_phi", p.device, p.lmax_phi)
        keep.append((T, E, B, P))
        for q, t in enumerate((T, E, B, P)):
            aarr[4 * i + q] = t.data_ptr() if t is not None else None
        for q, t in enumerate(o):
            oarr[3 * i + q] = t.data_ptr() if t is not None else None
    _check(lib().tl_lens_map_batch(n, ctypes.cast(harr, ctypes.c_void_p), ctypes.cast(aarr, ctypes.c_void_p),
                                   ctypes.cast(oarr, ctypes.c_void_p)))
    return keep


def lens_map(alm_T, alm_E, alm_B, alm_phi, lmax: int, order: int, ntheta: int, nphi: int, out=None,
             noalloc: bool = False):
    """lens_map(alm_T, alm_E, alm_B, alm_phi, lmax, order, grid) -> T', Q', U'
    (FP32, rotation on; Q'/U' None without alm_E).  Synchronizes.
    noalloc=True calls the allocation-free entry point (workspace in the
    library's static device array; out = preallocated (T, Q, U) maps, else
    they are allocated here by torch)."""
    dev = torch.device("cuda", torch.cuda.current_device())
    T = _alm(alm_T, "alm_T", dev, lmax)
    E = _alm(alm_E, "alm_E", dev, lmax)
    B = _alm(alm_B, "alm_B", dev, lmax)
    P = _alm(alm_phi, "alm_phi", dev, lmax)
    if out is None:
        mk = lambda: torch.empty((ntheta, nphi), dtype=torch.float32, device=dev)
        out = (mk(), mk() if E is not None else None, mk() if E is not None else None)
    To, Qo, Uo = out
    torch.cuda.synchronize()
    fn = lib().tl_lens_map_simple_noalloc if noalloc else lib().tl_lens_map_simple
    _check(fn(_ptr(T), _ptr(E), _ptr(B), _ptr(P), int(lmax), int(order), Grid(ntheta, nphi), _ptr(To), _ptr(Qo),
              _ptr(Uo)))
    return To, Qo, Uo


def version() -> int:
    return lib().tl_version()
