#!/usr/bin/env python3
"""Throughput of full-sky Taylor lensing on one MI355X.

One step = one pass of the whole lensing path (deflection synthesis, harmonic
stage of T and Q/U with theta-derivatives, ring FFTs with the phi-derivative
factors, remap + Taylor sum + polarization rotation) over one batch of
realizations whose a_lm are already resident in HBM.  Workload: T+Q/U,
lmax = 4096 on the 4097 x 8192 equal-theta ring grid, Taylor order 4.

Every precision form named by --forms ("fp32", "fp16:5" = FP16 tables, five
realizations per table pass, ...) is timed; ``value`` is the pixel rate of
the --headline form, the others go to ``forms`` with their speed-up over the
FP32 form and their relative RMS error against the FP64 CPU oracle on a band
of output rings.  ``roofline`` describes the headline's dominant kernel, its
average launch duration timed live with HIP events on the plan's stream, its
algorithmic work per launch from the plan's work counts.  ``cpu_baseline`` is
the oracle's rate on that band of rings.

Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import math
import json
import os
import sys
import time

# MI355X published peaks
PEAK = {
    "fp64": 78.6e12,        # FP64 vector (and matrix) FLOP/s
    "fp32_mfma": 157.3e12,  # FP32 matrix FLOP/s
    "f16_mfma": 2.5e15,     # dense FP16 / BF16 matrix FLOP/s
    "hbm": 8.0e12,          # bytes/s
}


def cols(order: int, pol: bool, hasb: bool):
    """Real right-hand-side columns of the L-power contraction per realization."""
    nT = 2 * (order // 2 + 1)
    nE = 2 * (order // 2 + 2) if pol else 0
    nB = nE if (pol and hasb) else 0
    return nT + nE + nB


def direct_flops_per_elem(J: int, spin: bool, hasb: bool):
    """FP64 flops of the direct kernels per (l, m, ring pair) element: the
    Leibniz recursion of the J+1 theta-derivatives, sum_j (2j + 4) + 1, plus
    4 (J+1) per complex right-hand side; two families for spin 2."""
    rec = (J + 1) * (J + 4) + 1
    if not spin:
        return rec + 4 * (J + 1)
    return 2 * (rec + 4 * (J + 1) * (2 if hasb else 1))


def a3_useful_flops(lmax: int, nrp: int, order: int, pol: bool, hasb: bool):
    """Useful flops of the harmonic stage as the plain contraction counts them:
    (N+1) theta-derivative rows times 2 real MACs for T and 8 for Q/U (16 with
    B) per (l, m, ring pair), dense."""
    nlm = (lmax + 1) * (lmax + 2) // 2
    R = 2 + ((16 if hasb else 8) if pol else 0)
    return 2 * nlm * nrp * (order + 1) * R


def stage_work(w, order, form, q, hasb, n, maps16=False):
    """Algorithmic work of each stage per step (n realizations, one table
    pass): (bound, amount, unit, peak).  Harmonic-stage element counts are
    those below the evanescent cut (plan work counts)."""
    nfield = 3 if w.pol else 1
    ndmap = (order + 1) * (order + 2) // 2
    npix = w.ntheta * w.nphi
    rowc = w.ntheta * (w.lmax + 1)
    nlm = (w.lmax + 1) * (w.lmax + 2) // 2
    fp64 = form == "fp64"
    tab = form in ("bf16x3", "fp16x2", "fp16", "bf16")
    # derivative-map bytes per pixel and field (maps16: D_jk with j + k >= 3
    # in FP16, orders >= 3)
    dbytes = ndmap * 8 if fp64 else (6 * 4 + (ndmap - 6) * 2 if maps16 and order >= 3 else ndmap * 4)
    caps = q["elems"] if fp64 else q["elems_caps"]
    cbytes = 16 if fp64 else 8
    # with the lensing potential in the table pass, the direct deflection
    # kernel covers the caps only
    defl = q["elems_caps"] if q["defl_folded"] else q["elems"]
    ncol = cols(order, w.pol, hasb) + (2 if q["defl_folded"] else 0)
    nrn = (w.ntheta + 1) // 2 - q["rpole"]  # ring pairs outside the caps
    colsum = n * ncol * 4 * 4 * nrn * (w.lmax + 1)
    out = {
        "defl_legendre": ("fp64", n * direct_flops_per_elem(1, False, False) * defl),
        "defl_fft": ("hbm", n * (2 * rowc * 16 + 2 * npix * 8)),
        "legendre_T": ("fp64", n * direct_flops_per_elem(order, False, False) * caps),
        "legendre_QU": ("fp64", n * direct_flops_per_elem(order, True, hasb) * caps),
        # the caps in one launch: T, Q/U and (folded) the deflection
        "legendre_caps": ("fp64", n * q["elems_caps"] * (direct_flops_per_elem(order, False, False)
                                                         + (direct_flops_per_elem(order, True, hasb) if w.pol else 0)
                                                         + (direct_flops_per_elem(1, False, False)
                                                            if q["defl_folded"] else 0))),
        "legendre_mfma": ("fp32_mfma", n * (q["elems"] - q["elems_caps"]) * 2 * cols(order, w.pol, hasb) * 2),
        "tab_rhs": ("hbm", n * nlm * 16 * (1 + (2 if hasb else 1) * w.pol + q["defl_folded"])),
        # table stream + the FP32 column sums (4 per column: lam / lam' x parity)
        "legendre_tab": ("hbm", q["tab_chunks"] * q["tab_chunk_bytes"] + colsum),
        # column sums back in, theta-derivative rows (and the potential's FP64 rows) out
        "tab_epi": ("hbm", colsum + n * nfield * (order + 1) * 2 * nrn * (w.lmax + 1) * 8
                    + n * q["defl_folded"] * 2 * 2 * nrn * (w.lmax + 1) * 16),
        "ring_fft": ("hbm", n * (nfield * (order + 1) * rowc * cbytes + nfield * npix * dbytes)),
        "remap": ("hbm", n * (npix * (16 + nfield * 4) + nfield * npix * dbytes)),
    }
    res = {}
    for k, (res_kind, amount) in out.items():
        unit = "GB/s" if res_kind == "hbm" else "TFLOP/s"
        res[k] = (res_kind, float(amount), unit, PEAK[res_kind])
    if tab:
        # the table GEMM also issues f16 MFMA work (useful columns only)
        res["legendre_tab_mfma"] = ("f16_mfma", float((q["elems"] - q["elems_caps"]) * 2 * n * ncol * 2),
                                    "TFLOP/s", PEAK["f16_mfma"])
    return res


def sources_digest():
    """sha256 over the kernel sources (file name, then bytes, sorted)."""
    import glob
    import hashlib

    h = hashlib.sha256()
    for fn in sorted(glob.glob(os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                            "paper_1307_0719_amd", "csrc", "*"))):
        h.update(os.path.basename(fn).encode())
        with open(fn, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(w, fname, kernel):
    """HBM bytes per dispatch of `kernel` from the committed rocprofv3 counter
    summary of this workload and form (FETCH_SIZE and WRITE_SIZE, each scaled
    by what they read for a copy of known size), or None when there is no
    summary, when it names no single matching kernel, or when the kernel
    sources changed since the counters were taken."""
    import re

    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                        f"hbm_traffic_{w}_order4_{fname.replace(':', 'x').replace('+', '_')}.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"sha256 over paper_1307_0719_amd/csrc/\*[^`]*`([0-9a-f]{64})`", text)
    if not m or m.group(1) != sources_digest():
        return None
    rows = re.findall(r"^\| `(" + re.escape(kernel) + r"<[^`]*)` \| \d+ \| [\d.]+ \| [\d.]+ \| ([\d.e+]+) \|$",
                      text, re.M)
    return float(rows[0][1]) if len(rows) == 1 else None


def measured_mfma_busy(w, form, kernel):
    """Matrix-core busy percentage of `kernel` (rocprofv3's MfmaUtil:
    SQ_VALU_MFMA_BUSY_CYCLES over the active cycles of all SIMDs) for this
    workload and form from the committed counter summary, or None when there
    is none, when it names no single matching row, or when the kernel sources
    changed since the counters were taken."""
    import re

    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", f"mfma_{w}_order4.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"sha256 over paper_1307_0719_amd/csrc/\*[^`]*`([0-9a-f]{64})`", text)
    if not m or m.group(1) != sources_digest():
        return None
    rows = re.findall(r"^\| " + re.escape(form) + r" \| `" + re.escape(kernel) + r"<[^`]*` \| \d+ \| [\d.]+ \| [\d.]+ \| ([\d.]+) \|",
                      text, re.M)
    return float(rows[0]) if len(rows) == 1 else None


def parse_form(s: str):
    """'prec[:batch][+m16]' -> (prec, batch, maps16)."""
    s, plus, opt = s.partition("+")
    if plus and opt != "m16":
        raise ValueError(f"unknown form option +{opt}")
    prec, _, b = s.partition(":")
    return prec, int(b) if b else 1, bool(plus)


def form_name(f):
    return (f[0] if f[1] == 1 else f"{f[0]}:{f[1]}") + ("+m16" if f[2] else "")


def run_form(args, w, order, prec, batch, skies_dev, maps16=False):
    import torch

    from paper_1307_0719_amd import taylens

    torch.cuda.synchronize()
    b0 = time.perf_counter()
    plan = taylens.Plan(w.lmax, w.ntheta, w.nphi, order, prec, pol=w.pol, batch=batch if batch > 1 else 0,
                        maps16=maps16)
    torch.cuda.synchronize()
    plan_s = time.perf_counter() - b0
    q = {k: plan.query(k) for k in taylens.QUERY_KEYS}
    outs = [(plan._maps(), plan._maps() if w.pol else None, plan._maps() if w.pol else None) for _ in range(batch)]
    alms = skies_dev[:batch]

    def step():
        if batch == 1:
            a = alms[0]
            plan.lens_map(a[0], a[1], a[2], a[3], out=outs[0])
        else:
            plan.lens_map_many(alms, outs)

    for _ in range(args.warmup):
        step()
    # timed region: K whole steps, an event pair around each on the plan's
    # stream (torch's current stream); ms per step = the median
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record()
    for i in range(args.steps):
        step()
        ev[i + 1].record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / args.steps
    per = sorted(ev[i].elapsed_time(ev[i + 1]) * 1e-3 for i in range(args.steps))
    sec = per[len(per) // 2] if len(per) % 2 else 0.5 * (per[len(per) // 2 - 1] + per[len(per) // 2])
    # the same K steps again with a HIP event pair around every kernel launch
    plan.profile(True)
    for _ in range(args.steps):
        step()
    st = plan.stage_times()
    plan.profile(False)
    per_step = {k: v[0] / args.steps for k, v in st.items() if v[1]}
    avg_launch = {k: v[0] / v[1] for k, v in st.items() if v[1]}
    launches = {k: v[1] // args.steps for k, v in st.items() if v[1]}
    ws = plan.workspace_bytes()
    first = tuple(x.cpu().numpy() if x is not None else None for x in outs[0])
    del outs
    plan.close()
    torch.cuda.empty_cache()
    return {"sec": sec, "wall_mean_sec": wall, "step_sec_min_max": (per[0], per[-1]), "per_step": per_step,
            "avg_launch": avg_launch, "launches": launches, "q": q, "workspace_bytes": ws, "plan_build_s": plan_s,
            "maps0": first}


def bench_batch(args, order=4, n=64):
    """The uneven-lmax batch: n T+Q/U realizations, lmax drawn from
    {512, 1024, 2048, 3000} (seeded), grids (lmax+1) x 2 lmax, FP32 form, one
    tl_batch pass per step (persistent harmonic launch, graph replay,
    autotuned work items; the first run, which tunes and captures, is part of
    the warm-up)."""
    import numpy as np
    import torch

    from paper_1307_0719_amd import skygen, taylens

    lm = skygen.batch_lmaxes(n, seed=3)
    dev = torch.device("cuda", 0)
    plans = {L: taylens.Plan(L, L + 1, 2 * L, order, "fp32", pol=True) for L in sorted(set(lm))}
    alms = []
    for i, L in enumerate(lm):
        s = skygen.make_sky(L, 3000 + i, pol=True)
        alms.append(tuple(None if a is None else torch.from_numpy(a).to(dev)
                          for a in (s.alm_T, s.alm_E, None, s.alm_phi)))
    b = taylens.Batch([plans[L] for L in lm], autotune=True, use_graph=True)
    outs = b.outputs()
    for _ in range(max(1, args.warmup)):
        b.run(alms, outs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        b.run(alms, outs)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / args.steps
    info = b.info()
    npix = sum((L + 1) * 2 * L for L in lm)
    # MFMA work of the persistent launch (useful columns, elements outside the caps)
    fl = 0.0
    for L in lm:
        q = {k: plans[L].query(k) for k in ("elems", "elems_caps")}
        fl += (q["elems"] - q["elems_caps"]) * 2 * cols(order, True, False) * 2
    res = {"realizations": n, "lmax_counts": {str(L): lm.count(L) for L in sorted(set(lm))},
           "pixels_per_step": npix, "ms_per_step": sec * 1e3, "pixels_per_s": npix / sec,
           "autotuned_item": {"m_per_item": 8 * info["m_groups"], "workgroups_per_cu": info["groups_per_cu"],
                              "tuned_harmonic_launch_ms": info["tuned_ms"]},
           "graph_replays": info["graph_replays"],
           "persistent_launch_fp32_mfma_tflops": fl / (info["tuned_ms"] * 1e-3) / 1e12 if info["tuned_ms"] else None}
    b.close()
    for p in plans.values():
        p.close()
    torch.cuda.empty_cache()
    return res


def bench_cnn(args, w, precision="fp16x2"):
    """Order 2 + learned correction at the workload's size (weights shipped
    with the package) in the given precision form, its forward kernel against
    the BF16 matrix peak, beside plain orders 2, 3, 4 and 6 in the same form
    (ms per map, one realization per call), and the RMS error of each against
    plain order 6 (FP32 form) on two held-out skies."""
    import numpy as np
    import torch

    from paper_1307_0719_amd import skygen, train_cnn, taylens

    here = os.path.dirname(os.path.abspath(__file__))
    params = np.load(os.path.join(here, "paper_1307_0719_amd", "cnn_weights.npy"))
    dev = torch.device("cuda", 0)
    s = skygen.make_sky(w.lmax, w.seed, pol=True)
    a = tuple(None if x is None else torch.from_numpy(x).to(dev) for x in (s.alm_T, s.alm_E, None, s.alm_phi))
    npix = w.ntheta * w.nphi

    def timed(run):
        for _ in range(args.warmup):
            run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            run()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / args.steps

    ms = {}
    plan = taylens.Plan(w.lmax, w.ntheta, w.nphi, 2, precision, pol=True)
    net = taylens.Cnn(params)
    outs = (plan._maps(), plan._maps(), plan._maps())
    sec = timed(lambda: net.lens_map(plan, *a, out=outs))
    plan.profile(True)
    for _ in range(args.steps):
        net.lens_map(plan, *a, out=outs)
    st = plan.stage_times()
    plan.profile(False)
    cnn_ms = st["cnn"][0] / st["cnn"][1]
    ms["order2_plus_cnn"] = sec * 1e3
    ms["order2"] = timed(lambda: plan.lens_map(*a, out=outs)) * 1e3
    net.close()
    plan.close()
    del outs
    torch.cuda.empty_cache()
    for N in (3, 4, 6):
        pn = taylens.Plan(w.lmax, w.ntheta, w.nphi, N, precision, pol=True)
        o = (pn._maps(), pn._maps(), pn._maps())
        ms[f"order{N}"] = timed(lambda: pn.lens_map(*a, out=o)) * 1e3
        pn.close()
        del o
        torch.cuda.empty_cache()
    flops = 2 * 61152 * npix  # MACs per pixel of the three layers (useful, unpadded)
    ev = train_cnn.evaluate(params, w.lmax, w.ntheta, w.nphi, [20000, 20001], precision=precision,
                            plain_orders=(3, 4))
    errs = {"order2": ev["rms_err_order2"], "order2_plus_cnn": ev["rms_err_cnn"],
            "order3": ev["rms_err_order3"], "order4": ev["rms_err_order4"]}
    return {"precision_form": precision, "pixels_per_s": npix / (ms["order2_plus_cnn"] * 1e-3),
            "ms_per_map": ms, "cnn_forward_ms": cnn_ms,
            "cnn_forward_bf16_tflops": flops / (cnn_ms * 1e-3) / 1e12,
            "cnn_forward_mfma_frac": flops / (cnn_ms * 1e-3) / PEAK["f16_mfma"],
            "rms_err_vs_order6": errs, "rms_signal": ev["rms_signal"], "gain_over_order2": ev["gain"],
            "held_out_seeds": ev["seeds"]}


def bench_healpix(args, with_oracle, precision="fp16x2", nside=2048, lmax=3072, order=2, batch=6):
    """Lensing onto and from HEALPix rings (the paper's pixelization): nside
    2048, lmax 3072, order 2 -- a row of the paper's fastest-settings table
    (32.5 CPU-minutes per map on 8-core Xeon E5540 nodes; at lmax 4096 the
    split tables of 8191 HEALPix rings take 258 GiB, too much beside six
    realizations' work buffers) -- six realizations per table pass.  Rate in lensed HEALPix pixels per second;
    error against the HEALPix oracle on two sampled rings (a 4-pixel polar ring
    and the equator) of realization 0."""
    import numpy as np
    import torch

    from paper_1307_0719_amd import skygen, taylens

    dev = torch.device("cuda", 0)
    skies = [skygen.make_sky(lmax, 2 + i, pol=True) for i in range(batch)]
    skies_dev = [tuple(None if x is None else torch.from_numpy(x).to(dev) for x in (s.alm_T, s.alm_E, None, s.alm_phi))
                 for s in skies]
    plan = taylens.Plan(lmax, 0, 0, order, precision, pol=True, nside=nside, batch=batch if batch > 1 else 0)
    outs = [(plan._maps(), plan._maps(), plan._maps()) for _ in range(batch)]
    alms = skies_dev[:batch]
    for _ in range(args.warmup):
        plan.lens_map_many(alms, outs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.lens_map_many(alms, outs)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / args.steps
    plan.profile(True)
    for _ in range(args.steps):
        plan.lens_map_many(alms, outs)
    st = plan.stage_times()
    plan.profile(False)
    npix = 12 * nside * nside
    res = {"nside": nside, "lmax": lmax, "order": order, "precision_form": precision,
           "realizations_per_step": batch, "ms_per_step": sec * 1e3, "pixels_per_s": batch * npix / sec,
           "stages_ms_per_step": {k: round(v[0] / args.steps, 3) for k, v in st.items() if v[1]},
           "paper_context": "Taylens at nside 2048, lmax 3072, order 2: 32.5 CPU-minutes per map on 8-core "
                            "Xeon E5540 nodes (25,811 pixels per CPU-second)"}
    if with_oracle:
        from oracle import healpix_oracle as hp

        ncores = min(16, os.cpu_count() or 1)
        rings = np.array([0, 2 * nside - 1])
        pix = hp.ring_pixels(nside, rings)
        s0 = skies[0]
        ref = hp.lens_pixels(lmax, order, nside, pix, s0.alm_T, s0.alm_E, s0.alm_B, s0.alm_phi, nthreads=ncores)
        ok = hp.ang2pix(nside, ref["_thp"] + 1e-12, ref["_php"] + 1e-12) == ref["_src"]
        idx = torch.from_numpy(pix).to(outs[0][0].device)
        errs = {}
        for f, g in zip("TQU", outs[0]):
            x = g[idx].cpu().numpy()[ok]
            y = ref[f][ok]
            errs[f] = float(np.sqrt(np.mean((x - y) ** 2)) / np.sqrt(np.mean(y ** 2)))
        res["rel_rms_err_vs_oracle"] = errs
        res["oracle_sample"] = f"rings {rings.tolist()} ({pix.size} pixels) of realization 0"
    del outs
    plan.close()
    torch.cuda.empty_cache()
    return res


def sweep_sample(lmax: int, nring: int = 16, ncol: int = 32):
    """Sky positions of the accuracy sweep, as (ring, column) on the grid of
    oversampling 1 (lmax + 1 rings of 2 lmax pixels): nring rings from the
    second ring to the equator and beyond, ncol columns each.  On the grid of
    oversampling g the same positions are (g ring, g column)."""
    import numpy as np

    nt = lmax + 1
    rings = np.unique(np.round(np.linspace(1, nt - 2, nring)).astype(np.int64))
    cols = (np.arange(ncol) * (2 * lmax) // ncol + 3) % (2 * lmax)
    R, C = np.meshgrid(rings, cols, indexing="ij")
    return R.ravel(), C.ravel()


def sweep_best(rows, targets=(1e-2, 1e-3, 1e-4, 1e-5, 1e-6)):
    """For each lmax (and band limit of the potential) and error target,
    the fastest row (time per map) whose worst field error is within the
    target: the structure of the paper's fastest-settings table."""
    out = []
    key = lambda r: (r["lmax"], r.get("lmax_phi", r["lmax"]))
    for lmax, lphi in sorted({key(r) for r in rows}):
        for t in targets:
            ok = [r for r in rows if key(r) == (lmax, lphi) and r["rel_rms_err_max"] <= t]
            if not ok:
                out.append({"lmax": lmax, "lmax_phi": lphi, "target": t, "row": None})
                continue
            b = min(ok, key=lambda r: r["ms_per_map"])
            out.append({"lmax": lmax, "lmax_phi": lphi, "target": t,
                        "row": {k: b[k] for k in ("oversampling", "order", "form", "ms_per_map", "rel_rms_err_max")}})
    return out


def bench_sweep(args):
    """Accuracy against time on the GPU (the structure of the paper's timing
    sweep and fastest-settings table, Sec. III.B): for each lmax, grid
    oversampling g (g lmax + 1 rings of 2 g lmax pixels) and Taylor order,
    the time per lensed T+Q/U map of the FP32 form and of the split-FP16
    form with six realizations per table pass (FP16 maps of order >= 3;
    skipped where its tables do not fit), and the relative RMS error of realization 0 against the exact
    lensed field (the unlensed field synthesized at each displaced position,
    rotated) at a fixed sample of sky positions shared by every grid.  With
    a phi factor F > 1 the lensing potential has its own band limit F lmax
    (lmax_phi, on grids of oversampling >= F), the paper's higher band limit
    of the deflection."""
    import numpy as np
    import torch

    from oracle import taylens_oracle as orc
    from paper_1307_0719_amd import skygen, taylens

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:
        nproc = os.cpu_count() or 1
    ncores = min(16, nproc)
    lmaxes = [int(x) for x in args.sweep_lmax.split(",")]
    gs = [int(x) for x in args.sweep_oversampling.split(",")]
    orders = [int(x) for x in args.sweep_orders.split(",")]
    phifs = [int(x) for x in args.sweep_phi_factor.split(",")]
    rows = []
    for lmax, fphi in [(l, f) for l in lmaxes for f in phifs]:
        lphi = fphi * lmax  # the potential's band limit: rings of 2 g lmax >= 2 lmax_phi points
        gl = [g for g in gs if g >= fphi]
        if not gl:
            continue
        skies = [skygen.make_sky(lmax, 30 + i, pol=True) for i in range(6)]
        if fphi > 1:
            for i, s in enumerate(skies):
                s.alm_phi = skygen.make_sky(lphi, 40 + i, pol=False).alm_phi
        to_dev = lambda a: None if a is None else torch.from_numpy(a).to(dev)
        sdev = [(to_dev(s.alm_T), to_dev(s.alm_E), None, to_dev(s.alm_phi)) for s in skies]
        R, C = sweep_sample(lmax)
        s0 = skies[0]
        o0 = time.perf_counter()
        # the same sky positions on the coarsest grid that carries the potential
        g0 = min(gl)
        ex = orc.exact_lensed_pixels(lmax, g0 * lmax + 1, 2 * g0 * lmax, g0 * R, g0 * C, s0.alm_T, s0.alm_E, None,
                                     s0.alm_phi, nthreads=ncores)
        oracle_s = time.perf_counter() - o0
        print(f"sweep lmax {lmax} lmax_phi {lphi}: exact reference at {R.size} positions in {oracle_s:.1f} s",
              file=sys.stderr, flush=True)
        for g in gl:
            nt, nph = g * lmax + 1, 2 * g * lmax
            idx = torch.from_numpy(g * R * nph + g * C).to(dev)
            forms = [("fp32", 1), ("fp16x2", 6)]
            for order in orders:
                for prec, batch in forms:
                    try:
                        plan = taylens.Plan(lmax, nt, nph, order, prec, pol=True, batch=batch if batch > 1 else 0,
                                            maps16=prec != "fp32", lmax_phi=lphi)
                    except taylens.TaylensError as e:
                        rows.append({"lmax": lmax, "lmax_phi": lphi, "oversampling": g, "order": order, "form": prec,
                                     "skipped": str(e)})
                        continue
                    outs = [(plan._maps(), plan._maps(), plan._maps()) for _ in range(batch)]

                    def step():
                        if batch == 1:
                            a = sdev[0]
                            plan.lens_map(a[0], a[1], a[2], a[3], out=outs[0])
                        else:
                            plan.lens_map_many(sdev[:batch], outs)

                    step()
                    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
                    torch.cuda.synchronize()
                    ev[0].record()
                    for i in range(args.steps):
                        step()
                        ev[i + 1].record()
                    torch.cuda.synchronize()
                    per = sorted(ev[i].elapsed_time(ev[i + 1]) for i in range(args.steps))
                    ms = per[len(per) // 2]
                    errs = {}
                    for f, t in zip("TQU", outs[0]):
                        x = t.view(-1)[idx].double().cpu().numpy()
                        y = ex[f]
                        errs[f] = float(np.sqrt(np.mean((x - y) ** 2)) / np.sqrt(np.mean(y ** 2)))
                    rows.append({"lmax": lmax, "lmax_phi": lphi, "oversampling": g, "ntheta": nt, "nphi": nph,
                                 "order": order,
                                 "form": prec if batch == 1 else f"{prec}:{batch}+m16",
                                 "ms_per_map": ms / batch, "pixels_per_s": batch * nt * nph / (ms * 1e-3),
                                 "rel_rms_err": errs, "rel_rms_err_max": max(errs.values())})
                    print(f"sweep lmax {lmax}/{lphi} g {g} order {order} {rows[-1]['form']}: {ms / batch:.2f} ms/map, "
                          f"err {rows[-1]['rel_rms_err_max']:.2e}", file=sys.stderr, flush=True)
                    del outs
                    plan.close()
                    torch.cuda.empty_cache()
    return {"metric": "accuracy vs time per lensed map (T+Q/U)", "unit": "ms per map",
            "reference": "exact lensed field at the sampled positions (unlensed field synthesized at each "
                         "displaced position, rotated), FP64 oracle",
            "sample": "16 rings x 32 columns on the oversampling-1 grid, the same sky positions on every grid",
            "deflection_rms_arcmin": skygen.DEFLECTION_RMS_ARCMIN, "steps": args.steps,
            "rows": rows, "fastest": sweep_best([r for r in rows if "skipped" not in r])}


def bench_theta_fft(args, lmax=4095, ntheta=4097, nphi=8192, order=4, reps=7):
    """Theta-derivatives by FFT along the great circles through both poles
    (tl_theta_derivs) on the 4097 x 8192 grid of lmax 4095: the j >= 1
    derivative maps of one field at order 4 (10 maps, from D_{0,k}, k <= 3),
    FP32 and FP64 maps; median of reps, the algorithmic HBM bytes (inputs
    read once, outputs written once) and their rate against 8 TB/s."""
    import statistics

    import torch

    from paper_1307_0719_amd import taylens as tl

    res = {"workload": f"{ntheta} x {nphi} rings (lmax {lmax}), order {order}: the {order * (order + 1) // 2} "
                       f"maps D_jk, j >= 1, of one field from its D_0k, k < {order}"}
    for prec in ("fp32", "fp64"):
        plan = tl.Plan(lmax, ntheta, nphi, 1, prec, pol=False)
        g = torch.Generator(device="cuda").manual_seed(5)
        maps = torch.randn((order, ntheta, nphi), generator=g, dtype=plan.real_dtype, device="cuda")
        outs = []

        def step():
            outs.clear()
            for k in range(order):
                outs.append(plan.theta_derivs(maps[k], order - k))

        step()
        torch.cuda.synchronize()
        times = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(plan.stream)
            step()
            b.record(plan.stream)
            b.synchronize()
            times.append(a.elapsed_time(b))
        ms = statistics.median(times)
        nout = order * (order + 1) // 2
        nbytes = (order + nout) * ntheta * nphi * maps.element_size()
        res[prec] = {"ms": round(ms, 4), "maps_in": order, "maps_out": nout, "algorithmic_bytes": nbytes,
                     "hbm_gbs": round(nbytes / ms / 1e6, 1), "frac_of_8tbs": round(nbytes / ms / 1e6 / 8000.0, 4)}
        del plan, maps, outs
        torch.cuda.empty_cache()

    # the FP64 form lensing T+Q/U at order 4 with the theta-derivatives from
    # the recursion (every row j) and from the FFTs (rows j = 0 only)
    from paper_1307_0719_amd import skygen

    sky = skygen.make_sky(lmax, 41, pol=True)
    a = (sky.alm_T, sky.alm_E, None, sky.alm_phi)
    fp64 = {"workload": f"T+Q/U lmax {lmax} on {ntheta} x {nphi} rings, order {order}, FP64 form, tl_lens_map"}
    maps = {}
    for tf in (False, True):
        plan = tl.Plan(lmax, ntheta, nphi, order, "fp64", pol=True, theta_fft=tf)
        out = plan.lens_map(*a)
        torch.cuda.synchronize()
        times = []
        for _ in range(3):
            t0 = torch.cuda.Event(enable_timing=True)
            t1 = torch.cuda.Event(enable_timing=True)
            t0.record(plan.stream)
            plan.lens_map(*a, out=out)
            t1.record(plan.stream)
            t1.synchronize()
            times.append(t0.elapsed_time(t1))
        plan.profile(True)
        plan.lens_map(*a, out=out)
        st = {k: round(v[0], 2) for k, v in plan.stage_times().items() if v[1]}
        plan.profile(False)
        key = "theta_fft" if tf else "recursion"
        fp64[key] = {"ms_per_map": round(statistics.median(times), 2), "stages_ms": st}
        maps[key] = [x.clone() for x in out]
        del plan, out
        torch.cuda.empty_cache()
    fp64["max_rel_rms_difference"] = max(
        float(torch.sqrt(torch.mean((x - y) ** 2)) / torch.sqrt(torch.mean(y ** 2)))
        for x, y in zip(maps["theta_fft"], maps["recursion"]))
    fp64["speedup"] = round(fp64["recursion"]["ms_per_map"] / fp64["theta_fft"]["ms_per_map"], 3)
    res["fp64_lens_map"] = fp64
    return res


def spectra_cl(alm, lmax):
    """C_l = (|a_l0|^2 + 2 sum_{m>0} |a_lm|^2) / (2l + 1) from triangular a_lm."""
    import numpy as np

    p = np.abs(np.asarray(alm)) ** 2
    cl = np.zeros(lmax + 1)
    for m in range(lmax + 1):
        off = m * (2 * lmax + 1 - m) // 2
        cl[m:] += p[off + m: off + lmax + 1] * (1.0 if m == 0 else 2.0)
    return cl / (2.0 * np.arange(lmax + 1) + 1.0)


def spectra_bins(cl, lmin=2, width=50):
    """Centres and means of C_l over bins of `width` multipoles from lmin."""
    import numpy as np

    cl = np.asarray(cl, dtype=np.float64)
    nb = (len(cl) - lmin) // width
    edges = lmin + width * np.arange(nb + 1)
    return 0.5 * (edges[:-1] + edges[1:] - 1), np.array([cl[edges[b]:edges[b + 1]].mean() for b in range(nb)])


def spectra_ell_star(centres, rel_err, limit=0.005, nsigma=4.0):
    """Sec. III.B: the centre of the last bin before the first whose mean
    relative error exceeds `limit` by more than `nsigma` standard errors of
    the mean over the simulations (None if the first bin fails)."""
    import numpy as np

    e = np.atleast_2d(np.asarray(rel_err, dtype=np.float64))
    mean = e.mean(axis=0)
    sem = e.std(axis=0, ddof=1) / np.sqrt(e.shape[0]) if e.shape[0] > 1 else np.zeros(e.shape[1])
    bad = np.abs(mean) - limit > nsigma * sem
    if not bad.any():
        return float(centres[-1])
    first = int(np.argmax(bad))
    return None if first == 0 else float(centres[first - 1])


def bench_spectra(args, lmax=2048, ntheta=4097, nphi=8192, orders=(0, 1, 2, 3, 4), nsim=4):
    """The lensed-spectrum accuracy measure of Sec. III.A-B on synthetic
    skies: T maps lensed at orders 0..4 (FP32 form) and at order 8 (FP64
    form, the reference) on the twice-oversampled 4097 x 8192 grid of lmax
    2048, analysed by tl_analysis_T (exact for the unlensed band limit on
    this grid), C_l in bins of 50 multipoles, the relative error of each
    order's binned spectrum against the reference's on the same sky, and
    l* (the last bin not above 0.5 % by more than 4 standard errors of the
    mean over nsim skies)."""
    import numpy as np
    import torch

    from paper_1307_0719_amd import skygen
    from paper_1307_0719_amd import taylens as tl

    def cl_of(alm):
        return spectra_cl(alm.cpu().numpy(), lmax)

    ana = tl.Plan(lmax, ntheta, nphi, 1, "fp64", pol=False)
    ref_plan = tl.Plan(lmax, ntheta, nphi, 8, "fp64", pol=False)
    plans = {N: tl.Plan(lmax, ntheta, nphi, N, "fp32", pol=False) for N in orders}
    errs = {N: [] for N in orders}
    t_ana = []
    centres = None
    for i in range(nsim):
        sky = skygen.make_sky(lmax, 900 + i, pol=False)
        ref = ref_plan.lens_map(sky.alm_T, None, None, sky.alm_phi)[0]
        a0 = torch.cuda.Event(enable_timing=True)
        a1 = torch.cuda.Event(enable_timing=True)
        a0.record(ana.stream)
        alm_ref = ana.analysis_T(ref)
        a1.record(ana.stream)
        a1.synchronize()
        t_ana.append(a0.elapsed_time(a1))
        centres, b_ref = spectra_bins(cl_of(alm_ref))
        for N, p in plans.items():
            T = p.lens_map(sky.alm_T, None, None, sky.alm_phi)[0].double()
            _, b = spectra_bins(cl_of(ana.analysis_T(T)))
            errs[N].append(b / b_ref - 1.0)
        print(f"spectra: sky {i + 1}/{nsim}", file=sys.stderr, flush=True)
    out = {"workload": f"T lensed at lmax {lmax} on {ntheta} x {nphi} rings, orders {list(orders)} (FP32 form) "
                       f"against order 8 (FP64 form) on the same {nsim} synthetic skies, bins of 50 multipoles",
           "analysis_ms": round(float(np.median(t_ana)), 3), "bin_centres": [float(c) for c in centres],
           "orders": {}}
    for N in orders:
        e = np.array(errs[N])
        out["orders"][str(N)] = {"ell_star": spectra_ell_star(centres, e),
                                 "mean_rel_err": [float(x) for x in e.mean(axis=0)]}
    return out


def deflection_check(w, skies, skies_dev):
    """The deflection field of the step's realizations, from the library's
    deflection entry point (direct FP64 synthesis of grad phi): its RMS |alpha|
    over the sphere (ring weights sin theta) against the value Parseval's
    identity gives for each realization's a_lm, sum_lm l(l+1)|phi_lm|^2 / 4 pi,
    and the mean over the realizations against the 2.5' the spectra are scaled
    to (the harness assertion: within 2 %).  Then the residual distribution
    of realization 0 (the paper's interpolation-distance diagnostic): the
    displaced position of every pixel relative to its nearest pixel centre,
    |dtheta|/dtheta_grid and |dphi|/dphi_grid, histogrammed in ten bins of
    [0, 1/2]; the share of pixels whose nearest centre is another pixel; the
    99 % quantile of |alpha|."""
    import numpy as np
    import torch

    from paper_1307_0719_amd import skygen, taylens

    dev = torch.device("cuda", 0)
    plan = taylens.Plan(w.lmax, w.ntheta, w.nphi, 1, "fp64", pol=False)
    th = torch.arange(w.ntheta, device=dev, dtype=torch.float64) * (math.pi / (w.ntheta - 1))
    wt = torch.sin(th)[:, None]
    ls, ms = skygen.lm_arrays(w.lmax)
    mult = np.where(ms == 0, 1.0, 2.0) * ls * (ls + 1.0)
    rows = []
    hist = None
    for i, (s, a) in enumerate(zip(skies, skies_dev)):
        at, ap = plan.deflection(a[3])
        a2 = at * at + ap * ap
        rms = math.sqrt(float((a2 * wt).sum() / (wt.sum() * w.nphi))) / skygen.ARCMIN
        pars = math.sqrt(float(np.sum(mult * np.abs(s.alm_phi) ** 2)) / (4 * math.pi)) / skygen.ARCMIN
        rows.append({"seed": s.seed, "rms_arcmin": rms, "parseval_arcmin": pars})
        if i == 0:
            ph = torch.arange(w.nphi, device=dev, dtype=torch.float64) * (2 * math.pi / w.nphi)
            st, ct = torch.sin(th)[:, None], torch.cos(th)[:, None]
            sp, cp = torch.sin(ph)[None, :], torch.cos(ph)[None, :]
            d = torch.sqrt(a2)
            sd = torch.where(d > 0, torch.sin(d) / torch.where(d > 0, d, torch.ones_like(d)), torch.ones_like(d))
            cd = torch.cos(d)
            # x' = cos d x + sin d (a_t e_t + a_p e_p) / d
            xx = cd * st * cp + sd * (at * ct * cp - ap * sp)
            yy = cd * st * sp + sd * (at * ct * sp + ap * cp)
            zz = cd * ct - sd * at * st
            thp = torch.atan2(torch.hypot(xx, yy), zz)
            php = torch.remainder(torch.atan2(yy, xx), 2 * math.pi)
            tt = thp / (math.pi / (w.ntheta - 1))
            tp = php / (2 * math.pi / w.nphi)
            it, ip = torch.floor(tt + 0.5), torch.floor(tp + 0.5)
            ut, up = (tt - it).abs(), (tp - ip).abs()
            moved = ((it != torch.arange(w.ntheta, device=dev)[:, None])
                     | (torch.remainder(ip, w.nphi) != torch.arange(w.nphi, device=dev)[None, :]))
            edges = [0.05 * k for k in range(11)]
            hist = {"bin_edges": edges,
                    "dtheta_over_pixel": [float(x) for x in torch.histc(ut.float(), 10, 0.0, 0.5).cpu() / ut.numel()],
                    "dphi_over_pixel": [float(x) for x in torch.histc(up.float(), 10, 0.0, 0.5).cpu() / up.numel()],
                    "share_moved_to_another_pixel": float(moved.double().mean()),
                    "alpha_q99_arcmin": float(torch.quantile(d.flatten()[::97].float(), 0.99)) / skygen.ARCMIN,
                    "max_residual_over_pixel": [float(ut.max()), float(up.max())]}
            del xx, yy, zz, thp, php, tt, tp, it, ip, ut, up, moved, d
        del at, ap, a2
    plan.close()
    torch.cuda.empty_cache()
    mean = sum(r["rms_arcmin"] for r in rows) / len(rows)
    quad_ok = all(abs(r["rms_arcmin"] / r["parseval_arcmin"] - 1) < 5e-3 for r in rows)
    target_ok = abs(mean / skygen.DEFLECTION_RMS_ARCMIN - 1) <= 0.02
    res = {"target_arcmin": skygen.DEFLECTION_RMS_ARCMIN, "mean_rms_arcmin": mean, "per_realization": rows,
           "within_2pct_of_target": target_ok, "matches_parseval_0p5pct": quad_ok, "residuals_realization0": hist}
    assert quad_ok and target_ok, ("deflection RMS check failed", res)
    return res


def copy_calibration(args):
    """A plain device copy of known size, for scaling the HBM byte counters."""
    import torch

    n = 1 << 28  # floats: 1 GiB
    a = torch.ones(n, device="cuda")
    b = torch.empty_like(a)
    for _ in range(max(1, args.steps)):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "launches": max(1, args.steps)}))


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="TP4096")
    ap.add_argument("--order", type=int, default=None)
    ap.add_argument("--forms", default="fp32,bf16:6,fp16:6,bf16x3:6,fp16x2:6,fp16x2:6+m16",
                    help="comma list of precision[:realizations per step][+m16 (FP16 maps of order >= 3)]; "
                         "fp32 is the speed-up reference")
    ap.add_argument("--headline", default=None, help="form reported as value (default: the last of --forms)")
    ap.add_argument("--cpu-rings", type=int, default=40, help="output rings in the CPU-oracle sample (five bands)")
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the oracle (no errors, no cpu_baseline)")
    ap.add_argument("--copy-calibration", action="store_true", help="only run a 1 GiB device copy (counter scale)")
    ap.add_argument("--healpix-only", action="store_true",
                    help="only the HEALPix leg (nside 2048, lmax 3072, order 2, split FP16, six per pass), "
                         "without the oracle; one JSON line")
    ap.add_argument("--spectra", action="store_true",
                    help="only the lensed-spectrum accuracy measure (T, lmax 2048, orders 0-4 against order 8, "
                         "bins of 50, l*); one JSON line")
    ap.add_argument("--theta-fft-only", action="store_true",
                    help="only the theta-derivative FFTs (tl_theta_derivs) on the 4097 x 8192 grid; one JSON line")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the uneven-lmax batch and the learned-correction measurements")
    ap.add_argument("--sweep", action="store_true",
                    help="only the accuracy-vs-time sweep (lmax x grid oversampling x order against the exact "
                         "lensed field); one JSON line")
    ap.add_argument("--sweep-lmax", default="1024,2048,4096")
    ap.add_argument("--sweep-oversampling", default="1,2")
    ap.add_argument("--sweep-orders", default="1,2,3,4,5,6")
    ap.add_argument("--sweep-phi-factor", default="1,2",
                    help="lmax_phi / lmax of the lensing potential (rows on grids of oversampling >= the factor)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "independent realizations would shard across GPUs without communication.", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration(args)
        return
    if args.healpix_only:
        print(json.dumps(bench_healpix(args, False)))
        return
    if args.sweep:
        print(json.dumps(bench_sweep(args)))
        return
    if args.theta_fft_only:
        print(json.dumps(bench_theta_fft(args)))
        return
    if args.spectra:
        print(json.dumps(bench_spectra(args)))
        return

    import numpy as np
    import torch

    from paper_1307_0719_amd import skygen

    w = skygen.WORKLOADS[args.workload]
    order = w.order if args.order is None else args.order
    forms = [parse_form(f) for f in args.forms.split(",") if f]
    headline = parse_form(args.headline) if args.headline else forms[-1]
    if headline not in forms:
        forms.append(headline)
    nmax = max(f[1] for f in forms)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    skies = [skygen.make_sky(w.lmax, w.seed + i, pol=w.pol) for i in range(nmax)]
    to_dev = lambda a: None if a is None else torch.from_numpy(a).to(dev)
    # B = 0 in these workloads: pass NULL (the library then skips the B sums)
    hasb = any(s.alm_B is not None and np.any(s.alm_B) for s in skies)
    skies_dev = [(to_dev(s.alm_T), to_dev(s.alm_E), to_dev(s.alm_B) if hasb else None, to_dev(s.alm_phi))
                 for s in skies]
    npix = w.ntheta * w.nphi

    # oracle on five bands of output rings of realization 0: inside the polar
    # cap (direct FP64 kernels), across the cap boundary (sin theta = 0.15,
    # where the reduced forms' epilogue amplifies most), mid-latitude, equator
    ref, rings, cpu, bands = None, None, None, None
    if not args.no_cpu_baseline:
        from oracle import taylens_oracle as orc

        try:
            nproc = len(os.sched_getaffinity(0))
        except AttributeError:
            nproc = os.cpu_count() or 1
        ncores = min(16, nproc)
        nb = max(1, args.cpu_rings // 5)

        def first_ring(smin):
            e = 1
            while e < w.ntheta // 2 and math.sin(math.pi * e / (w.ntheta - 1)) < smin:
                e += 1
            return e

        # caps end at sin theta 0.05 (split FP16 form) or 0.15 (the others)
        e1, e2 = first_ring(0.05), first_ring(0.15)
        starts = {"cap": min(4, e1 - nb) if e1 > nb else 0, "cap_edge_0.05": max(0, e1 - nb // 2),
                  "cap_edge_0.15": max(0, e2 - nb // 2),
                  "mid_latitude": w.ntheta // 4, "equator": w.ntheta // 2 - nb // 2}
        bands = {k: np.arange(v, v + nb) for k, v in starts.items()}
        rings = np.unique(np.concatenate(list(bands.values())))
        nr = len(rings)
        s0 = skies[0]
        o0 = time.perf_counter()
        ref = orc.lens_rings(w.lmax, order, w.ntheta, w.nphi, rings, s0.alm_T, s0.alm_E, s0.alm_B, s0.alm_phi,
                             nthreads=ncores)
        o1 = time.perf_counter()
        # the same oracle on one thread, on the first four equator rings
        r1 = bands["equator"][:4]
        orc.lens_rings(w.lmax, order, w.ntheta, w.nphi, r1, s0.alm_T, s0.alm_E, s0.alm_B, s0.alm_phi, nthreads=1)
        o2 = time.perf_counter()
        cpu = {
            "value": nr * w.nphi / (o1 - o0), "unit": "pixels/s", "cores": ncores, "kind": "oracle",
            "nproc": nproc, "os_cpu_count": os.cpu_count(),
            "sample": f"{nr} output rings of realization 0 in five bands of {nb} "
                      f"({', '.join(f'{k} from {v}' for k, v in starts.items())}): deflection on those rings, "
                      f"derivative maps of every source ring they need, remap, Taylor sum, rotation; "
                      f"{o1 - o0:.1f} s, FP64, {ncores} threads",
            "value_1core": len(r1) * w.nphi / (o2 - o1),
            "sample_1core": f"rings {int(r1[0])}..{int(r1[-1])} of the same realization on one thread, "
                            f"{o2 - o1:.1f} s",
        }

    # the harness assertion on the deflection scale, and the residual
    # distribution, before anything is timed
    defl = deflection_check(w, skies[:nmax], skies_dev[:nmax])

    results = {}
    for prec, batch, m16 in forms:
        r = run_form(args, w, order, prec, batch, skies_dev, m16)
        if ref is not None:
            mask = ref["_tie"] > 1e-9
            errs = {}
            for f, g in zip(("T", "Q", "U"), r["maps0"]):
                if g is None:
                    continue
                x = g[rings][mask]
                y = ref[f][mask]
                errs[f] = float(np.sqrt(np.mean((x - y) ** 2)) / np.sqrt(np.mean(y ** 2)))
            r["errs"] = errs
            # per band (largest field error)
            r["errs_band"] = {}
            for bname, br in bands.items():
                sel = np.isin(rings, br)
                e = 0.0
                for f, g in zip(("T", "Q", "U"), r["maps0"]):
                    if g is None:
                        continue
                    mk = mask[sel]
                    x = g[rings[sel]][mk]
                    y = ref[f][sel][mk]
                    e = max(e, float(np.sqrt(np.mean((x - y) ** 2)) / np.sqrt(np.mean(y ** 2))))
                r["errs_band"][bname] = e
        results[(prec, batch, m16)] = r

    name = form_name
    fp32 = results.get(("fp32", 1, False))
    forms_out = {}
    for f, r in results.items():
        px = f[1] * npix / r["sec"]
        leg = sum(r["per_step"].get(k, 0.0) for k in ("legendre_T", "legendre_QU", "legendre_mfma", "tab_rhs",
                                                       "legendre_tab", "tab_epi", "legendre_caps"))
        useful = f[1] * a3_useful_flops(w.lmax, (w.ntheta + 1) // 2, order, w.pol, hasb)
        if r["q"]["defl_folded"]:
            # the table pass also synthesizes the deflection's two rows (order 1 of phi)
            useful += f[1] * a3_useful_flops(w.lmax, (w.ntheta + 1) // 2, 1, False, False)
        tabform = f[0] in ("bf16x3", "fp16x2", "fp16", "bf16")
        pk = PEAK["f16_mfma"] if tabform else (PEAK["fp32_mfma"] if f[0] == "fp32" else PEAK["fp64"])
        ent = {
            "pixels_per_s": px, "ms_per_step": r["sec"] * 1e3, "realizations_per_step": f[1],
            "ms_per_map": r["sec"] * 1e3 / f[1],
            "speedup_vs_fp32": (px / (npix / fp32["sec"])) if fp32 else None,
            "rel_rms_err_vs_oracle": r.get("errs"),
            "rel_rms_err_max_field_by_band": r.get("errs_band"),
            "stages_ms_per_step": {k: round(v, 3) for k, v in r["per_step"].items()},
            "legendre_ms_per_step": leg,
            "legendre_a3_useful_tflops": useful / (leg * 1e-3) / 1e12 if leg else None,
            "legendre_mfma_util_pct": 100.0 * useful / (leg * 1e-3) / pk if leg else None,
            "legendre_mfma_util_pct_after_skip": (100.0 * useful * r["q"]["elems"]
                                                  / ((w.lmax + 1) * (w.lmax + 2) // 2 * ((w.ntheta + 1) // 2))
                                                  / (leg * 1e-3) / pk) if leg else None,
            "workspace_gib": r["workspace_bytes"] / 2**30,
            "workspace_gib_per_map": r["workspace_bytes"] / 2**30 / f[1],
            "plan_build_s": r["plan_build_s"],
            "ms_per_step_wall_mean": r["wall_mean_sec"] * 1e3,
            "ms_per_step_min_max": [x * 1e3 for x in r["step_sec_min_max"]],
        }
        forms_out[name(f)] = ent

    H = results[headline]
    work = stage_work(w, order, headline[0], H["q"], hasb, headline[1], headline[2])
    dom = max(H["per_step"], key=lambda k: H["per_step"][k])
    kind, amount, unit, peak = work[dom]
    from paper_1307_0719_amd import taylens

    # achieved = the stage's algorithmic work per step over its kernel time
    # per step (HIP events around every launch); work_per_launch is the mean
    # share of one launch (the direct kernels take up to four realizations a
    # launch).  The matrix-core harmonic kernels count the useful flops of the
    # plain contraction, 2 (N+1) R per (l, m, ring pair) and realization
    # (R = 2 + 8 real right-hand sides for T + Q/U; two more rows of the
    # lensing potential when it rides in the pass), over the elements they
    # cover below the evanescent cut; "frac_dense" counts every (l, m).
    t = H["per_step"][dom] * 1e-3
    nl = H["launches"][dom]
    kname = taylens.STAGE_KERNELS[dom]
    if dom == "legendre_tab" and os.environ.get("TAYLENS_ONTHEFLY") == "1":
        kname = "k_legendre_lp"
    nrn = (w.ntheta + 1) // 2 - H["q"]["rpole"]
    if dom in ("legendre_tab", "legendre_mfma"):
        n = headline[1]
        per_elem = 2 * (order + 1) * (2 + ((16 if hasb else 8) if w.pol else 0))
        if H["q"]["defl_folded"]:
            per_elem += 2 * 2 * 2
        elems = H["q"]["elems"] - H["q"]["elems_caps"]
        nlm = (w.lmax + 1) * (w.lmax + 2) // 2
        useful = n * per_elem * elems
        pk = PEAK["f16_mfma"] if dom == "legendre_tab" else PEAK["fp32_mfma"]
        roof = {
            "kernel": kname, "stage": dom, "bound": "mfma",
            "achieved": useful / t / 1e12, "peak": pk / 1e12, "unit": "TFLOP/s", "frac": useful / t / pk,
            "frac_dense": n * per_elem * nlm * nrn / t / pk,
            "traffic": measured_traffic(args.workload, name(headline), kname),
            "work_per_launch": useful / nl, "work_unit": f"useful flop: {per_elem} per (l, m, ring pair) "
                                                         f"below the cut outside the caps, x {n} realizations",
            "avg_launch_ms": H["avg_launch"][dom], "launches_per_step": nl,
        }
        if dom == "legendre_tab":
            roof["hbm_table_stream"] = {"achieved": amount / t / 1e9, "unit": "GB/s", "frac": amount / t / PEAK["hbm"],
                                        "bytes_per_launch": amount / nl}
    else:
        scale = 1e9 if unit == "GB/s" else 1e12
        roof = {
            "kernel": kname, "stage": dom,
            "bound": "hbm" if kind == "hbm" else ("alu" if kind == "fp64" else "mfma"),
            "achieved": amount / t / scale,
            "peak": peak / scale, "unit": unit, "frac": amount / t / peak,
            "traffic": measured_traffic(args.workload, name(headline), kname),
            "work_per_launch": amount / nl, "avg_launch_ms": H["avg_launch"][dom], "launches_per_step": nl,
            "peak_note": "FP64 vector peak (ALU-bound recursion)" if kind == "fp64" else None,
        }
    other = {}
    for k in H["per_step"]:
        if k in work:
            kk, am, un, pk = work[k]
            sc = 1e9 if un == "GB/s" else 1e12
            a = H["per_step"][k] * 1e-3
            other[k] = {"kernel": taylens.STAGE_KERNELS[k], "resource": kk, "achieved": am / a / sc, "unit": un,
                        "frac": am / a / pk, "avg_launch_ms": H["avg_launch"][k], "ms_per_step": H["per_step"][k],
                        "launches_per_step": H["launches"][k]}
    if "legendre_tab" in H["per_step"]:
        kk, am, un, pk = work["legendre_tab_mfma"]
        a = H["per_step"]["legendre_tab"] * 1e-3
        other["legendre_tab"]["mfma_f16_achieved_tflops"] = am / a / 1e12
        other["legendre_tab"]["mfma_f16_frac"] = am / a / pk

    hf = forms_out[name(headline)]
    dt = {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16x3", "fp16x2": "f16x2", "fp16": "f16", "bf16": "bf16"}
    res = {
        "metric": "lensed pixels/sec (T+Q/U, lmax=4096) at stated rel. error; Legendre MFMA util %",
        "value": hf["pixels_per_s"],
        "unit": "pixels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": hf["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dt[headline[0]],
        "data": "synthetic",
        "config": {
            "workload": f"T+Q/U lmax={w.lmax}, {w.ntheta}x{w.nphi} equal-theta rings, Taylor order {order}, "
                        f"{headline[1]} realization(s) per step, {headline[0]} harmonic-stage contraction "
                        f"(FP64 recursion, positions and rotation)"
                        + (", derivative maps of order j+k >= 3 stored in FP16" if headline[2] else ""),
            "lmax": w.lmax, "ntheta": w.ntheta, "nphi": w.nphi, "order": order, "fields": "TQU" if w.pol else "T",
            "precision_form": headline[0], "realizations_per_step": headline[1], "maps16": headline[2],
            "rel_rms_err_vs_oracle": hf["rel_rms_err_vs_oracle"],
            "speedup_vs_fp32": hf["speedup_vs_fp32"],
            "timing": f"median of {args.steps} steps (HIP events on the plan's stream); "
                      f"wall-clock mean {hf['ms_per_step_wall_mean']:.2f} ms",
            "plan_build_s": hf["plan_build_s"], "workspace_gib_per_map": hf["workspace_gib_per_map"],
            "legendre_mfma_util_pct": hf["legendre_mfma_util_pct"],
            "legendre_mfma_util_pct_after_skip": hf["legendre_mfma_util_pct_after_skip"],
            "legendre_mfma_busy_pct_counters": next(
                (measured_mfma_busy(args.workload, name(headline), taylens.STAGE_KERNELS[st])
                 for st in ("legendre_tab", "legendre_mfma") if st in H["per_step"]), None),
            "pixels": npix,
        },
        "roofline": roof,
        "kernels": other,
        "forms": forms_out,
    }
    if cpu is not None:
        res["cpu_baseline"] = cpu
    res["deflection"] = defl
    if not args.no_extras:
        res["healpix"] = bench_healpix(args, ref is not None)
        res["batch_uneven_lmax"] = bench_batch(args, order)
        res["learned_correction"] = bench_cnn(args, w)
        res["theta_fft"] = bench_theta_fft(args)
        res["spectra"] = bench_spectra(args)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
