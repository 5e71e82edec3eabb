#!/usr/bin/env python3
"""Throughput of full-sky Taylor lensing on one MI355X.

One step = one call of the whole lensing path (deflection synthesis, harmonic
stage of T and Q/U with theta-derivatives, ring FFTs with the phi-derivative
factors, remap + Taylor sum + polarization rotation) on one realization whose
a_lm are already resident in HBM.  Default workload: T+Q/U, lmax = 4096 on the
4097 x 8192 equal-theta ring grid, Taylor order 4, FP32 form.

Prints ONE JSON line (see keys below).  ``roofline`` describes the dominant
kernel, timed live with HIP events on the plan's stream; ``cpu_baseline`` is
the CPU oracle timed on a bounded sample of the same workload (a band of
output rings), which also gives the stated relative error of the GPU maps.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

FP64_VECTOR_PEAK = 78.6e12      # MI355X FP64 vector FLOP/s
FP32_VECTOR_PEAK = 157.3e12
HBM_PEAK = 8.0e12               # bytes/s


def legendre_flops(lmax: int, nrp: int, J: int, pol: bool, hasb: bool):
    """Algorithmic FP64 flops of the harmonic stage per launch (direct
    recursion): per (l, m, ring-pair) element and family,
      recursion  sum_j [2(j+1) + 3] = (J+1)(J+5),
      contraction 4 (J+1) per complex right-hand side."""
    nalm = (lmax + 1) * (lmax + 2) // 2
    per = (J + 1) * (J + 5)
    t = nalm * nrp * (per + 4 * (J + 1))
    if not pol or lmax < 2:
        return t, 0
    nspin = (nalm - 3) * nrp
    s = 2 * nspin * (per + 4 * (J + 1) * (2 if hasb else 1))
    return t, s


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="TP4096")
    ap.add_argument("--precision", default="fp32")
    ap.add_argument("--order", type=int, default=None)
    ap.add_argument("--cpu-rings", type=int, default=16, help="output rings in the CPU-oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "independent realizations would shard across GPUs without communication.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1307_0719_amd import skygen, taylens

    w = skygen.WORKLOADS[args.workload]
    order = w.order if args.order is None else args.order
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    sky = skygen.make_sky(w.lmax, w.seed, pol=w.pol)
    to_dev = lambda a: None if a is None else torch.from_numpy(a).to(dev)
    aT, aE, aP = to_dev(sky.alm_T), to_dev(sky.alm_E), to_dev(sky.alm_phi)
    # B = 0 in these workloads: pass NULL (the library then skips the B sums)
    aB = to_dev(sky.alm_B) if (sky.alm_B is not None and np.any(sky.alm_B)) else None
    plan = taylens.Plan(w.lmax, w.ntheta, w.nphi, order, args.precision, pol=w.pol)
    outs = (plan._maps(), plan._maps() if w.pol else None, plan._maps() if w.pol else None)
    npix = w.ntheta * w.nphi

    for _ in range(args.warmup):
        plan.lens_map(aT, aE, aB, aP, out=outs)
    torch.cuda.synchronize()

    # timed region: K whole steps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.lens_map(aT, aE, aB, aP, out=outs)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sec = (t1 - t0) / args.steps

    # the same K steps again with per-stage HIP events on the plan's stream
    plan.profile(True)
    for _ in range(args.steps):
        plan.lens_map(aT, aE, aB, aP, out=outs)
    st = plan.stage_times()
    plan.profile(False)
    stages_ms = {k: (v[0] / v[1] if v[1] else 0.0) for k, v in st.items()}

    nrp = (w.ntheta + 1) // 2
    fl_T, fl_S = legendre_flops(w.lmax, nrp, order, w.pol, aB is not None)
    kern = {"legendre_QU": fl_S, "legendre_T": fl_T}
    dom = max(("legendre_QU", "legendre_T", "ring_fft", "remap", "deflection"), key=lambda k: stages_ms[k])
    if dom in kern:
        flops = kern[dom]
        achieved = flops / (stages_ms[dom] * 1e-3)
        roof = {"kernel": "k_legendre_spin" if dom == "legendre_QU" else "k_legendre_scalar",
                "bound": "alu", "achieved": achieved / 1e12, "peak": FP64_VECTOR_PEAK / 1e12,
                "unit": "TFLOP/s", "frac": achieved / FP64_VECTOR_PEAK, "traffic": None,
                "flops_per_launch": flops, "avg_launch_ms": stages_ms[dom]}
    else:
        roof = {"kernel": dom, "bound": "hbm", "achieved": None, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                "frac": None, "traffic": None}

    res = {
        "metric": "lensed pixels/sec (T+Q/U, lmax=4096) at stated rel. error; Legendre MFMA util %",
        "value": npix / sec,
        "unit": "pixels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64/f32" if args.precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {
            "workload": w.name if order == w.order else f"{w.name} (order {order})",
            "lmax": w.lmax, "ntheta": w.ntheta, "nphi": w.nphi, "order": order,
            "precision_form": args.precision, "fields": "TQU" if w.pol else "T", "pixels": npix,
            "legendre_mfma_util_pct": 0.0,
            "stages_ms": stages_ms,
        },
        "roofline": roof,
    }

    if not args.no_cpu_baseline:
        from oracle import taylens_oracle as orc

        ncores = min(16, os.cpu_count() or 1)
        nr = max(1, args.cpu_rings)
        c = w.ntheta // 2
        rings = np.arange(c - nr // 2, c - nr // 2 + nr)
        o0 = time.perf_counter()
        ref = orc.lens_rings(w.lmax, order, w.ntheta, w.nphi, rings, sky.alm_T, sky.alm_E, sky.alm_B,
                             sky.alm_phi, nthreads=ncores)
        o1 = time.perf_counter()
        errs = {}
        mask = ref["_tie"] > 1e-9
        for f, g in zip(("T", "Q", "U"), outs):
            if g is None:
                continue
            x = g.cpu().numpy()[rings][mask]
            r = ref[f][mask]
            errs[f] = float(np.sqrt(np.mean((x - r) ** 2)) / np.sqrt(np.mean(r ** 2)))
        res["config"]["rel_rms_err_vs_oracle"] = errs
        res["cpu_baseline"] = {
            "value": nr * w.nphi / (o1 - o0), "unit": "pixels/s", "cores": ncores, "kind": "oracle",
            "sample": f"{nr} output rings ({rings[0]}..{rings[-1]}) of the same map: deflection on those "
                      f"rings, derivative maps of every source ring they need, remap, Taylor sum, rotation; "
                      f"{o1 - o0:.1f} s",
        }
    print(json.dumps(res))


if __name__ == "__main__":
    main()
