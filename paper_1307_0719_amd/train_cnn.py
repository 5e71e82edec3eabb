"""Training and evaluation of the learned remainder correction.

Training pairs come from the method itself: for each seeded realization the
order-2 and order-6 Taylor sums of the same lensed sky (rotation off, so the
target is the remainder in the local frame where the correction is added);
the network is trained on random pixels of each realization with Adam, by
the library's own forward and backward kernels (``taylens.Cnn``).
Evaluation lenses held-out realizations with order 2 + correction and with
plain order 6, rotation on, and reports the RMS of each against order 6.

``python -m paper_1307_0719_amd.train_cnn`` runs the stated configuration:
200 realizations at lmax 2048 (2049 x 4096 grid, seeds 10000..10199), evaluated
at lmax 4096 (4097 x 8192, seeds 20000..20009); writes the weights with
numpy.save.
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np
import torch

from paper_1307_0719_amd import skygen, taylens


def _dev(a, dev):
    return None if a is None else torch.from_numpy(a).to(dev)


class PairMaker:
    """Order-2 inputs and order-6 - order-2 targets of one grid."""

    def __init__(self, lmax, ntheta, nphi, precision="fp32"):
        self.lmax, self.ntheta, self.nphi = lmax, ntheta, nphi
        self.p2 = taylens.Plan(lmax, ntheta, nphi, 2, precision, pol=True)
        self.p2n = taylens.Plan(lmax, ntheta, nphi, 2, precision, pol=True, rotate=False)
        self.p6n = taylens.Plan(lmax, ntheta, nphi, 6, precision, pol=True, rotate=False)
        self.dev = self.p2.device

    def sky(self, seed):
        s = skygen.make_sky(self.lmax, seed, pol=True)
        return tuple(_dev(a, self.dev) for a in (s.alm_T, s.alm_E, None, s.alm_phi))

    def pair(self, alms):
        T, E, B, P = alms
        D = self.p2.synth_derivs(T, E, B).clone()
        at, ap = (x.clone() for x in self.p2.deflection(P))
        s2 = torch.stack(self.p2n.lens_map(T, E, B, P)).reshape(3, -1).clone()
        s6 = torch.stack(self.p6n.lens_map(T, E, B, P)).reshape(3, -1)
        return D, at, ap, s6 - s2

    def close(self):
        for p in (self.p2, self.p2n, self.p6n):
            p.close()


def output_scales(pm: PairMaker, net: taylens.Cnn, seed: int, npix_sample: int = 65536):
    """scale_f = RMS over sampled pixels of target_f / sigma_f (sigma_f the
    patch RMS the network divides by): the network then learns O(1) outputs.
    sigma comes from a forward pass with unit scales and the output layer's
    bias pinned to one."""
    alms = pm.sky(seed)
    D, at, ap, tgt = pm.pair(alms)
    pix = torch.from_numpy(skygen.sample_pixels(pm.ntheta * pm.nphi, npix_sample, seed)).to(pm.dev)
    p0 = net.params()
    probe = p0.copy()
    probe[-3 - 3 - 3 * 32:-3 - 3] = 0.0  # W3 = 0
    probe[-6:-3] = 1.0                    # b3 = 1  -> y = 1
    probe[-3:] = 1.0                      # scale 1 -> corr = sigma
    net.set_params(probe)
    sig = net.forward(pm.p2, D, at, ap, pix)
    t = tgt[:, pix]
    sc = torch.sqrt(torch.mean((t / sig) ** 2, dim=1)).cpu().numpy()
    p0[-3:] = np.where(sc > 0, sc, 1.0)
    net.set_params(p0)
    return p0[-3:].copy()


def train(lmax, ntheta, nphi, seeds, steps_per_real=20, batch_pixels=32768, lr=2e-3, lr_end=2e-4,
          init_seed=1, log=None):
    pm = PairMaker(lmax, ntheta, nphi)
    net = taylens.Cnn(skygen.cnn_init(init_seed))
    scales = output_scales(pm, net, seeds[0])
    nsteps = len(seeds) * steps_per_real
    hist = []
    step = 0
    t0 = time.perf_counter()
    for i, sd in enumerate(seeds):
        D, at, ap, tgt = pm.pair(pm.sky(sd))
        for k in range(steps_per_real):
            frac = step / max(1, nsteps - 1)
            cur = lr * (lr_end / lr) ** frac  # geometric decay
            pix = torch.from_numpy(skygen.sample_pixels(ntheta * nphi, batch_pixels, sd * 1000 + k)).to(pm.dev)
            loss = net.train_step(pm.p2, D, at, ap, pix, tgt[:, pix], cur)
            step += 1
        hist.append(float(loss.item()))
        if log and (i % 10 == 0 or i == len(seeds) - 1):
            log(f"realization {i + 1}/{len(seeds)} seed {sd} loss {hist[-1]:.4f} {time.perf_counter() - t0:.1f}s")
    params = net.params()
    pm.close()
    net.close()
    return params, {"loss_per_realization": hist, "scales": scales.tolist()}


def evaluate(params, lmax, ntheta, nphi, seeds, precision="fp32", plain_orders=()):
    """RMS (over all pixels and the given seeds) against plain order 6 in the
    FP32 form (rotation on), per field, of: order 2 and order 2 + correction
    in the given precision form, and the plain orders in plain_orders (same
    form).  Plans are made one at a time (a tabulated plan at lmax 4096 holds
    its tables)."""
    dev = torch.device("cuda", torch.cuda.current_device())
    skies = []
    ref6 = []
    p6 = taylens.Plan(lmax, ntheta, nphi, 6, "fp32", pol=True)
    for sd in seeds:
        s = skygen.make_sky(lmax, sd, pol=True)
        a = (_dev(s.alm_T, dev), _dev(s.alm_E, dev), None, _dev(s.alm_phi, dev))
        skies.append(a)
        ref6.append(torch.stack(p6.lens_map(*a)).reshape(3, -1).cpu())
    p6.close()
    torch.cuda.empty_cache()

    def rms_against_ref6(run):
        acc = np.zeros(3)
        for a, m6 in zip(skies, ref6):
            m = run(a).reshape(3, -1).double()
            acc += torch.mean((m - m6.to(dev).double()) ** 2, dim=1).cpu().numpy()
        return np.sqrt(acc / len(seeds))

    p2 = taylens.Plan(lmax, ntheta, nphi, 2, precision, pol=True)
    net = taylens.Cnn(params)
    out = {"order2": rms_against_ref6(lambda a: torch.stack(p2.lens_map(*a))),
           "cnn": rms_against_ref6(lambda a: torch.stack(net.lens_map(p2, *a)))}
    net.close()
    p2.close()
    torch.cuda.empty_cache()
    for N in plain_orders:
        pn = taylens.Plan(lmax, ntheta, nphi, N, precision, pol=True)
        out[f"order{N}"] = rms_against_ref6(lambda a: torch.stack(pn.lens_map(*a)))
        pn.close()
        torch.cuda.empty_cache()
    signal = np.sqrt(sum(torch.mean(m6.double() ** 2, dim=1).numpy() for m6 in ref6) / len(seeds))
    res = {"rms_err_order2": out["order2"].tolist(), "rms_err_cnn": out["cnn"].tolist(),
           "rms_signal": signal.tolist(), "gain": (out["order2"] / out["cnn"]).tolist(),
           "precision": precision, "seeds": list(seeds)}
    for N in plain_orders:
        res[f"rms_err_order{N}"] = out[f"order{N}"].tolist()
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--lmax", type=int, default=2048)
    ap.add_argument("--nreal", type=int, default=200)
    ap.add_argument("--steps-per-real", type=int, default=20)
    ap.add_argument("--batch-pixels", type=int, default=32768)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--eval-lmax", type=int, default=4096)
    ap.add_argument("--eval-nreal", type=int, default=10)
    ap.add_argument("--out", default=os.path.join(os.path.dirname(os.path.abspath(__file__)), "cnn_weights.npy"))
    a = ap.parse_args()
    say = lambda m: print(m, flush=True)
    seeds = list(range(10000, 10000 + a.nreal))
    t0 = time.perf_counter()
    params, info = train(a.lmax, a.lmax + 1, 2 * a.lmax, seeds, a.steps_per_real, a.batch_pixels, a.lr, log=say)
    t_train = time.perf_counter() - t0
    np.save(a.out, params)
    res = {"train": {"lmax": a.lmax, "realizations": a.nreal, "steps": a.nreal * a.steps_per_real,
                     "batch_pixels": a.batch_pixels, "seconds": t_train, "final_loss": info["loss_per_realization"][-1],
                     "scales": info["scales"]}}
    same = evaluate(params, a.lmax, a.lmax + 1, 2 * a.lmax, list(range(20000, 20000 + min(3, a.eval_nreal))))
    res["held_out_same_grid"] = same
    say(json.dumps({"held_out_same_grid": same}))
    if a.eval_lmax:
        J = a.eval_lmax
        res["eval"] = evaluate(params, J, J + 1, 2 * J, list(range(20000, 20000 + a.eval_nreal)))
        res["eval"]["lmax"] = J
    print(json.dumps(res))


if __name__ == "__main__":
    main()
