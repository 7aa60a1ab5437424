"""Training and evaluation of the learned setup.

A gauge-covariant network (layers of colour hops with complex channel
weights, mgdd_net_*) maps random vectors to test vectors in place of most
iterations of the bootstrap setup. It is trained on gauge fields of one
recipe: on each training field the bootstrap setup runs once and its
interpolation P is the target; the loss is the part of the network's output
outside range(P), ||(1 - P P^H) f||^2 / ||f||^2, averaged over random
inputs, minimised by Adam. Evaluation on held-out fields compares the outer
iteration count and the setup time of the solve with the network's vectors
against the plain bootstrap setup, which stays the fallback: a field whose
learned setup needs more outer iterations than the bootstrap's (by more
than `fallback_margin`) is solved with the bootstrap.

usage: python -m paper_1202_2462_amd.learned [--train 8] [--eval 2] [--steps 300]
           [--widths 1,16,16,16,1] [--out weights.npz]
       python -m paper_1202_2462_amd.learned --weights weights.npz --eval 4   (evaluation only)
"""
from __future__ import annotations

import argparse
import json
import time
import multiprocessing as mp
from concurrent.futures import ProcessPoolExecutor

import numpy as np

from . import mgdd

WORKLOAD = dict(dims=(16, 16, 16, 32), block=(4, 4, 4, 4), agg=(4, 4, 4, 4), ntv=20, eps=0.5, ape=2, csw=1.0,
                nu=3, iota=3, mr=4, restart=20, tol=1e-10)
TRAIN_SEED0, EVAL_SEED0 = 4000, 4100


def _gauge(args):
    import latgen
    dims, eps, seed, ape = args
    return latgen.gauge_field(dims, eps, seed, ape_steps=ape)


def gauge_fields(seeds, w=WORKLOAD, workers=8):
    """seeded gauge fields of the workload recipe (host, in parallel)"""
    # fresh interpreters (no fork of a process that may hold GPU state)
    with ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        return list(ex.map(_gauge, [(w["dims"], w["eps"], s, w["ape"]) for s in seeds]))


def tile_field(U, dims, reps):
    """a gauge field repeated reps[mu] times along each direction"""
    U4 = np.asarray(U).reshape(dims[3], dims[2], dims[1], dims[0], 4, 3, 3)
    return np.ascontiguousarray(np.tile(U4, (reps[3], reps[2], reps[1], reps[0], 1, 1, 1)).reshape(-1, 4, 3, 3))


class Field:
    """one gauge field in its own context, with the bootstrap setup done"""

    def __init__(self, U, seed, m0, w=WORKLOAD):
        import torch

        import latgen
        self.w, self.seed = w, seed
        self.lat = mgdd.Lattice(w["dims"], w["block"])
        self.U = torch.tensor(np.ascontiguousarray(U).view(np.float64), device="cuda")
        self.m0 = m0
        self.lat.set_gauge(self.U, m0, w["csw"])
        V = int(np.prod(w["dims"]))
        self.rnd = self.lat.pack(latgen.gaussian_fields(w["dims"], w["ntv"], seed + 7), mgdd.F64)
        Vc = V // int(np.prod(w["agg"]))
        st = latgen.gaussian_vector(Vc * 2 * w["ntv"], seed + 8)
        self.start = torch.tensor(np.stack([st.real, st.imag], -1), dtype=torch.float64, device="cuda")
        self.b = self.lat.pack(latgen.gaussian_fields(w["dims"], 1, seed + 9), mgdd.F64)

    def bootstrap(self, nu=None, n_part2=1, rnd=None):
        import torch
        w = self.w
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        self.lat.setup(w["agg"], self.rnd if rnd is None else rnd, self.start, nu=w["nu"] if nu is None else nu,
                       iota=w["iota"], mr_iters=w["mr"], n_part2=n_part2, prec=mgdd.F32)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    def learned(self, widths, weights, nu=1, n_part2=1):
        import torch
        w = self.w
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        self.lat.setup_learned(widths, weights, w["agg"], self.rnd, self.start, nu=nu, iota=w["iota"],
                               mr_iters=w["mr"], n_part2=n_part2, prec=mgdd.F32)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    def solve(self):
        w = self.w
        t0 = time.perf_counter()
        z, st = self.lat.solve(self.b, precision=mgdd.MIXED, restart=w["restart"], tol=w["tol"], maxit=3000,
                               mr_iters=w["mr"], allow_noconv=True)
        return dict(iters=st[0].iters, converged=bool(st[0].converged), solve_s=time.perf_counter() - t0)

    def close(self):
        self.lat.close()


def train(fields, widths, steps, lr=1e-2, samples=2, seed=5, log=print):
    """Adam on the mean loss over `samples` random inputs per step, cycling
    over the training fields (each with its bootstrap P in its context)"""
    import torch

    import latgen
    w0 = fields[0].lat.weights_to_dev(latgen.network_weights(widths, seed))
    m, v = torch.zeros_like(w0), torch.zeros_like(w0)
    W = w0
    hist = []
    dims = fields[0].w["dims"]
    for step in range(1, steps + 1):
        f = fields[step % len(fields)]
        x = f.lat.pack(latgen.gaussian_fields(dims, samples, 100000 + step), mgdd.F32)
        L, g = f.lat.net_grad(widths, W, x)
        f.lat.net_adam(widths, W, g, m, v, step, lr)
        hist.append(L)
        if step % 25 == 0 or step == 1:
            log(f"step {step}: loss {np.mean(hist[-25:]):.4f}")
    return W, hist


def evaluate(fields, widths, W, nu_learned=(0, 1), fallback_margin=0.1, log=print):
    """per field: bootstrap (nu rounds + second part) against the learned
    setup (network, then nu rounds for each nu in nu_learned, + second part)
    and, as a control, random vectors with the same rounds; outer iterations
    and setup time. The learned setup with the most rounds decides the
    fallback."""
    out = []
    for f in fields:
        rec = {"seed": f.seed}
        rec["bootstrap_setup_s"] = f.bootstrap()
        rec["bootstrap"] = f.solve()
        for nu in nu_learned:
            rec[f"control_nu{nu}_setup_s"] = f.bootstrap(nu=nu)
            rec[f"control_nu{nu}"] = f.solve()
            rec[f"learned_nu{nu}_setup_s"] = f.learned(widths, W, nu=nu)
            rec[f"learned_nu{nu}"] = f.solve()
        last = rec[f"learned_nu{max(nu_learned)}"]
        lb = last["iters"] if last["converged"] else np.inf
        rec["fallback"] = bool(lb > (1 + fallback_margin) * rec["bootstrap"]["iters"])
        out.append(rec)
        log(json.dumps(rec))
    return out


def main():
    import torch
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=8)
    ap.add_argument("--eval", type=int, default=2)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--lr", type=float, default=1e-2)
    ap.add_argument("--samples", type=int, default=2)
    ap.add_argument("--widths", default="1,16,16,16,1")
    ap.add_argument("--nu-learned", default="0,1")
    ap.add_argument("--m0", type=float, default=None)
    ap.add_argument("--eval-tiled", type=int, default=0,
                    help="also evaluate on this many held-out fields repeated twice in every direction")
    ap.add_argument("--weights", default=None, help="evaluate these weights (.npz) instead of training")
    ap.add_argument("--out", default=None)
    a = ap.parse_args()
    widths = [int(t) for t in a.widths.split(",")]
    if a.weights:
        d = np.load(a.weights)
        widths = [int(t) for t in d["widths"]]
        a.train = 0
    if a.m0 is None:
        import os
        root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
        with open(os.path.join(root, "tests", "golden", "m0.json")) as fh:
            a.m0 = json.load(fh)["c1"]["m0"]
    log = lambda *s: print(*s, flush=True)
    t0 = time.time()
    tseeds = [TRAIN_SEED0 + i for i in range(a.train)]
    eseeds = [EVAL_SEED0 + i for i in range(a.eval)]
    Us = gauge_fields(tseeds + eseeds)
    log(f"{len(Us)} gauge fields in {time.time() - t0:.1f} s")
    if a.weights:
        hist, train_s = [np.nan], 0.0
        eval_f = [Field(U, s, a.m0) for U, s in zip(Us[a.train:], eseeds)]
        W = eval_f[0].lat.weights_to_dev([d[f"W{l}"] for l in range(len(widths) - 1)])
    else:
        train_f = [Field(U, s, a.m0) for U, s in zip(Us[:a.train], tseeds)]
        for f in train_f:
            f.bootstrap()
            f.lat.release_workspace()   # keep only P, D_c and the links of each training field
        log("bootstrap setups of the training fields done")
        t1 = time.time()
        W, hist = train(train_f, widths, a.steps, a.lr, a.samples, log=log)
        torch.cuda.synchronize()
        train_s = time.time() - t1
        for f in train_f:
            f.close()
        eval_f = [Field(U, s, a.m0) for U, s in zip(Us[a.train:], eseeds)]
    nus = tuple(int(t) for t in a.nu_learned.split(","))
    res = evaluate(eval_f, widths, W, nus, log=log)
    for f in eval_f:
        f.close()
    big = []
    if a.eval_tiled:
        wb = dict(WORKLOAD, dims=tuple(2 * d for d in WORKLOAD["dims"]))
        big_f = [Field(tile_field(U, WORKLOAD["dims"], (2, 2, 2, 2)), s, a.m0, wb)
                 for U, s in zip(Us[a.train:a.train + a.eval_tiled], eseeds)]
        big = evaluate(big_f, widths, W, nus, log=log)
        for f in big_f:
            f.close()
    summary = dict(widths=widths, train_fields=a.train, eval_fields=a.eval, steps=a.steps, lr=a.lr,
                   samples=a.samples, train_s=train_s, loss_first=float(np.mean(hist[:10])),
                   loss_last=float(np.mean(hist[-10:])), eval=res, eval_tiled=big)
    log(json.dumps(summary))
    if a.out:
        Ws = mgdd.Lattice.weights_from_dev(W, widths)
        np.savez(a.out, widths=np.array(widths), **{f"W{l}": Wl for l, Wl in enumerate(Ws)})


if __name__ == "__main__":
    main()
