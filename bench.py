#!/usr/bin/env python3
"""Benchmark of the SAP + aggregation two-level solver on one MI355X.

One step = one pass of the whole hot path on the 16^3 x 32 workload: gauge
ingest with the clover term, the bootstrap setup (Schwarz sweeps in FP32,
P and D_c, harmonic Ritz vectors, second setup part) and the mixed-precision
FGMRES solve of one Gaussian right-hand side to ||b - D z|| <= 1e-10 ||b||.
`value` is solves per second (setup included). Beside it the same JSON line
carries the Wilson-clover apply rates (Dirac applies/s and HBM GB/s), the
time-to-1e-10 of the plain FP64 two-level solve, of the three-level variant,
of the paper's own protocol (GMRES(3) block solves, FGMRES(25)), of the
setup with the shipped learned network in place of most bootstrap
iterations, of plain
FP64 CGN (the paper's comparator) and GCR (also even-odd), the roofline of
the dominant kernel, and the oracle on the host cores as a CPU baseline.

usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
       python bench.py --kernel-only step|sap|dirac|copy   (short runs for hardware counters:
           one step, Schwarz sweeps alone, Wilson-clover applies alone; each followed
           by a 256 MiB copy that calibrates the traffic counters)
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# FP32 vector peak without packed FP32 instructions (the library is built with
# them disabled): 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz
FP32_VALU_PEAK_TFLOPS = 78.6
WORKLOAD = "c1"
# algorithmic cost of one site update of a Schwarz colour step with k MR steps
# (FP32): bytes = z in 96 + b 96 + links 288 + clover 288 + z out 96;
# flops = (1 + k) operator applications of 1896 + k MR updates of 336
SAP_BYTES_PER_SITE = 864
# the three-level variant timed beside the two-level method: aggregates of
# 2^4 coarse sites, 28 level-2 test vectors (the 20 restricted fine ones and
# 8 random), two smoothing rounds of level-2 Schwarz sweeps on 2^4 blocks in
# the setup; in the solve 8 flexible GMRES steps on D_c per coarse solve,
# each preconditioned by one level-2 Schwarz sweep (4 MR steps) after 12
# GMRES steps on D_cc
LEVEL3 = dict(agg2=(2, 2, 2, 2), ntv2=28, block2=(2, 2, 2, 2), setup_nu2=2, k2=8, nu2=1, mr2=4, cit=12)


def sap_flops_per_site(k):
    return (1 + k) * 1896 + k * 336


# HBM traffic of the FP32 Schwarz kernel from hardware counters, and the
# sources it was taken from (the figure is dropped when they have changed)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "sap4_kernel_f32_16x16x16x32_hbm_traffic.md")
SAP_SOURCES = ["paper_1202_2462_amd/csrc/sap.hip", "paper_1202_2462_amd/csrc/stencil.h",
               "paper_1202_2462_amd/csrc/mgdd_internal.h", "paper_1202_2462_amd/csrc/geometry.h"]


def sap_sources_digest():
    import hashlib
    h = hashlib.sha256()
    for f in SAP_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def sap_traffic_per_site():
    """HBM bytes per site update from the committed counter summary, or None
    when there is none or the kernel's sources differ from the measured ones."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    vals = {}
    with open(TRAFFIC_FILE) as f:
        for line in f:
            if ":" in line and line.split(":", 1)[0].strip() in ("hbm_bytes_per_site_update", "kernel_sources_sha256"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip().strip("`")
    if vals.get("kernel_sources_sha256") != sap_sources_digest() or "hbm_bytes_per_site_update" not in vals:
        return None
    return float(vals["hbm_bytes_per_site_update"])


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def load_m0(name):
    path = os.path.join(ROOT, "tests", "golden", "m0.json")
    with open(path) as f:
        return float(json.load(f)[name]["m0"])


class Bench:
    def __init__(self, name=WORKLOAD, m0=None):
        import torch

        import latgen
        from paper_1202_2462_amd import mgdd
        self.torch, self.mgdd, self.latgen = torch, mgdd, latgen
        w = latgen.WORKLOADS[name]
        self.name, self.w = name, w
        self.dims, self.block, self.agg, self.N = tuple(w["dims"]), tuple(w["block"]), tuple(w["agg"]), w["ntv"]
        self.V = int(np.prod(self.dims))
        self.m0, self.csw = (load_m0(name) if m0 is None else m0), w["csw"]
        k = int(name[1:])
        t0 = time.time()
        U = latgen.workload_gauge(name)
        log(f"gauge field {self.dims} generated in {time.time() - t0:.1f} s")
        self.U_host = U
        self.lat = mgdd.Lattice(self.dims, self.block)
        F64 = mgdd.F64
        # inputs resident in HBM before any timed region
        self.U_dev = torch.tensor(U.view(np.float64), device="cuda")
        self.rnd_host = latgen.gaussian_fields(self.dims, self.N, 1000 * k + latgen.TAG_TV)
        self.rnd = self.lat.pack(self.rnd_host, F64)
        self.Vc = self.V // int(np.prod(self.agg))
        st = latgen.gaussian_vector(self.Vc * 2 * self.N, 1000 * k + latgen.TAG_ARNOLDI)
        self.start_host = st
        self.start = torch.tensor(np.stack([st.real, st.imag], -1), dtype=torch.float64, device="cuda")
        n2 = max(LEVEL3["ntv2"] - self.N, 1)
        r2 = latgen.gaussian_vector(n2 * self.Vc * 2 * self.N, 1000 * k + latgen.TAG_TV2)
        self.rnd2 = torch.tensor(np.stack([r2.real, r2.imag], -1), dtype=torch.float64,
                                 device="cuda").reshape(n2, self.Vc, 2, self.N, 2)
        self.b_host = latgen.gaussian_fields(self.dims, 1, 1000 * k + latgen.TAG_RHS)
        self.b = self.lat.pack(self.b_host, F64)
        torch.cuda.synchronize()

    # one pass of the hot path
    def step(self, setup_prec=None, solve_prec=None, split=None, levels=2, paper_protocol=False):
        mg = self.mgdd
        w = self.w
        setup_prec = mg.F32 if setup_prec is None else setup_prec
        solve_prec = mg.MIXED if solve_prec is None else solve_prec
        t0 = time.perf_counter()
        self.lat.set_gauge(self.U_dev, self.m0, self.csw)
        self.lat.setup(self.agg, self.rnd, self.start, nu=w["nu"], iota=w["iota"], mr_iters=w["mr"], prec=setup_prec)
        l3 = {}
        if levels == 3:
            q = LEVEL3
            self.lat.setup_level2(q["agg2"], q["ntv2"], q["block2"], random2=self.rnd2, nu2=q["setup_nu2"],
                                  mr_iters=q["mr2"])
            l3 = dict(levels=3, k2=q["k2"], nu2=q["nu2"], mr2=q["mr2"])
        t1 = time.perf_counter()
        if paper_protocol:   # GMRES(3) block solves, FGMRES(25)
            z, stats = self.lat.solve(self.b, precision=solve_prec, restart=25, tol=w["tol"], maxit=2000,
                                      coarse_iters=12, nu=1, mr_iters=3, block_solver=mg.BLOCK_GMRES)
        else:
            z, stats = self.lat.solve(self.b, precision=solve_prec, restart=w["restart"], tol=w["tol"], maxit=2000,
                                      coarse_iters=LEVEL3["cit"] if levels == 3 else 12, nu=1, mr_iters=w["mr"],
                                      **l3)
        t2 = time.perf_counter()
        if split is not None:
            split.update(setup_s=t1 - t0, solve_s=t2 - t1, iters=stats[0].iters, restarts=stats[0].restarts,
                         relres=stats[0].relres)
        return z, stats[0]

    def learned_step(self, split):
        """gauge ingest + learned setup (the shipped network on the random
        vectors, one round of Schwarz sweeps, the second setup part) + the
        mixed-precision solve; None without the shipped weights"""
        path = os.path.join(ROOT, "paper_1202_2462_amd", "learned_weights_16x16x16x32.npz")
        if not os.path.exists(path):
            return None
        d = np.load(path)
        widths = [int(t) for t in d["widths"]]
        W = self.lat.weights_to_dev([d[f"W{l}"] for l in range(len(widths) - 1)])
        mg, w = self.mgdd, self.w
        self.torch.cuda.synchronize()
        t0 = time.perf_counter()
        self.lat.set_gauge(self.U_dev, self.m0, self.csw)
        self.lat.setup_learned(widths, W, self.agg, self.rnd, self.start, nu=1, iota=w["iota"], mr_iters=w["mr"],
                               n_part2=1, prec=mg.F32)
        self.torch.cuda.synchronize()
        t1 = time.perf_counter()
        z, stats = self.lat.solve(self.b, precision=mg.MIXED, restart=w["restart"], tol=w["tol"], maxit=2000,
                                  coarse_iters=12, nu=1, mr_iters=w["mr"])
        t2 = time.perf_counter()
        split.update(setup_s=t1 - t0, solve_s=t2 - t1, iters=stats[0].iters, restarts=stats[0].restarts,
                     relres=stats[0].relres, converged=bool(stats[0].converged), widths=widths)
        return split

    def cgn(self):
        mg = self.mgdd
        t0 = time.perf_counter()
        z, stats = self.lat.solve(self.b, solver=mg.SOLVER_CGN, tol=self.w["tol"], maxit=200000)
        return dict(seconds=time.perf_counter() - t0, iters=stats[0].iters, restarts=stats[0].restarts,
                    relres=stats[0].relres, converged=bool(stats[0].converged)), z

    def gcr(self, even_odd):
        mg = self.mgdd
        t0 = time.perf_counter()
        z, stats = self.lat.solve(self.b, solver=mg.SOLVER_GCR_EO if even_odd else mg.SOLVER_GCR, restart=16,
                                  tol=self.w["tol"], maxit=100000)
        return dict(seconds=time.perf_counter() - t0, iters=stats[0].iters, relres=stats[0].relres,
                    converged=bool(stats[0].converged)), z

    def time_calls(self, fn, n, warm=3):
        torch = self.torch
        for _ in range(warm):
            fn()
        torch.cuda.synchronize()
        s = torch.cuda.current_stream()   # the stream the library was created on
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(n):
            fn()
        e1.record(s)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e-3 / n

    def dirac_rates(self):
        mg = self.mgdd
        out = {}
        # bytes per site: spinor in + out, 4 links, clover (FP16: half spinors, FP32 links and clover)
        for prec, name, bps in ((mg.F64, "f64", 1536), (mg.F32, "f32", 768), (mg.F16, "f16", 672)):
            x = self.lat.field(prec, 1)
            x.normal_()
            y = self.lat.field(prec, 1)
            t = self.time_calls(lambda: mg.mgdd_dirac_apply(self.lat.ctx, prec, 1, x, y), 50)
            out[name] = dict(applies_per_s=1.0 / t, us_per_apply=t * 1e6, gbs=bps * self.V / t / 1e9)
        return out

    def copy_rate(self):
        """Device-to-device copy of 1 GiB (read + write), the stream-copy
        ceiling the stencil rates can be read against."""
        torch = self.torch
        x = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
        y = torch.empty_like(x)
        t = self.time_calls(lambda: y.copy_(x), 10)
        del x, y
        return 2 * (1 << 30) / t / 1e9

    def sap_launch_time(self):
        """Average duration of one colour step of the FP32 Schwarz kernel
        (mgdd_sap with one sweep launches one kernel per colour)."""
        mg = self.mgdd
        b = self.lat.field(mg.F32, 1)
        b.normal_()
        z = self.lat.field(mg.F32, 1)
        t = self.time_calls(lambda: mg.mgdd_sap(self.lat.ctx, mg.F32, 1, None, 1, self.w["mr"], 0.0, b, z), 50)
        return t / 2.0


def cpu_baseline(bench, gpu_split, sample_iters=10):
    """The oracle on the host cores, on a bounded sample of the same workload:
    its full bootstrap setup (same random vectors and Arnoldi start; FP64
    sweeps, as the oracle computes), then `sample_iters` iterations of its
    two-level FGMRES on the same right-hand side; the solve is scaled to the
    GPU step's iteration count. Solves per second of that composite."""
    import oracle
    from oracle import solvers
    w = bench.w
    op = solvers.Operator(bench.dims, bench.U_host, bench.m0, bench.csw)
    t0 = time.perf_counter()
    _, tl = solvers.bootstrap(op, bench.block, bench.agg, bench.N, w["nu"], w["iota"], w["mr"], bench.rnd_host,
                              bench.start_host)
    t_setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    _, st = solvers.fgmres(op.apply, tl.precond, bench.b_host[0], w["restart"], w["tol"], sample_iters)
    t_iters = time.perf_counter() - t0
    per_iter = t_iters / max(st.iters, 1)
    iters = gpu_split["iters"]
    total = t_setup + per_iter * iters
    sample = ("oracle FP64 on the same workload: its bootstrap setup in full (%.1f s) and %d iterations of its "
              "two-level FGMRES (%.1f s), the solve scaled to the GPU step's %d iterations"
              % (t_setup, st.iters, t_iters, iters))
    return dict(value=1.0 / total, unit="solves/s", cores=oracle.num_threads(), kind="oracle", sample=sample,
                seconds_per_solve=total, sample_cpu_seconds=round(t_setup + t_iters, 2),
                setup_s=round(t_setup, 3), seconds_per_iteration=round(per_iter, 4))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-compare", action="store_true")
    ap.add_argument("--kernel-only", choices=["step", "sap", "dirac", "copy"], default=None)
    ap.add_argument("--m0", type=float, default=None, help="override the tuned bare mass")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU per process and bench.py on one GPU; run with --gpus 1"}))
        sys.exit(2)

    import torch
    bench = Bench(m0=args.m0)
    mg = bench.mgdd

    if args.kernel_only:
        # short run of one kernel for hardware counters (rocprofv3 --pmc)
        bench.lat.set_gauge(bench.U_dev, bench.m0, bench.csw)
        if args.kernel_only == "step":
            bench.step()
        elif args.kernel_only == "sap":
            bench.sap_launch_time()
        elif args.kernel_only == "dirac":
            bench.dirac_rates()
        x = torch.empty(256 * 1024 * 1024 // 4, dtype=torch.float32, device="cuda").normal_()
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)    # reference copy kernel: 256 MiB read + 256 MiB written
        torch.cuda.synchronize()
        print(json.dumps({"kernel_only": args.kernel_only, "copy_bytes_each_way": x.numel() * 4}))
        return

    log("warmup")
    for _ in range(args.warmup):
        bench.step()
    torch.cuda.synchronize()
    log("timed steps")
    ctx = bench.lat.ctx
    for kern, prec in ((mg.KERNEL_SAP, mg.F32), (mg.KERNEL_DIRAC, mg.F64)):
        mg.mgdd_timing_read(ctx, kern, prec, reset=True)
    mg.mgdd_timing_enable(ctx, True)    # HIP events around each launch, on the library's stream
    t0 = time.perf_counter()
    last = None
    for _ in range(args.steps):
        _, last = bench.step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    mg.mgdd_timing_enable(ctx, False)
    sap_ms, sap_units, sap_n = mg.mgdd_timing_read(ctx, mg.KERNEL_SAP, mg.F32, reset=True)
    d_ms, d_units, d_n = mg.mgdd_timing_read(ctx, mg.KERNEL_DIRAC, mg.F64, reset=True)
    ms = elapsed / args.steps * 1e3
    split = {}
    bench.step(split=split)
    log("split", split)

    result = {
        "metric": "Dirac applies/s + HBM GB/s; time-to-1e-10 solve vs plain FP64 GCR (1 GPU)",
        "value": 1000.0 / ms,
        "unit": "solves/s (bootstrap setup + mixed-precision FGMRES to 1e-10, 1 RHS)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 (smoother, transfers, coarse solve) + f64 (outer FGMRES, true residual)",
        "data": "synthetic (seeded SU(3) links exp(i eps H) + 2 APE steps, Gaussian RHS)",
        "config": {"workload": "16^3x32 Wilson-clover c_sw=1.0, min Re eig(D) = %.2f, SAP blocks 4^4 with 4 MR "
                               "steps and 1 sweep, aggregates 4^4, 20 test vectors, FGMRES(20), tol 1e-10"
                               % bench.w["target"],
                   "lattice": list(bench.dims), "m0": bench.m0, "global_batch": 1, "parallelism": "single GPU"},
        "time_to_solution": {"mg_mixed": split},
    }
    if last is not None:
        result["time_to_solution"]["mg_mixed"]["converged"] = bool(last.converged)

    if not args.no_compare:
        log("plain FP64 multilevel")
        s64 = {}
        bench.step(setup_prec=mg.F64, solve_prec=mg.PLAIN_F64, split=s64)
        result["time_to_solution"]["mg_fp64"] = s64
        log("three-level, mixed precision")
        s3 = {}
        bench.step(levels=3, split=s3)
        s3["params"] = LEVEL3
        result["time_to_solution"]["mg3_mixed"] = s3
        log("paper protocol (GMRES(3) blocks, FGMRES(25)), mixed precision")
        sp = {}
        bench.step(paper_protocol=True, split=sp)
        result["time_to_solution"]["mg_paper_protocol"] = sp
        log("learned setup")
        sl = bench.learned_step({})
        if sl is not None:
            result["time_to_solution"]["mg_learned"] = sl
        log("plain FP64 CGN")
        result["time_to_solution"]["cgn_fp64"], _ = bench.cgn()
        log("plain FP64 GCR")
        result["time_to_solution"]["gcr_fp64"], _ = bench.gcr(False)
        log("even-odd FP64 GCR")
        result["time_to_solution"]["gcr_eo_fp64"], _ = bench.gcr(True)
        tts = result["time_to_solution"]
        mgt = tts["mg_mixed"]["setup_s"] + tts["mg_mixed"]["solve_s"]
        result["speedup_vs_gcr_fp64"] = {"solve_only": tts["gcr_fp64"]["seconds"] / tts["mg_mixed"]["solve_s"],
                                         "with_setup": tts["gcr_fp64"]["seconds"] / mgt}
        result["speedup_vs_cgn_fp64"] = {"solve_only": tts["cgn_fp64"]["seconds"] / tts["mg_mixed"]["solve_s"],
                                         "with_setup": tts["cgn_fp64"]["seconds"] / mgt}

    bench.lat.set_gauge(bench.U_dev, bench.m0, bench.csw)
    result["dirac"] = bench.dirac_rates()
    result["stream_copy_gbs"] = bench.copy_rate()
    if d_n:
        result["dirac"]["f64_in_timed_steps"] = {"launches": d_n, "us_per_launch": d_ms * 1e3 / d_n,
                                            "gbs": 1536 * d_units / (d_ms * 1e-3) / 1e9}
    # roofline of the dominant kernel of the step, the FP32 Schwarz colour
    # kernel, from its launches in the timed steps (HIP events around each
    # launch on the library's stream). At k MR steps it performs
    # sap_flops_per_site(k) flops on 864 algorithmic bytes per site update,
    # above the FP32 ridge (78.6 TFLOP/s / 8 TB/s = 9.8 flop/B): ALU-bound.
    if sap_n:
        t_launch = sap_ms * 1e-3 / sap_n
        units_launch = sap_units / sap_n
        flops_launch = sap_flops_per_site(bench.w["mr"]) * units_launch
        achieved = flops_launch / t_launch / 1e12
        tps = sap_traffic_per_site()
        result["roofline"] = {
            "bound": "alu", "kernel": "sap4_kernel<float> (Schwarz colour step, 4 MR steps)",
            "achieved": achieved, "peak": FP32_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / FP32_VALU_PEAK_TFLOPS,
            "traffic": None if tps is None else tps * units_launch,
            "launches": sap_n, "us_per_launch": t_launch * 1e6, "site_updates_per_launch": units_launch,
            "algorithmic_flops_per_launch": flops_launch,
            "algorithmic_bytes_per_launch": SAP_BYTES_PER_SITE * units_launch,
            "hbm_gbs": SAP_BYTES_PER_SITE * units_launch / t_launch / 1e9,
            "hbm_frac": SAP_BYTES_PER_SITE * units_launch / t_launch / 1e9 / HBM_PEAK_GBS}

    if not args.no_cpu:
        log("cpu baseline (oracle)")
        result["cpu_baseline"] = cpu_baseline(bench, split)
    print(json.dumps(result))


if __name__ == "__main__":
    main()
