#!/usr/bin/env python3
"""Benchmark of the SAP + aggregation two-level solver on one MI355X.

Default workload: the 48^3 x 96 lattice (10 616 832 sites), the largest of
the solver's configurations: c_sw = 1.0, SAP blocks 4^4 with 4 MR steps and
one sweep, aggregates 4^4, 20 test vectors, 3 + 3 bootstrap sweeps in FP32,
FGMRES(30) to ||b - D z|| <= 1e-10 ||b||, one Gaussian right-hand side. The
gauge field is the 16^3 x 32 workload field (links exp(0.5 i H), 2 APE steps)
repeated three times in every direction, with that field's tuned bare mass
(leftmost eigenvalue of the 16^3 x 32 operator at real part 0.01).

One step = one pass of the whole hot path: gauge ingest with the clover term,
the bootstrap setup (memory-lean form) and the mixed-precision FGMRES solve.
`value` is solves per second (setup included). The same JSON line carries the
time-to-1e-10 of plain FP64 multigrid, even-odd FP64 GCR(16) and FP64 CGN on
the same lattice, and the solve with half-precision storage in the
preconditioner; the Wilson-clover apply and Schwarz sweep rates at this size
(median of 100 launches after 10, algorithmic GB/s against 8 TB/s); the
roofline of the kernel family with the largest share of the timed steps
(`roofline`: the coarse GMRES step or the Schwarz colour step) and of the
other one (`roofline_other`); and the oracle on the host cores as a CPU
baseline.

usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c3|c2|c1] [--no-cpu] [--no-compare]
       python bench.py --kernel-only step|sap|dirac|coarse|coarse12   (short runs for hardware
           counters: one step, Schwarz sweeps alone, Wilson-clover applies alone, coarse
           GMRES(12) solves alone, the 12-RHS coarse apply; each followed by five 256 MiB
           device copies and additions that calibrate the traffic counters)
       python bench.py --workload c2 --autotune   (Schwarz block shape x lanes per site)
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

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP32_PEAK_TFLOPS = 157.3       # MI355X FP32 vector (published)
REPS = {"c3": 3, "c2": 2}      # 48^3 x 96 and 32^3 x 64: the 16^3 x 32 field repeated per direction


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def load_m0(name):
    with open(os.path.join(ROOT, "tests", "golden", "m0.json")) as f:
        return float(json.load(f)[name]["m0"])


# algorithmic HBM bytes per site (links and clover term read once per launch,
# each field read / written once)
def dirac_bytes(prec_name, nrhs=1):
    """algorithmic bytes per site of one Wilson-clover launch on special unitary
    links (the library reads two rows of each and rebuilds the third): links
    4 x 6 complex and the clover term's 72 reals once per launch, the spinor
    in and out per field; the library's own count (mgdd_timing_read)"""
    lc, sp = {"f64": (384 + 576, 384), "f32": (192 + 288, 192), "f16": (192 + 288, 96)}[prec_name]
    return lc + sp * nrhs


# one colour step, FP32, per site of the colour: links 192 (rows 0 and 1 of the
# four forward links, the third row rebuilt: the fields here are special
# unitary) + clover 288 + z in, b, z out 288
SAP_BYTES_PER_SITE = 768


def sap_flops_per_site(k):
    """(1 + k) operator applications of 1896 flops + k MR updates of 336"""
    return (1 + k) * 1896 + k * 336


# HBM traffic of the Schwarz kernel from hardware counters at this workload,
# and the sources it was taken from (the figure is dropped when they changed)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "sapc_kernel_f32_48x48x48x96_hbm_traffic.md")
SAP_SOURCES = ["paper_1202_2462_amd/csrc/sap.hip", "paper_1202_2462_amd/csrc/stencil.h",
               "paper_1202_2462_amd/csrc/mgdd_internal.h", "paper_1202_2462_amd/csrc/geometry.h"]
COARSE_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "arnoldi_apply_f32_48x48x48x96_hbm_traffic.md")
COARSE_SOURCES = ["paper_1202_2462_amd/csrc/arnoldi.hip", "paper_1202_2462_amd/csrc/coarse.h",
                  "paper_1202_2462_amd/csrc/mgdd_internal.h", "paper_1202_2462_amd/csrc/transfer.h"]


def sources_digest(files):
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def counter_traffic(path, files):
    """HBM bytes per site update from a committed counter summary, or None
    when there is none or the kernel's sources differ from the measured ones."""
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if ":" in line:
                k, v = line.split(":", 1)
                vals[k.strip().strip("`* ")] = v.strip().strip("`")
    if vals.get("kernel_sources_sha256") != sources_digest(files) or not (
            "hbm_bytes_per_site_update" in vals or "hbm_bytes_per_unit" in vals):
        return None
    return float(vals.get("hbm_bytes_per_site_update", vals.get("hbm_bytes_per_unit")))


class Bench:
    def __init__(self, name="c3", m0=None):
        import torch

        import latgen
        from paper_1202_2462_amd import mgdd
        self.torch, self.mgdd, self.latgen = torch, mgdd, latgen
        self.name = name
        w = dict(latgen.WORKLOADS[name])
        self.w = w
        base = "c1" if name in REPS else name      # the field the workload is made of
        small = tuple(latgen.WORKLOADS[base]["dims"])
        self.reps = REPS.get(name, 1)
        self.dims = tuple(self.reps * L for L in small)
        assert self.dims == tuple(w["dims"])
        self.block, self.agg, self.N = tuple(w["block"]), tuple(w["agg"]), w["ntv"]
        self.V = int(np.prod(self.dims))
        self.Vc = self.V // int(np.prod(self.agg))
        self.m0, self.csw = (load_m0(base) if m0 is None else m0), w["csw"]
        k = int(name[1:])
        t0 = time.time()
        self.U_small = latgen.workload_gauge(base)
        log(f"gauge field {small} generated in {time.time() - t0:.1f} s")
        self.lat = mgdd.Lattice(self.dims, self.block)
        # inputs resident in HBM before any timed region: the gauge field
        # (repeated on the device), the Arnoldi start vector and the
        # right-hand side; the setup's random vectors are drawn by the
        # library from a seeded stream of its counter-based generator
        Us = torch.tensor(self.U_small.view(np.float64), device="cuda")
        Us = Us.reshape(small[3], small[2], small[1], small[0], 4, 3, 3, 2)
        self.U_dev = Us.repeat(self.reps, self.reps, self.reps, self.reps, 1, 1, 1, 1).contiguous()
        del Us
        self.tv_seed = 1000 * k + latgen.TAG_TV
        st = latgen.gaussian_vector(self.Vc * 2 * self.N, 1000 * k + latgen.TAG_ARNOLDI)
        self.start = torch.tensor(np.stack([st.real, st.imag], -1), dtype=torch.float64, device="cuda")
        gen = torch.Generator(device="cuda")
        gen.manual_seed(1000 * k + latgen.TAG_RHS)
        self.b = torch.randn((1, 12, self.V, 2), dtype=torch.float64, device="cuda", generator=gen)
        torch.cuda.synchronize()

    # one pass of the hot path
    def step(self, setup_prec=None, solve_prec=None, split=None):
        mg, w = self.mgdd, self.w
        setup_prec = mg.F32 if setup_prec is None else setup_prec
        solve_prec = mg.MIXED if solve_prec is None else solve_prec
        t0 = time.perf_counter()
        self.lat.set_gauge(self.U_dev, self.m0, self.csw)
        self.lat.setup(self.agg, None, self.start, nu=w["nu"], iota=w["iota"], mr_iters=w["mr"], prec=setup_prec,
                       ntv=self.N, seed=self.tv_seed)
        t1 = time.perf_counter()
        z, stats = self.lat.solve(self.b, precision=solve_prec, restart=w["restart"], tol=w["tol"], maxit=3000,
                                  coarse_iters=12, nu=1, mr_iters=w["mr"])
        t2 = time.perf_counter()
        if split is not None:
            split.update(setup_s=t1 - t0, solve_s=t2 - t1, iters=stats[0].iters, restarts=stats[0].restarts,
                         relres=stats[0].relres, converged=bool(stats[0].converged))
        return z, stats[0]

    def learned_step(self, boot):
        """The learned setup on this workload: the shipped network (trained on
        16^3 x 32 fields; local and gauge covariant, so it applies at any
        size) maps the random vectors the bootstrap step draws (the library's
        seeded stream), then one Schwarz round and the
        second setup part, then the same solve as the step. The plain
        bootstrap is the fallback, judged by outer iterations: when the learned
        setup's solve needs more than 10 % more of them than the bootstrap's
        (`boot`, the step's split), the cost of the learned attempt is added to
        a bootstrap step. The library itself falls back when the network's
        vectors cannot form P (mgdd_setup_fallback)."""
        mg, torch, w = self.mgdd, self.torch, self.w
        d = np.load(os.path.join(ROOT, "paper_1202_2462_amd", "learned_weights_16x16x16x32.npz"))
        widths = [int(t) for t in d["widths"]]
        W = self.lat.weights_to_dev([d[f"W{l}"] for l in range(len(widths) - 1)])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        self.lat.set_gauge(self.U_dev, self.m0, self.csw)
        # the random vectors the bootstrap step draws (same stream and seed)
        self.lat.setup_learned(widths, W, self.agg, None, self.start, nu=1, iota=w["iota"], mr_iters=w["mr"],
                               n_part2=1, prec=mg.F32, ntv=self.N, seed=self.tv_seed)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        z, stats = self.lat.solve(self.b, precision=mg.MIXED, restart=w["restart"], tol=w["tol"], maxit=3000,
                                  coarse_iters=12, nu=1, mr_iters=w["mr"])
        t2 = time.perf_counter()
        del z
        out = dict(network_widths=widths, setup_s=t1 - t0, solve_s=t2 - t1, iters=stats[0].iters,
                   relres=stats[0].relres, converged=bool(stats[0].converged),
                   library_fallback=self.lat.setup_fell_back(), bootstrap_iters=boot["iters"])
        worse = (not stats[0].converged) or stats[0].iters > 1.1 * boot["iters"]
        out["fallback"] = bool(worse)
        out["seconds_with_fallback"] = (t2 - t0) + (boot["setup_s"] + boot["solve_s"] if worse else 0.0)
        return out

    def comparator(self, solver):
        mg = self.mgdd
        t0 = time.perf_counter()
        z, stats = self.lat.solve(self.b, solver=solver, restart=16, tol=self.w["tol"], maxit=200000)
        out = dict(seconds=time.perf_counter() - t0, iters=stats[0].iters, relres=stats[0].relres,
                   converged=bool(stats[0].converged))
        if solver == mg.SOLVER_CGN:
            out["restarts"] = stats[0].restarts
        del z
        return out

    def launch_times(self, fn, n=100, warm=10):
        """median duration of n launches (HIP events on torch's current
        stream, the stream the library was created on), after warm ones"""
        torch = self.torch
        for _ in range(warm):
            fn()
        s = torch.cuda.current_stream()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
        for a, b in ev:
            a.record(s)
            fn()
            b.record(s)
        torch.cuda.synchronize()
        return float(np.median([a.elapsed_time(b) for a, b in ev])) * 1e-3

    def op_rates(self):
        """Wilson-clover apply (FP64, FP32, half spinors, FP32 x 12 fields)
        and one FP32 Schwarz sweep (two colour launches) at this size"""
        mg, torch = self.mgdd, self.torch
        out = {}
        for prec, pname, nrhs in ((mg.F64, "f64", 1), (mg.F32, "f32", 1), (mg.F16, "f16", 1), (mg.F32, "f32", 12)):
            x = self.lat.field(prec, nrhs)
            x.normal_()
            y = self.lat.field(prec, nrhs)
            t = self.launch_times(lambda: mg.mgdd_dirac_apply(self.lat.ctx, prec, nrhs, x, y))
            gbs = dirac_bytes(pname, nrhs) * self.V / t / 1e9
            out[pname if nrhs == 1 else f"{pname}_x{nrhs}"] = dict(
                applies_per_s=nrhs / t, us_per_launch=t * 1e6,
                algorithmic_bytes_per_launch=dirac_bytes(pname, nrhs) * self.V,
                algorithmic_gbs=gbs, frac_of_8tbs=gbs / HBM_PEAK_GBS)
            del x, y
            torch.cuda.empty_cache()
        b = self.lat.field(mg.F32, 1)
        b.normal_()
        z = self.lat.field(mg.F32, 1)
        t = self.launch_times(lambda: mg.mgdd_sap(self.lat.ctx, mg.F32, 1, None, 1, self.w["mr"], 0.0, b, z))
        gbs = SAP_BYTES_PER_SITE * self.V / t / 1e9
        out["sap_f32_sweep"] = dict(sweeps_per_s=1.0 / t, us_per_sweep=t * 1e6,
                                    algorithmic_bytes_per_sweep=SAP_BYTES_PER_SITE * self.V, algorithmic_gbs=gbs,
                                    frac_of_8tbs=gbs / HBM_PEAK_GBS)
        return out

    def copy_rate(self):
        """device-to-device copy of 1 GiB (read + write), the attainable
        stream ceiling the stencil rates can be read against"""
        torch = self.torch
        x = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
        y = torch.empty_like(x)
        t = self.launch_times(lambda: y.copy_(x), n=20, warm=3)
        del x, y
        return 2 * (1 << 30) / t / 1e9


def cpu_baseline(bench, gpu_split):
    """The oracle on the host cores, on a bounded sample: the 16^3 x 32 field
    the workload repeats (1/81 of the sites). Timed there: the Wilson-clover
    apply and one Schwarz sweep (all cores and one thread), the full bootstrap
    setup (FP64) and 10 iterations of the two-level FGMRES(30). The oracle's
    loops are site-local, so its time per site does not depend on the lattice
    size: the solve rate at 48^3 x 96 is taken as 1 / (81 x (setup +
    iterations x time per iteration)) with the GPU step's iteration count."""
    import ctypes
    import platform

    import latgen
    import oracle
    from oracle import solvers
    w = bench.w
    base = "c1" if bench.name in REPS else bench.name
    small = tuple(latgen.WORKLOADS[base]["dims"])
    scale = bench.V / int(np.prod(small))
    op = solvers.Operator(small, bench.U_small, bench.m0, bench.csw)
    psi = latgen.gaussian_fields(small, 1, 1000 * int(bench.name[1:]) + latgen.TAG_RHS)[0]
    gomp = ctypes.CDLL("libgomp.so.1")
    nthreads = oracle.num_threads()

    def timed(fn, n):
        fn()
        t0 = time.perf_counter()
        for _ in range(n):
            fn()
        return (time.perf_counter() - t0) / n

    zero = np.zeros_like(psi)
    per_op = {}
    for threads in (nthreads, 1):
        gomp.omp_set_num_threads(threads)
        d = timed(lambda: op.apply(psi), 10 if threads > 1 else 2)
        s = timed(lambda: op.sap(bench.block, psi, zero, 1, w["mr"]), 3 if threads > 1 else 1)
        key = "all_cores" if threads > 1 else "one_thread"
        per_op[key] = {"threads": threads, "dirac_apply_s_at_workload": d * scale, "sap_sweep_s_at_workload": s * scale,
                       "dirac_apply_ns_per_site": d / op.A.shape[0] * 1e9, "sap_sweep_ns_per_site": s / op.A.shape[0] * 1e9}
    gomp.omp_set_num_threads(nthreads)
    rnd = latgen.gaussian_fields(small, bench.N, 1000 * 1 + latgen.TAG_TV)
    st = latgen.gaussian_vector(int(np.prod(small)) // int(np.prod(bench.agg)) * 2 * bench.N,
                                1000 * 1 + latgen.TAG_ARNOLDI)
    t0 = time.perf_counter()
    _, tl = solvers.bootstrap(op, bench.block, bench.agg, bench.N, w["nu"], w["iota"], w["mr"], rnd, st)
    t_setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    _, so = solvers.fgmres(op.apply, tl.precond, psi, w["restart"], w["tol"], 10)
    t_iters = time.perf_counter() - t0
    per_iter = t_iters / max(so.iters, 1)
    iters = gpu_split["iters"]
    total = scale * (t_setup + per_iter * iters)
    cpu = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    cpu = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    sample = ("oracle FP64 on the 16^3 x 32 field the workload repeats (1/%d of its sites): bootstrap setup in full "
              "(%.1f s), %d iterations of two-level FGMRES(%d) (%.1f s), Wilson-clover applies and Schwarz sweeps with "
              "all cores and one thread; time per solve = %d x (setup + %d GPU iterations x time per iteration)"
              % (round(scale), t_setup, so.iters, w["restart"], t_iters, round(scale), iters))
    return dict(value=1.0 / total, unit="solves/s", cores=nthreads, kind="oracle", sample=sample,
                seconds_per_solve=total, cpu_model=cpu, nproc=os.cpu_count(), platform=platform.machine(),
                setup_s_sample=round(t_setup, 3), seconds_per_iteration_sample=round(per_iter, 4), per_op=per_op)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=["c3", "c2", "c1"], default="c3")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-compare", action="store_true")
    ap.add_argument("--kernel-only", choices=["step", "sap", "dirac", "coarse", "coarse12"], default=None)
    ap.add_argument("--m0", type=float, default=None, help="override the tuned bare mass")
    ap.add_argument("--autotune", action="store_true",
                    help="run the Schwarz block-shape and lanes-per-site autotuner on the workload's batched "
                         "12-point-source solve instead of the benchmark")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU: the library drives one device per process and "
                                   "bench.py measures one GPU; run it with --gpus 1"}))
        sys.exit(2)

    import torch
    bench = Bench(args.workload, m0=args.m0)
    mg = bench.mgdd
    lat = bench.lat

    if args.autotune:
        from paper_1202_2462_amd.autotune import tune_sap_block
        w = bench.w
        k = int(bench.name[1:])
        b = bench.latgen.point_sources(bench.dims, 1000 * k + bench.latgen.TAG_RHS)
        cands = [(4, 4, 4, 4), (2, 4, 4, 4), (4, 4, 4, 2), (4, 4, 2, 2)]
        lat.close()
        t0 = time.time()
        res = tune_sap_block(bench.dims, bench.U_dev, bench.m0, bench.csw, bench.agg, None, bench.start, b,
                             nu=w["nu"], iota=w["iota"], mr_iters=w["mr"], restart=w["restart"], tol=w["tol"],
                             maxit=3000, lanes=(2, 4), candidates=cands,
                             setup_kwargs=dict(ntv=bench.N, seed=bench.tv_seed), log=log)
        print(json.dumps({"autotune": "Schwarz block shape x lanes per site", "workload": bench.name,
                          "dims": bench.dims, "rhs": "12 point sources (one site, every spin and colour), batched",
                          "setup": "bootstrap, FP32 sweeps, N = %d, nu = iota = %d" % (bench.N, w["nu"]),
                          "solve": "FGMRES(%d) mixed precision, tol %g" % (w["restart"], w["tol"]),
                          "seconds_total": time.time() - t0, **res}))
        return

    if args.kernel_only:
        # short run of one kernel family for hardware counters (rocprofv3 --pmc)
        lat.set_gauge(bench.U_dev, bench.m0, bench.csw)
        if args.kernel_only == "step":
            bench.step()
        elif args.kernel_only == "coarse":
            # five coarse GMRES(12) solves of one FP32 right-hand side (the
            # coarse step kernel of the solve, on the compact FP32 D_c), D_c
            # from the workload's number of random test vectors
            lat.setup(bench.agg, None, bench.start, nu=0, iota=0, mr_iters=4, n_part2=0, prec=mg.F32,
                      ntv=bench.N, seed=bench.tv_seed)
            cb = lat.coarse_field(mg.F32, 1)
            cb.normal_()
            for _ in range(5):
                lat.coarse_solve(cb, 12)
        elif args.kernel_only == "coarse12":
            # D_c from the workload's number of random test vectors (no
            # smoothing), applied to 12 FP32 right-hand sides: the matrix-core path
            lat.setup(bench.agg, None, bench.start, nu=0, iota=0, mr_iters=4, n_part2=0, prec=mg.F32,
                      ntv=bench.N, seed=bench.tv_seed)
            x = lat.coarse_field(mg.F32, 12)
            x.normal_()
            y = torch.empty_like(x)
            for _ in range(10):
                mg.mgdd_coarse_apply(lat.ctx, mg.F32, 12, x, y)
        elif args.kernel_only == "sap":
            b = lat.field(mg.F32, 1)
            b.normal_()
            z = lat.field(mg.F32, 1)
            for _ in range(5):
                mg.mgdd_sap(lat.ctx, mg.F32, 1, None, 1, bench.w["mr"], 0.0, b, z)
        else:
            for prec in (mg.F64, mg.F32):
                x = lat.field(prec, 1)
                x.normal_()
                y = lat.field(prec, 1)
                for _ in range(5):
                    mg.mgdd_dirac_apply(lat.ctx, prec, 1, x, y)
        torch.cuda.synchronize()
        x = torch.empty(256 * 1024 * 1024 // 4, dtype=torch.float32, device="cuda").normal_()
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)    # reference copy (runtime blit kernel): 256 MiB read + 256 MiB written
        for _ in range(5):
            torch.add(x, 0.5, out=y)    # reference elementwise kernel: 256 MiB read + 256 MiB written
        torch.cuda.synchronize()
        print(json.dumps({"kernel_only": args.kernel_only, "workload": bench.name,
                          "copy_bytes_each_way": x.numel() * 4}))
        return

    for i in range(args.warmup):
        t0 = time.perf_counter()
        bench.step()
        torch.cuda.synchronize()
        log(f"warmup step {i + 1}/{args.warmup}: {time.perf_counter() - t0:.2f} s")
    ctx = lat.ctx
    for kern, prec in ((mg.KERNEL_SAP, mg.F32), (mg.KERNEL_DIRAC, mg.F64), (mg.KERNEL_COARSE, mg.F32)):
        mg.mgdd_timing_read(ctx, kern, prec, reset=True)
    mg.mgdd_timing_enable(ctx, True)    # HIP events around each launch, on the library's stream
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    last = None
    for i in range(args.steps):
        _, last = bench.step()
        log(f"timed step {i + 1}/{args.steps}: {last.iters} iterations, relres {last.relres:.2e}, "
            f"{time.perf_counter() - t0:.2f} s so far")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    mg.mgdd_timing_enable(ctx, False)
    sap_ms, sap_units, sap_n, sap_bytes = mg.mgdd_timing_read(ctx, mg.KERNEL_SAP, mg.F32, reset=True)
    c_ms, c_units, c_n, c_bytes = mg.mgdd_timing_read(ctx, mg.KERNEL_COARSE, mg.F32, reset=True)
    d_ms, d_units, d_n, d_bytes = mg.mgdd_timing_read(ctx, mg.KERNEL_DIRAC, mg.F64, reset=True)
    ms = elapsed / args.steps * 1e3
    split = {}
    bench.step(split=split)
    log("split", split)

    big = bench.name == "c3"
    result = {
        "metric": "Dirac applies/s + HBM GB/s; time-to-1e-10 solve vs plain FP64 GCR (1 GPU)",
        "value": 1000.0 / ms,
        "unit": "solves/s (gauge ingest + bootstrap setup + mixed-precision FGMRES to 1e-10, 1 RHS)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 (smoother, transfers, coarse solve) + f64 (outer FGMRES, true residual)",
        "data": "synthetic (seeded SU(3) links exp(i eps H) + 2 APE steps; Gaussian random vectors and RHS)",
        "config": {"workload": ("%s Wilson-clover c_sw=1.0; gauge field = the 16^3x32 workload field (eps 0.5, 2 APE "
                                "steps, seed 1001) repeated %dx per direction, bare mass of that field (min Re eig "
                                "0.01 at 16^3x32); SAP blocks 4^4, 4 MR steps, 1 sweep; aggregates 4^4, %d test "
                                "vectors, 3+3 bootstrap sweeps (FP32); FGMRES(%d), tol 1e-10"
                                % ("x".join(map(str, bench.dims)), bench.reps, bench.N, bench.w["restart"])),
                   "lattice": list(bench.dims), "sites": bench.V, "m0": bench.m0, "global_batch": 1,
                   "parallelism": "single GPU"},
        "time_to_solution": {"mg_mixed": split},
    }
    if last is not None:
        result["time_to_solution"]["mg_mixed"]["converged_in_timed_steps"] = bool(last.converged)

    if not args.no_compare:
        log("multilevel with half-precision storage in the preconditioner")
        s16 = {}
        try:
            bench.step(solve_prec=mg.MIXED_F16, split=s16)
        except mg.MgddError as e:
            s16 = {"error": str(e)}
        result["time_to_solution"]["mg_mixed_f16"] = s16
        lat.release_workspace()
        log("learned setup (shipped network), the bootstrap as fallback")
        try:
            bench.learned_step(split)     # warm: the network's and the solve's workspaces
            result["time_to_solution"]["mg_learned"] = bench.learned_step(split)
        except mg.MgddError as e:
            result["time_to_solution"]["mg_learned"] = {"error": str(e)}
        lat.release_workspace()
        torch.cuda.empty_cache()
        log("plain FP64 multilevel")
        s64 = {}
        try:
            lat.release_workspace()
            torch.cuda.empty_cache()
            bench.step(setup_prec=mg.F64, solve_prec=mg.PLAIN_F64, split=s64)
        except mg.MgddError as e:
            s64 = {"error": str(e)}
        result["time_to_solution"]["mg_fp64"] = s64
        lat.release_workspace()
        log("even-odd FP64 GCR(16)")
        result["time_to_solution"]["gcr_eo_fp64"] = bench.comparator(mg.SOLVER_GCR_EO)
        log("plain FP64 CGN")
        result["time_to_solution"]["cgn_fp64"] = bench.comparator(mg.SOLVER_CGN)
        if not big:
            log("plain FP64 GCR(16)")
            result["time_to_solution"]["gcr_fp64"] = bench.comparator(mg.SOLVER_GCR)
        tts = result["time_to_solution"]
        mgt = tts["mg_mixed"]["setup_s"] + tts["mg_mixed"]["solve_s"]
        for k in ("gcr_eo_fp64", "gcr_fp64", "cgn_fp64"):
            if k in tts:
                result[f"speedup_vs_{k}"] = {"solve_only": tts[k]["seconds"] / tts["mg_mixed"]["solve_s"],
                                             "with_setup": tts[k]["seconds"] / mgt}
        lat.release_workspace()

    torch.cuda.empty_cache()
    log("per-operation rates")
    lat.set_gauge(bench.U_dev, bench.m0, bench.csw)
    rates = bench.op_rates()
    result["dirac"] = {k: v for k, v in rates.items() if not k.startswith("sap")}
    result["sap"] = rates["sap_f32_sweep"]
    result["stream_copy_gbs"] = bench.copy_rate()
    if d_n:
        result["dirac"]["f64_in_timed_steps"] = {
            "launches": d_n, "us_per_launch": d_ms * 1e3 / d_n, "site_updates": d_units,
            "algorithmic_gbs": d_bytes / (d_ms * 1e-3) / 1e9,
            "note": "FP64 applies of the solve (FP32 input widened in the kernel) and of the setup, each launch "
                    "charged its own algorithmic bytes (links and clover term once per launch)"}
    # rooflines over the timed steps (HIP events around each launch on the
    # library's stream). The Schwarz colour kernel: 768 algorithmic bytes (the
    # library's count for the two-lanes kernel: links as two rows) and
    # sap_flops_per_site(4) = 10 824 flops per site update for one right-hand
    # side, 14.1 flop/B, below the FP32 ridge of 157.3 TFLOP/s / 8 TB/s =
    # 19.7 flop/B. The coarse GMRES step (y = D_c v_j on the compact FP32
    # blocks with the Arnoldi dot products): per coarse site 5 (2N)^2 complex
    # FP32 block entries (read once per launch) and (3 + j) 2N vector entries,
    # 8 (2N)^2 * 9 / (5 (2N)^2 8) = 1.8 flop/B. Both bound by HBM bandwidth.
    lines = {}
    if sap_n:
        t_launch = sap_ms * 1e-3 / sap_n
        units_launch = sap_units / sap_n
        bytes_launch = sap_bytes / sap_n
        achieved = bytes_launch / t_launch / 1e9
        tps = counter_traffic(TRAFFIC_FILE, SAP_SOURCES) if big else None
        lines["sap"] = (sap_ms, {
            "bound": "hbm", "kernel": "sapc_kernel<256> (FP32 Schwarz colour step, 4 MR steps)",
            "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
            "traffic": None if tps is None else tps * units_launch,
            "launches": sap_n, "us_per_launch": t_launch * 1e6, "total_ms_in_timed_steps": sap_ms,
            "site_updates_per_launch": units_launch,
            "algorithmic_bytes_per_launch": bytes_launch,
            "algorithmic_flops_per_launch": sap_flops_per_site(bench.w["mr"]) * units_launch,
            "tflops": sap_flops_per_site(bench.w["mr"]) * units_launch / t_launch / 1e12,
            "fp32_peak_tflops": FP32_PEAK_TFLOPS})
    if c_n:
        t_launch = c_ms * 1e-3 / c_n
        units_launch = c_units / c_n
        bytes_launch = c_bytes / c_n
        achieved = bytes_launch / t_launch / 1e9
        tpc = counter_traffic(COARSE_TRAFFIC_FILE, COARSE_SOURCES) if big else None
        n2 = 2 * bench.N
        lines["coarse"] = (c_ms, {
            "bound": "hbm", "kernel": "arnoldi_apply_kernel<float, true> (coarse GMRES step on the compact FP32 "
                                      "D_c: self block and forward hops stored, backward hops from "
                                      "gamma5^c-hermiticity)",
            "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
            "traffic": None if tpc is None else tpc * units_launch,
            "launches": c_n, "us_per_launch": t_launch * 1e6, "total_ms_in_timed_steps": c_ms,
            "coarse_sites_per_launch": units_launch, "algorithmic_bytes_per_launch": bytes_launch,
            "tflops": 8.0 * 9 * n2 * n2 * units_launch / t_launch / 1e12})
    if lines:
        order = sorted(lines, key=lambda k: -lines[k][0])
        result["roofline"] = lines[order[0]][1]
        if len(order) > 1:
            result["roofline_other"] = lines[order[1]][1]

    if not args.no_cpu:
        log("cpu baseline (oracle)")
        result["cpu_baseline"] = cpu_baseline(bench, split)
    print(json.dumps(result))


if __name__ == "__main__":
    main()
