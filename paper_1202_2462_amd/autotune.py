"""Autotuner of the Schwarz block shape and of the Schwarz kernel's thread
tile.

The block decomposition of the SAP smoother (Section 2, Algorithm 2.1) is a
free parameter of the method: smaller blocks make each colour step cheaper
and the smoother weaker, so the best shape is the one with the shortest
time to solution, setup included. The FP32 Schwarz kernel has a second,
schedule-only parameter: the lanes per lattice site (1, 2 or 4; see
mgdd_set_kernel_options). `tune_sap_block` times the whole path (gauge
ingest, bootstrap setup, FGMRES solve) through the library for every
candidate (block shape, lanes) on the same inputs and returns the fastest
converged one with the table it was chosen from. The library's site order
depends on the block shape, so every candidate gets its own context and its
own packing of the (canonical) inputs; packing is outside the timed region.

The choice changes the smoother and hence the iterates; it does not change
what is solved (every candidate's solution meets the same tolerance). The
Schwarz kernel supports blocks of 64 to 256 sites with power-of-two extents.
"""
from __future__ import annotations

import itertools
import time

import numpy as np

from . import mgdd


def candidate_blocks(dims, vmin=64, vmax=256, extents=(2, 4, 8)):
    """Block shapes the library accepts for this lattice: power-of-two extents
    that divide the lattice with an even number of blocks per direction (or
    one block), block volume in [vmin, vmax]."""
    out = []
    for blk in itertools.product(extents, repeat=4):
        vb = int(np.prod(blk))
        if not (vmin <= vb <= vmax):
            continue
        ok = True
        for L, b in zip(dims, blk):
            if L % b or (L // b > 1 and (L // b) % 2):
                ok = False
        if ok:
            out.append(tuple(blk))
    return out


def tune_sap_block(dims, U, m0, csw, agg, random_vectors, arnoldi_start, b, *, nu=3, iota=3, mr_iters=4,
                   restart=20, tol=1e-10, maxit=2000, setup_prec=mgdd.F32, precision=mgdd.MIXED, candidates=None,
                   lanes=(0,), repeats=1, log=None, setup_kwargs=None):
    """Times setup + solve for every candidate (block shape, lanes per site).

    U: canonical gauge field (host array or FP64 device tensor, as for
    mgdd_set_gauge); random_vectors: canonical (N, V, 4, 3) test-vector
    start fields, or None (the library draws them; setup_kwargs then gives
    ntv and seed); arnoldi_start: device tensor of the coarse start vector;
    b: canonical (nrhs, V, 4, 3) right-hand sides (solved together, batched).
    lanes: the lanes-per-site values tried with every shape (0: the
    library's automatic choice). Returns {"best": shape, "best_lanes": l,
    "results": [{"block", "lanes", "seconds", "setup_s", "solve_s", "iters",
    "converged"} or {"block", "lanes", "error"}, ...]} with the fastest
    converged candidate, the minimum over `repeats` timings per candidate; a
    candidate the library cannot run (MGDD_ESHAPE, e.g. two lanes per site
    without special unitary links) is listed with its error."""
    import torch
    cands = candidate_blocks(dims) if candidates is None else [tuple(c) for c in candidates]
    if not cands:
        raise ValueError("no admissible Schwarz block shape for this lattice")
    results = []
    for blk, nl in itertools.product(cands, lanes):
        lat = mgdd.Lattice(dims, blk)
        try:
            mgdd.mgdd_set_kernel_options(lat.ctx, sap_lanes=nl)
            rnd = None if random_vectors is None else lat.pack(random_vectors, mgdd.F64)
            bb = lat.pack(b, mgdd.F64)
            best = None
            for _ in range(repeats):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                lat.set_gauge(U, m0, csw)
                lat.setup(agg, rnd, arnoldi_start, nu=nu, iota=iota, mr_iters=mr_iters, prec=setup_prec,
                          **(setup_kwargs or {}))
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                z, stats = lat.solve(bb, precision=precision, restart=restart, tol=tol, maxit=maxit,
                                     mr_iters=mr_iters, allow_noconv=True)
                torch.cuda.synchronize()
                t2 = time.perf_counter()
                rec = dict(block=blk, lanes=nl, seconds=t2 - t0, setup_s=t1 - t0, solve_s=t2 - t1,
                           iters=max(s.iters for s in stats), converged=all(bool(s.converged) for s in stats))
                if best is None or rec["seconds"] < best["seconds"]:
                    best = rec
                del z
            results.append(best)
            if log:
                log(f"block {blk}, lanes {nl}: {best['seconds'] * 1e3:.1f} ms, {best['iters']} iterations"
                    f"{'' if best['converged'] else ' (not converged)'}")
        except mgdd.MgddError as e:
            if e.code != mgdd.ESHAPE:
                raise
            results.append(dict(block=blk, lanes=nl, error=str(e)))
            if log:
                log(f"block {blk}, lanes {nl}: not runnable ({e})")
        finally:
            lat.close()
            torch.cuda.empty_cache()
    ok = [r for r in results if r.get("converged")]
    if not ok:
        raise RuntimeError("no candidate reached the tolerance")
    win = min(ok, key=lambda r: r["seconds"])
    return {"best": win["block"], "best_lanes": win["lanes"], "results": results}
