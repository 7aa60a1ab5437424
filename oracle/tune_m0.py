"""Choose the bare mass m0 of a synthetic workload so that the eigenvalue of
D(m0) with the smallest real part sits at a target value.

TEST INFRASTRUCTURE / INPUT PREPARATION: calls only the oracle. D(m0) =
D(0) + m0 (the mass enters the clover diagonal only), so
m0 = target - min Re spec D(0). The leftmost eigenvalue of D(0) comes from
implicitly restarted Arnoldi (ARPACK through scipy) on the oracle's operator.

usage: python -m oracle.tune_m0 c0 c1 [--write]
writes tests/golden/m0.json with the estimate, its residual and the recipe.
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np
import scipy.sparse.linalg as sla

import latgen
from oracle.solvers import Operator

GOLDEN = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "tests", "golden", "m0.json")


def leftmost(dims, U, csw, tol=1e-6, k=6, ncv=40):
    op = Operator(dims, U, 0.0, csw)
    n = int(np.prod(dims)) * 12
    shape = (int(np.prod(dims)), 4, 3)
    count = [0]
    t0 = time.time()

    def mv(v):
        count[0] += 1
        if count[0] % 200 == 0:
            print(f"  {count[0]} applications of D, {time.time() - t0:.0f} s", flush=True)
        return op.apply(v.reshape(shape)).ravel()

    L = sla.LinearOperator((n, n), matvec=mv, dtype=np.complex128)
    v0 = latgen.gaussian_vector(n, 12345)
    vals, vecs = sla.eigs(L, k=k, which="SR", tol=tol, v0=v0, ncv=max(ncv, 3 * k), maxiter=5000)
    i = int(np.argmin(vals.real))
    lam = vals[i]
    v = vecs[:, i]
    res = np.linalg.norm(L.matvec(v) - lam * v) / np.linalg.norm(v)
    return complex(lam), float(res)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("configs", nargs="+")
    ap.add_argument("--write", action="store_true")
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--k", type=int, default=6)
    ap.add_argument("--ncv", type=int, default=40)
    args = ap.parse_args()
    data = json.load(open(GOLDEN)) if os.path.exists(GOLDEN) else {}
    for name in args.configs:
        w = latgen.WORKLOADS[name]
        t0 = time.time()
        U = latgen.workload_gauge(name)
        lam, res = leftmost(w["dims"], U, w["csw"], tol=args.tol, k=args.k, ncv=args.ncv)
        m0 = w["target"] - lam.real
        data[name] = dict(m0=m0, leftmost_D0=[lam.real, lam.imag], residual=res, target=w["target"],
                          dims=list(w["dims"]), csw=w["csw"],
                          recipe=f"m0 = target - min Re spec D(0); ARPACK 'SR' on the oracle operator, tol {args.tol}, k {args.k}, ncv {args.ncv}",
                          seconds=round(time.time() - t0, 1))
        print(name, data[name], flush=True)
    if args.write:
        with open(GOLDEN, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
