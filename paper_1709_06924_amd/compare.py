"""Method comparison of section 4.1 (Tables 1 and 2): Lloyd, plain LBFGS and
Lloyd-preconditioned LBFGS on the same start, with the paper's stopping
tests -- at most 2,000 iterations, point movement (max |l_ik|) below 5e-4,
and for the quasi-Newton methods |grad F| / F <= 5e-4 or |dF| / F < 1e-7.

    python -m paper_1709_06924_amd.compare [--n 2562] [--seed 31] [--densities x3,x16,x64]

Each density is integrated with the rule size the paper uses for it
(4 points for X3 and X16, 9 for X64).  Starts are seeded uniform points
(the paper samples its densities by Monte Carlo), so absolute iteration
counts differ from the paper's; the comparison is between the methods on a
common start.
"""
import argparse
import json
import time

from . import inputs as I
from . import scvt

PAPER_TESTS = dict(max_iter=2000, step_tol=5e-4, grad_rel_tol=5e-4, f_rel_tol=1e-7)
DENSITIES = {"x3": I.density_x3, "x16": I.density_x16, "x64": I.density_x64}
PAPER_RULE = {"x3": 4, "x16": 4, "x64": 9}


def run_method(Z0, density, method, m_hist=7, precision="fp64", tests=PAPER_TESTS, quad_rule=7):
    S = scvt.Solver(Z0, density, method=method, m_hist=m_hist, precision=precision,
                    quad_rule=quad_rule)
    t0 = time.perf_counter()
    info = S.solve_rel(**tests)
    dt = time.perf_counter() - t0
    S.close()
    return {"method": method, "iterations": info["iter"], "evaluations": info["n_evals"],
            "F": info["F"], "grad_norm": info["grad_norm2"], "step_inf": info["step_inf"],
            "converged": info["converged"], "seconds": dt}


def compare(n=2562, seed=31, densities=("x3", "x16", "x64"), methods=("lloyd", "lbfgs", "plbfgs")):
    Z0 = I.uniform_sphere(n, seed)
    rows = []
    for dn in densities:
        for m in methods:
            r = run_method(Z0, DENSITIES[dn](), m, quad_rule=PAPER_RULE[dn])
            r["density"] = dn
            r["n"] = n
            rows.append(r)
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=2562)
    ap.add_argument("--seed", type=int, default=31)
    ap.add_argument("--densities", default="x3,x16,x64")
    args = ap.parse_args()
    rows = compare(args.n, args.seed, args.densities.split(","))
    print("%-5s %-7s %6s %6s %14s %12s %10s %9s" % ("rho", "method", "iter", "evals", "F", "|grad F|",
                                                      "step_inf", "seconds"))
    for r in rows:
        print("%-5s %-7s %6d %6d %14.8e %12.4e %10.3e %9.3f" % (
            r["density"], r["method"], r["iterations"], r["evaluations"], r["F"], r["grad_norm"],
            r["step_inf"], r["seconds"]))
    print(json.dumps(rows))


if __name__ == "__main__":
    main()
