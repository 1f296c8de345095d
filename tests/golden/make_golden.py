"""Write oracle reference values for full-size workloads (FP64 CPU oracle only).

    python tests/golden/make_golden.py c2 [--tol 1e-9] [--seed 0]

Writes tests/golden/oracle_<name>_s<seed>.json with E_G, the Ritz values,
iteration count and residuals of ``oracle.solve``.  Nothing here touches the
GPU library.
"""

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from workloads import config_problem  # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("name")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--tol", type=float, default=1e-9)
    ap.add_argument("--k-rot", type=int, default=50)
    ap.add_argument("--max-iter", type=int, default=20000)
    a = ap.parse_args()
    p = config_problem(a.name, seed=a.seed)
    H = oracle.csr_matrix(*p.csr(), p.N)
    t0 = time.time()

    def progress(i, E, rho):
        if i % 25 == 0:
            print(f"it {i} E {E:.15e} rho {rho:.3e} t {time.time() - t0:.0f}s", flush=True)

    r = oracle.solve(H, p.C0(), oracle.OracleOptions(tol=a.tol, k_rot=a.k_rot,
                                                      max_iter=a.max_iter), callback=progress)
    out = dict(config=a.name, seed=a.seed, N=p.N, m=p.m, tol=a.tol, k_rot=a.k_rot,
               E_G=r.E_G, eigenvalues=[float(x) for x in r.eigenvalues],
               iterations=r.iterations, converged=r.converged,
               max_residual=r.max_residual, frob_residual=r.frob_residual,
               orth_err=r.orth_err, restarts=r.restarts,
               energies_first=[float(x) for x in r.energies[:200]],
               seconds=time.time() - t0,
               generator="tests/golden/make_golden.py (oracle.solve, FP64 CPU)")
    path = os.path.join(HERE, f"oracle_{a.name}_s{a.seed}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path, "E_G", r.E_G, "iterations", r.iterations, flush=True)


if __name__ == "__main__":
    main()
