"""Write tests/golden/oracle_full_size.json from the CPU oracle alone.

Runs the oracle (and the seeded input generators) on the full-size
workloads whose end-to-end results the GPU tests cannot recompute within a
test's time limit, and stores iteration counts, residuals and hierarchy
sizes.  Usage: python tests/golden/make_oracle_golden.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import workloads as W  # noqa: E402


def run(name, A, seed, params):
    t0 = time.time()
    xs, b = W.manufactured_rhs(A, seed)
    H = oracle.Hierarchy(A, params)
    t1 = time.time()
    x, it, rel, st = H.pcg(b, rtol=1e-6, maxit=1000)
    t2 = time.time()
    true_rel = float(np.linalg.norm(b - A.scipy() @ x) / np.linalg.norm(b))
    rec = dict(workload=name, seed=seed, status=st, iterations=it, relres=rel, true_relres=true_rel,
               levels=[list(s) for s in H.sizes()], opc=H.opc(), oracle_setup_s=t1 - t0,
               oracle_solve_s=t2 - t1, params={k: int(v) for k, v in params.__dict__.items()})
    print(json.dumps(rec), flush=True)
    return rec


def main():
    out = {}
    out["poisson7_160"] = run("poisson7_160", W.poisson7(160), 2, oracle.AMGParams())
    out["diffusion27_128"] = run("diffusion27_128", W.diffusion27(128, 3), 4,
                                 oracle.AMGParams(smooth_vec=1))
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_full_size.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
