"""Write tests/golden/oracle_full_size.json and oracle_batched64x16.json from
the CPU oracle alone.

Runs the oracle (and the seeded input generators) on the full-size
workloads whose end-to-end results the GPU tests cannot recompute within a
test's time limit, and stores iteration counts, residuals, hierarchy sizes and sampled entries
of one V-cycle (binary64 and binary32) as hex floats.  The batched record
covers sampled (system, right-hand side) pairs of the 64-system x 16
right-hand-side batch: the oracle's mixed-precision PCG and binary32 V-cycle
of each pair's own system.  The learned record holds the network's forward
prediction (float64 with bfloat16 storage emulated) on the 128^3 log-normal
field with seeded initial weights: sampled entries and the norm of the whole
vector.
Usage: python tests/golden/make_oracle_golden.py [all|single|batched|learned]
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


# One V-cycle on a seeded residual, sampled: VCYCLE_SEED feeds the residual,
# SAMPLE_SEED the row indices (SAMPLES of them, plus the first and last row).
VCYCLE_SEED, SAMPLE_SEED, SAMPLES = 77, 78, 256


def sample_rows(n):
    idx = np.floor(W.uniform(SAMPLE_SEED, SAMPLES) * n).astype(np.int64)
    return sorted(set(idx.tolist()) | {0, n - 1})


def run(name, A, seed, params, f32=False):
    t0 = time.time()
    xs, b = W.manufactured_rhs(A, seed)
    H = oracle.Hierarchy(A, params)
    t1 = time.time()
    x, it, rel, st = H.pcg(b, rtol=1e-6, maxit=1000)
    t2 = time.time()
    true_rel = float(np.linalg.norm(b - A.scipy() @ x) / np.linalg.norm(b))
    r = W.uniform_pm1(VCYCLE_SEED, A.n)
    rows = sample_rows(A.n)
    z = H.vcycle(r)
    rec = dict(workload=name, seed=seed, status=st, iterations=it, relres=rel, true_relres=true_rel,
               levels=[list(s) for s in H.sizes()], opc=H.opc(), oracle_setup_s=t1 - t0,
               oracle_solve_s=t2 - t1, params={k: int(v) for k, v in params.__dict__.items()},
               vcycle=dict(r_seed=VCYCLE_SEED, rows=rows, z=[float(z[i]).hex() for i in rows]))
    if f32:
        z32 = H.vcycle_f32(r)
        rec["vcycle_f32"] = dict(r_seed=VCYCLE_SEED, rows=rows, z=[float(z32[i]).hex() for i in rows])
        xm, itm, relm, stm = H.pcg(b, rtol=1e-6, maxit=1000, mixed=True)
        rec["mixed"] = dict(status=stm, iterations=itm, relres=relm)
    print(json.dumps({k: v for k, v in rec.items() if k not in ("vcycle", "vcycle_f32")}), flush=True)
    return rec


# The batch: 64 systems with edges W.batched_edges(64, 5), 16 right-hand
# sides b_s = A_s X_s with X_s = W.batched_rhs(s, n_s, 16).T; the V-cycle
# residual of system s is W.uniform_pm1(BATCH_R_SEED + s, n_s * 16) as an
# (n_s, 16) row-major block.  Sampled pairs: the smallest, a median and the
# largest system, first and last column.
BATCH_NSYS, BATCH_SEED, BATCH_NRHS, BATCH_R_SEED = 64, 5, 16, 900
BATCH_COLS = (0, 15)


def batched_systems():
    edges = W.batched_edges(BATCH_NSYS, BATCH_SEED)
    order = sorted(range(BATCH_NSYS), key=lambda s: (edges[s], s))
    return edges, [order[0], order[BATCH_NSYS // 2], order[-1]]


def run_batched():
    edges, picks = batched_systems()
    pairs = []
    for s in picks:
        A = W.poisson7(edges[s])
        t0 = time.time()
        H = oracle.Hierarchy(A)
        bs = A.scipy() @ W.batched_rhs(s, A.n, BATCH_NRHS).T
        R = W.uniform_pm1(BATCH_R_SEED + s, A.n * BATCH_NRHS).reshape(A.n, BATCH_NRHS)
        rows = sample_rows(A.n)
        for c in BATCH_COLS:
            x, it, rel, st = H.pcg(np.ascontiguousarray(bs[:, c]), rtol=1e-6, maxit=1000, mixed=True)
            z32 = H.vcycle_f32(np.ascontiguousarray(R[:, c]))
            pairs.append(dict(system=s, edge=int(edges[s]), column=c, status=st, iterations=it,
                              relres=rel, rows=rows, z=[float(z32[i]).hex() for i in rows]))
        print(json.dumps(dict(system=s, edge=int(edges[s]), n=A.n, oracle_s=time.time() - t0,
                              iterations=[p["iterations"] for p in pairs if p["system"] == s])),
              flush=True)
    return dict(nsys=BATCH_NSYS, edges_seed=BATCH_SEED, nrhs=BATCH_NRHS, r_seed=BATCH_R_SEED,
                edges=[int(e) for e in edges], pairs=pairs)


# The learned form's field and weights: W.lognormal7(128, 7) (sigma^2 = 2,
# ell = 8) and oracle.mpnn.init_params(LEARN_THETA_SEED) rounded to binary32
# (the weights the device keeps).
LEARN_N, LEARN_FIELD_SEED, LEARN_THETA_SEED = 128, 7, 7


def run_learned():
    import oracle.mpnn as M
    A = W.lognormal7(LEARN_N, LEARN_FIELD_SEED)
    theta = M.init_params(LEARN_THETA_SEED).astype(np.float32).astype(np.float64)
    t0 = time.time()
    y, _ = M.forward(theta, A, bf16=True)
    rows = sample_rows(A.n)
    print(json.dumps(dict(n=A.n, oracle_forward_s=time.time() - t0)), flush=True)
    return dict(n_edge=LEARN_N, field_seed=LEARN_FIELD_SEED, theta_seed=LEARN_THETA_SEED,
                norm_y=float(np.linalg.norm(y)), rows=rows, y=[float(y[i]).hex() for i in rows])


def write(name, out):
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), name)
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


def main(which="all"):
    if which in ("all", "single"):
        out = {}
        out["poisson7_160"] = run("poisson7_160", W.poisson7(160), 2, oracle.AMGParams(), f32=True)
        out["diffusion27_128"] = run("diffusion27_128", W.diffusion27(128, 3), 4,
                                     oracle.AMGParams(smooth_vec=1), f32=True)
        write("oracle_full_size.json", out)
    if which in ("all", "batched"):
        write("oracle_batched64x16.json", run_batched())
    if which in ("all", "learned"):
        write("oracle_learned128.json", run_learned())


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "all")
