"""Write tests/golden/oracle_full_size.json, oracle_batched64x16.json,
oracle_learned128.json and oracle_paper300.json from the CPU oracle alone.

Runs the oracle (and the seeded input generators) on the full-size
workloads whose end-to-end results the GPU tests cannot recompute within a
test's time limit, and stores iteration counts, residuals, hierarchy sizes,
sampled entries of one V-cycle (binary64 and binary32) as hex floats, and
SHA-256 digests of whole arrays (every level's CSR arrays, l1 diagonal,
smooth vector, aggregate map and P values, and the whole V-cycle outputs),
so that the GPU tests compare complete results bit for bit.  The batched record
covers sampled (system, right-hand side) pairs of the 64-system x 16
right-hand-side batch: the oracle's mixed-precision PCG and binary32 V-cycle
of each pair's own system.  The learned record holds the network's forward
prediction (float64 with bfloat16 storage emulated) on the 128^3 log-normal
field with seeded initial weights: sampled entries and the norm of the whole
vector.
The paper record holds the oracle's hierarchy digests and PCG result for the
paper's own configuration (Sec. 5: s = 3, coarsest <= 40 nd by 20 sweeps,
f = 1) at 300^3.
Usage: python tests/golden/make_oracle_golden.py [all|single|batched|learned|paper]
"""
import hashlib
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


def digest(a, dtype):
    """SHA-256 of the array's little-endian bytes as `dtype` (int32 / float64)."""
    return hashlib.sha256(np.ascontiguousarray(a, dtype=np.dtype(dtype).newbyteorder("<")).tobytes()).hexdigest()


def level_digests(H):
    out = []
    for k in range(H.nlevels):
        lv = H.level(k)
        rec = dict(row_ptr=digest(lv["row_ptr"], np.int32), col=digest(lv["col"], np.int32),
                   val=digest(lv["val"], np.float64), dinv=digest(lv["dinv"], np.float64),
                   w=digest(lv["w"], np.float64))
        if k < H.nlevels - 1:
            rec["agg"] = digest(lv["agg"], np.int32)
            rec["pval"] = digest(lv["pval"], np.float64)
        out.append(rec)
    return out


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
               vcycle=dict(r_seed=VCYCLE_SEED, rows=rows, z=[float(z[i]).hex() for i in rows],
                           sha256=digest(z, np.float64)),
               level_sha256=level_digests(H))
    if f32:
        z32 = H.vcycle_f32(r)
        rec["vcycle_f32"] = dict(r_seed=VCYCLE_SEED, rows=rows, z=[float(z32[i]).hex() for i in rows],
                                 sha256=digest(z32, np.float64))
        xm, itm, relm, stm = H.pcg(b, rtol=1e-6, maxit=1000, mixed=True)
        rec["mixed"] = dict(status=stm, iterations=itm, relres=relm)
    print(json.dumps({k: v for k, v in rec.items() if k not in ("vcycle", "vcycle_f32", "level_sha256")}),
          flush=True)
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


# The paper's configuration (Sec. 5 and Appendix A) on 300^3 Poisson with the
# unit right-hand side: parameters from tests/golden/paper_hierarchy.json.
PAPER_ND = 300


def run_paper():
    g = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_hierarchy.json")))
    gp = g["params"]
    params = oracle.AMGParams(aggr_steps=gp["aggr_steps"], coarse_max=gp["coarse_max_per_nd"] * PAPER_ND,
                              max_levels=gp["max_levels"], coarse_solver=1,
                              coarse_sweeps=gp["coarse_sweeps"], pre_sweeps=gp["pre_sweeps"],
                              post_sweeps=gp["post_sweeps"])
    A = W.poisson7(PAPER_ND)
    t0 = time.time()
    H = oracle.Hierarchy(A, params)
    t1 = time.time()
    b = np.ones(A.n)
    x, it, rel, st = H.pcg(b, rtol=1e-6, maxit=1000)
    t2 = time.time()
    rec = dict(workload="poisson7_300 paper configuration, b = 1", nd=PAPER_ND, status=st, iterations=it,
               relres=rel, levels=[list(s) for s in H.sizes()], opc=H.opc(),
               oracle_setup_s=t1 - t0, oracle_solve_s=t2 - t1,
               params={k: int(v) for k, v in params.__dict__.items()},
               solution_sha256=digest(x, np.float64), level_sha256=level_digests(H))
    print(json.dumps({k: v for k, v in rec.items() if k != "level_sha256"}), flush=True)
    return rec


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
    if which in ("all", "paper"):
        write("oracle_paper300.json", run_paper())


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "all")
