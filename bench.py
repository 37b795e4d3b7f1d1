"""Benchmark: AMG-PCG on 3D Poisson 160^3 (7-point, FP64) on one MI355X.

One step = one pass of the whole path on the resident input: amg_setup
(smooth vector, matching, aggregation, Galerkin products, coarsest factor)
followed by amg_pcg_solve from x0 = 0 to a relative residual of 1e-6.
`value` is the PCG solve time in seconds (HIP events on the hierarchy's
stream around amg_pcg_solve, mean over the timed steps).

Printed JSON line (rank 0): the contract fields plus
  roofline      the fine-level l1-Jacobi sweep on binary64 value arrays
                (7 of the 9 fine-level matrix passes of an iteration are
                sweeps): plain-CSR algorithmic bytes per launch
                ((8 + 4) nnz + 4 (n + 1) + 3 * 8 n) / mean launch time (HIP
                events on the library stream, the solve's launch
                configuration), against 8 TB/s HBM;
  cpu_baseline  the CPU oracle on the same 160^3 system: single thread, and
                its OpenMP timing build on all allowed threads;
  detail        setup/solve split, iterations, per-kernel GB/s, the coded
                sweep the default solve runs, and the other forms.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
N_EDGE = 160
SEED = 2
RTOL = 1e-6
MAXIT = 1000
METRIC = "AMG-PCG solve s & SpMV GB/s, 3D Poisson 160³ FP64 vs mixed/learned"


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("solve.hip", "amg_internal.hpp"):
        h.update(open(os.path.join(ROOT, "paper_2303_02352_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(kernel_name, algorithmic_bytes):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when it is missing or was taken on a different kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic_%s.txt" % kernel_name)
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("source_hash") != kernel_source_hash():
        return None
    return rec.get("hbm_bytes_per_launch")


def cpu_baseline(A, b, runs=3):
    """The CPU oracle on the same 160^3 system: 1 warm-up solve and `runs`
    timed solves (median), (i) the parity oracle as it stands, one thread;
    (ii) the OpenMP timing build of the same source (-O3 -march=native, rows
    of SpMV / sweeps / residuals / prolongation / updates split over all
    threads OMP_NUM_THREADS allows, setup sequential)."""
    import numpy as np
    import oracle

    def leg(timing):
        t0 = time.perf_counter()
        H = oracle.Hierarchy(A, timing=timing)
        t_setup = time.perf_counter() - t0
        times, it, rel = [], 0, 0.0
        for rep in range(runs + 1):
            t1 = time.perf_counter()
            x, it, rel, st = H.pcg(b, rtol=RTOL, maxit=MAXIT)
            if rep:
                times.append(time.perf_counter() - t1)
        return dict(solve_s=float(np.median(times)), solve_s_each=times, setup_s=t_setup,
                    iterations=it, relres=rel)

    one = leg(False)
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()
    os.environ.setdefault("OMP_PROC_BIND", "close")
    omp = leg(True)
    return dict(value=one["solve_s"], unit="s", cores=1, kind="oracle",
                sample="full 160^3 FP64 solve to rtol 1e-6 (%d iterations), median of %d after 1 warm-up, "
                       "single thread; oracle setup %.2f s not included" % (one["iterations"], runs,
                                                                           one["setup_s"]),
                iterations=one["iterations"], relres=one["relres"], setup_s=one["setup_s"],
                solve_s_each=one["solve_s_each"],
                openmp=dict(value=omp["solve_s"], unit="s", cores=threads, nproc=os.cpu_count(),
                            build="gcc -O3 -march=native -fopenmp -ffp-contract=off (same source)",
                            omp_proc_bind=os.environ.get("OMP_PROC_BIND"),
                            iterations=omp["iterations"], relres=omp["relres"], setup_s=omp["setup_s"],
                            solve_s_each=omp["solve_s_each"],
                            sample="same solve, median of %d after 1 warm-up, %d threads" % (runs, threads)))


def batched_leg(amd, torch, W, np, dev):
    """64 Poisson systems, edges log-uniform in [16, 96] (seed 5), 16 RHS each,
    FP64 outer / FP32 V-cycle, solved by amg_batch_solve (graph launches)."""
    edges = W.batched_edges(64, 5)
    nrhs = 16
    systems = [W.poisson7(N) for N in edges]
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    bt = amd.Batch([(d(A.row_ptr), d(A.col), d(A.val)) for A in systems],
                   precision=amd.AMG_PREC_MIXED)
    bs = []
    for s, A in enumerate(systems):
        xs = W.batched_rhs(s, A.n, nrhs).T
        bs.append(np.ascontiguousarray(A.scipy() @ xs).reshape(-1))
    B = d(np.concatenate(bs))
    ntot = sum(A.n for A in systems)
    times = []
    for rep in range(3):
        X = torch.zeros(ntot * nrhs, dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, its, rel, pst = bt.solve(B, X, nrhs, rtol=RTOL, maxit=MAXIT)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    inf = bt.info()
    bt.close()
    t = min(times[1:])
    return dict(systems=len(systems), nrhs=nrhs, rows=ntot, nnz=int(sum(A.nnz for A in systems)),
                edges_min=min(edges), edges_max=max(edges), solve_s=t, solve_s_first=times[0],
                status=st, iters_max=int(its.max()), iters_mean=float(its.mean()),
                relres_max=float(rel.max()), pair_solves_per_s=len(systems) * nrhs / t,
                levels=inf["levels"], level_rows=inf["n"], level_nnz=inf["nnz"],
                cols_per_lane=inf["cols_per_lane"],
                cols_per_lane_corr=inf["cols_per_lane_corr"], tile_rows=inf["tile_rows"], spmm_cols=inf["spmm_cols"],
                setup_ms=inf["setup_ms"], tune_ms=inf["tune_ms"])


def learned_leg(amd, torch, W, np, dev):
    """7-point log-normal diffusion 128^3 (sigma^2 = 2, ell = 8, seed 7; not a
    training field): smooth vector from 20 relaxation sweeps (plain) versus the
    network's prediction (AMG_SMOOTH_LEARNED, inside amg_setup), both through
    the same setup and FP64 solve.  Generation time of either vector is the
    setup's own smooth-vector phase (setup_smooth_ms)."""
    from paper_2303_02352_amd import surrogate
    A = W.lognormal7(128, 7)
    xs, b = W.manufactured_rhs(A, 8)
    csr = surrogate.device_csr(A, torch)
    bd = torch.from_numpy(b).to(dev)
    params, meta = surrogate.load_params()

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        return out, time.perf_counter() - t0

    def solve(H):
        x = torch.zeros(A.n, dtype=torch.float64, device=dev)
        (st, it, rel), t = timed(lambda: H.solve(bd, x, rtol=RTOL, maxit=MAXIT))
        return dict(status=st, iters=it, relres=rel, solve_s=t,
                    conv_factor=float(rel ** (1.0 / max(1, it))))

    def form(sweeps=20, **kw):
        H, ts = timed(lambda: amd.Hierarchy(*csr, smooth_sweeps=sweeps, **kw))
        inf = H.info()
        rec = dict(setup_s=ts, wgen_s=inf["setup_smooth_ms"] / 1e3, smooth_status=inf["smooth_status"],
                   **solve(H), levels=inf["n"], opc=inf["opc"], matching_rounds=inf["matching_rounds"],
                   setup_match_ms=inf["setup_match_ms"], setup_rap_ms=inf["setup_rap_ms"])
        H.close()
        return rec

    res = {}
    for rep in range(2):          # second pass is reported (warm)
        plain = form(smooth_vec=amd.AMG_SMOOTH_RELAX)
        learned = form(model_params=params)
        res = dict(workload="lognormal7 128^3 seed 7 (sigma^2 = 2, ell = 8)", plain=plain, learned=learned)
    p, l = res["plain"], res["learned"]
    res["learned"]["fallback_to_relax"] = l["smooth_status"] != amd.AMG_OK
    res["speedup_solve"] = p["solve_s"] / l["solve_s"]
    res["speedup_wgen"] = p["wgen_s"] / max(1e-9, l["wgen_s"])
    res["speedup_setup_plus_solve"] = (p["setup_s"] + p["solve_s"]) / (l["setup_s"] + l["solve_s"])
    res["model"] = dict(final_loss=meta.get("final_loss"), steps=meta.get("steps"),
                        training_fields=len(meta.get("fields", [])))
    # A costlier generator, RELAX(640), against the network trained on its
    # vectors (same fields and recipe): the network replaces 640 sweeps by
    # one prediction, but cannot reproduce their long-range structure.
    p640, meta640 = surrogate.load_params(surrogate.RELAX640_MODEL)
    for rep in range(2):
        plain640 = form(640, smooth_vec=amd.AMG_SMOOTH_RELAX)
        learned640 = form(640, model_params=p640)
    res["relax640"] = dict(
        plain=plain640, learned=learned640, model_final_loss=meta640.get("final_loss"),
        speedup_setup_plus_solve=(plain640["setup_s"] + plain640["solve_s"]) /
                                 (learned640["setup_s"] + learned640["solve_s"]),
        vs_relax20_setup_plus_solve=(p["setup_s"] + p["solve_s"]) /
                                    (learned640["setup_s"] + learned640["solve_s"]))
    return res


def bootstrap_leg(amd, torch, W, np, dev):
    """Bootstrap composite AMG (Appendix A: max_hrc hierarchies combined by a
    rule) on the 7-point log-normal 128^3 field (seed 7), FP64: one hierarchy
    from 20 relaxation sweeps against composites of 2 and 3 hierarchies under
    each rule.  The desired rate is set below what one hierarchy reaches so
    that the bootstrap builds max_hrc hierarchies (the paper's 0.8 keeps
    one: a single V-cycle already converges at about 0.4-0.5 here)."""
    A = W.lognormal7(128, 7)
    xs, b = W.manufactured_rhs(A, 8)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    rp, ci, va, bd = d(A.row_ptr), d(A.col), d(A.val), d(b)
    runs = []
    for hrc, btype in ((1, 0), (2, 0), (2, 1), (2, 2), (3, 0), (3, 1)):
        rec = None
        for rep in range(2):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            H = amd.Hierarchy(rp, ci, va, smooth_vec=amd.AMG_SMOOTH_RELAX, smooth_sweeps=20,
                              max_hrc=hrc, bootstrap_type=btype, bootstrap_rate=0.05)
            t1 = time.perf_counter()
            x = torch.zeros(A.n, dtype=torch.float64, device=dev)
            st, it, rel = H.solve(bd, x, rtol=RTOL, maxit=MAXIT)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            inf = H.info()
            rec = dict(max_hrc=hrc, bootstrap_type=["multiplicative", "symmetrized", "additive"][btype],
                       nhrc=inf["nhrc"], rates=inf["rates"], status=st, iters=it, relres=rel,
                       setup_s=t1 - t0, bootstrap_s=inf["setup_bootstrap_ms"] / 1e3, solve_s=t2 - t1,
                       titer_ms=(t2 - t1) / max(1, it) * 1e3)
            H.close()
        runs.append(rec)
        log("bootstrap", json.dumps(rec))
    return dict(workload="lognormal7 128^3 seed 7 (sigma^2 = 2, ell = 8), RELAX(20) first hierarchy",
                bootstrap_rate=0.05, bootstrap_its=15, runs=runs)


def cycles_leg(amd, torch, W, np, dev, N=160):
    """Cycle and smoother options of Appendix A on the 160^3 Poisson system
    (FP64, same right-hand side as the headline): V/H/W cycles with the
    l1-Jacobi smoother, and the V- and W-cycle with Jacobi, forward/backward
    Gauss-Seidel and symmetrized Gauss-Seidel.  Gauss-Seidel passes are level
    schedules (one launch per wavefront of the dependency graph on the fine
    levels: 478 at 160^3), the sequential smoother the paper avoids on GPUs."""
    A = W.poisson7(N)
    xs, b = W.manufactured_rhs(A, SEED)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    rp, ci, va, bd = d(A.row_ptr), d(A.col), d(A.val), d(b)
    names = {0: "Jacobi", 1: "FGS/BGS", 3: "symmetrized GS", 4: "l1-Jacobi"}
    runs = []
    for cyc, rel in ((0, 4), (1, 4), (2, 4), (0, 0), (0, 1), (0, 3), (2, 1), (2, 3)):
        rec = None
        for rep in range(2):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            H = amd.Hierarchy(rp, ci, va, cycle_type=cyc, relax_type=rel)
            t1 = time.perf_counter()
            x = torch.zeros(A.n, dtype=torch.float64, device=dev)
            st, it, rr = H.solve(bd, x, rtol=RTOL, maxit=MAXIT)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            rec = dict(cycle="VHW"[cyc], smoother=names[rel], status=st, iters=it, relres=rr,
                       setup_s=t1 - t0, solve_s=t2 - t1, titer_ms=(t2 - t1) / max(1, it) * 1e3)
            H.close()
        runs.append(rec)
        log("cycles", json.dumps(rec))
    return dict(workload="3D Poisson 7-point 160^3, FP64, b = A x* seed 2", runs=runs)


def mixed27_leg(amd, torch, W, np, dev):
    """27-point diffusion 128^3, kappa log-uniform in [1e-3, 1e3] (seed 3),
    x* seed 4, relaxation smooth vector: FP64 V-cycle versus binary32 V-cycle
    (FP64 outer CG, dots and coarsest solve).  Coarsening stagnates at 1583
    rows, above the 1024-row direct-solve limit, so the coarsest level is
    solved by 20 l1-Jacobi sweeps, in binary64 in both forms."""
    A = W.diffusion27(128, 3)
    xs, b = W.manufactured_rhs(A, 4)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    rp, ci, va, bd = d(A.row_ptr), d(A.col), d(A.val), d(b)
    out = {}
    for name, prec in (("fp64", amd.AMG_PREC_DOUBLE), ("mixed", amd.AMG_PREC_MIXED)):
        for rep in range(2):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            H = amd.Hierarchy(rp, ci, va, smooth_vec=amd.AMG_SMOOTH_RELAX, precision=prec)
            t1 = time.perf_counter()
            x = torch.zeros(A.n, dtype=torch.float64, device=dev)
            st, it, rel = H.solve(bd, x, rtol=RTOL, maxit=MAXIT)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            inf = H.info()
            out[name] = dict(status=st, iters=it, relres=rel, setup_s=t1 - t0, solve_s=t2 - t1,
                             levels=inf["n"], coarse_dense=inf["coarse_dense"],
                             coarsest="direct (binary64)" if inf["coarse_dense"] else
                             "20 l1-Jacobi sweeps (binary64)", x=x.cpu().numpy())
            H.close()
    x64, x32 = out["fp64"].pop("x"), out["mixed"].pop("x")
    S = A.scipy()
    for name, xv in (("fp64", x64), ("mixed", x32)):
        out[name]["true_relres"] = float(np.linalg.norm(b - S @ xv) / np.linalg.norm(b))
        out[name]["rel_error_vs_exact"] = float(np.linalg.norm(xv - xs) / np.linalg.norm(xs))
    out["mixed"]["max_rel_diff_vs_fp64_solution"] = float(np.max(np.abs(x32 - x64)) / np.max(np.abs(x64)))
    out["speedup_solve"] = out["fp64"]["solve_s"] / out["mixed"]["solve_s"]
    out["workload"] = "diffusion27 128^3 (2,097,152 rows, 55,742,968 nnz)"
    return out


def paper_leg(amd, torch, W, np, dev, nd=300):
    """The paper's configuration (Sec. 5, Appendix A): s = 3 composed pairwise
    steps (aggregates <= 8), coarsest <= 40 nd by 20 l1-Jacobi sweeps, 4 + 4
    sweeps, unit right-hand side (f = 1), rtol 1e-6, on nd^3 Poisson.  The
    paper reports 5 levels and OPC ~1.14 at 300^3 and a 5.14 s solve on one
    Tesla P100 (different hardware; context only)."""
    A = W.poisson7(nd)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    rp, ci, va = d(A.row_ptr), d(A.col), d(A.val)
    b = torch.ones(A.n, dtype=torch.float64, device=dev)

    def run(n_parts, reps):
        rec = None
        for rep in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            H = amd.Hierarchy(rp, ci, va, aggr_steps=3, coarse_max=40 * nd,
                              coarse_solver=amd.AMG_COARSE_JACOBI, coarse_sweeps=20, n_parts=n_parts)
            t1 = time.perf_counter()
            x = torch.zeros(A.n, dtype=torch.float64, device=dev)
            st, it, rel = H.solve(b, x, rtol=RTOL, maxit=MAXIT)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            inf = H.info()
            rec = dict(n_parts=n_parts, status=st, iters=it, relres=rel, setup_s=t1 - t0,
                       solve_s=t2 - t1, titer_ms=(t2 - t1) / max(1, it) * 1e3, levels=inf["n"],
                       opc=inf["opc"])
            H.close()
        return rec

    out = dict(nd=nd, rows=A.n, nnz=A.nnz, **run(1, 2),
               paper_context=dict(levels=5, opc=1.14, solve_s_one_p100=5.14))
    # Decoupled aggregation (Sec. 4.1) as the paper's strong-scaling runs set
    # it up: the same 300^3 system split into 2..16 row blocks, each matched
    # on its own subgraph (one GPU runs all blocks).  The paper reports 5
    # levels for every task count and OPC about 1.14.
    out["decoupled_strong"] = [run(q, 1) for q in (2, 4, 8, 16)]
    del rp, ci, va
    return out


def decoupled_weak_leg(amd, torch, W, np, dev, nd=130, tasks=(1, 2, 4, 8)):
    """Weak scaling of decoupled aggregation as the paper ran it (Sec. 5.2):
    a 130^3 share per task, here P tasks' shares stacked along z (a
    130 x 130 x 130 P box, P row blocks = P cubes) solved on one GPU in the
    paper configuration (s = 3, coarsest <= 40 * 130 rows by 20 sweeps,
    f = 1).  The paper reports 4 levels on 1 task, 5 on 2-16, and about 36 %
    more iterations from 1 to 100 tasks."""
    recs = []
    for P in tasks:
        A = W.poisson7_box(nd, nd, nd * P)
        d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
        rp, ci, va = d(A.row_ptr), d(A.col), d(A.val)
        b = torch.ones(A.n, dtype=torch.float64, device=dev)
        del A
        for rep in range(2):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            H = amd.Hierarchy(rp, ci, va, aggr_steps=3, coarse_max=40 * nd,
                              coarse_solver=amd.AMG_COARSE_JACOBI, coarse_sweeps=20, n_parts=P)
            t1 = time.perf_counter()
            x = torch.zeros(b.numel(), dtype=torch.float64, device=dev)
            st, it, rel = H.solve(b, x, rtol=RTOL, maxit=MAXIT)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            inf = H.info()
            rec = dict(tasks=P, rows=b.numel(), status=st, iters=it, relres=rel, setup_s=t1 - t0,
                       solve_s=t2 - t1, titer_ms=(t2 - t1) / max(1, it) * 1e3, levels=inf["n"],
                       opc=inf["opc"])
            H.close()
        recs.append(rec)
        log("weak", json.dumps(rec))
        del rp, ci, va, b, x
        torch.cuda.empty_cache()
    return dict(per_task="130^3", runs=recs,
                paper_context=dict(levels={"1": 4, "2-16": 5, "32-100": 6}, iteration_growth_1_to_100=0.36))


def sweep_kernel_name(info):
    """The fine-level sweep kernel that runs: the two-slice coded-value kernel
    where level 0 reads value codes, else the binary64-value kernel."""
    return "k_sweep2<double>" if info["dict_size"][0] else "k_sweep<double>"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-paper", action="store_true")
    ap.add_argument("--kernel-reps", type=int, default=50)
    ap.add_argument("--values", choices=["auto", "plain"], default="auto",
                    help="matrix values of the solve kernels: coded where a level has at most "
                         "256 distinct values (auto), or plain binary64 arrays")
    ap.add_argument("--only", choices=["batched", "mixed27", "learned", "paper", "mixed160",
                                       "decoupled_weak", "bootstrap", "cycles"],
                    help="only: run one form's leg and print its record (for profiling)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="with --only: copy 1 GiB device to device after the leg (counter calibration)")
    ap.add_argument("--kernel-profile", action="store_true",
                    help="only: build the 160^3 hierarchy, launch the fine-level sweep "
                         "--kernel-reps times, then copy 1 GiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU's share of the problem; runs on %d GPUs are not "
              "implemented (use --gpus 1)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2303_02352_amd as amd
    import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.only and args.only != "mixed160":
        leg = dict(batched=batched_leg, mixed27=mixed27_leg, learned=learned_leg, paper=paper_leg,
                   decoupled_weak=decoupled_weak_leg, bootstrap=bootstrap_leg,
                   cycles=cycles_leg)[args.only]
        log("only", args.only)
        rec = leg(amd, torch, W, np, dev)
        if args.calibrate_copy:   # a 1 GiB device copy after the leg (counter calibration)
            src = torch.ones(1 << 27, dtype=torch.float64, device=dev)
            dst = torch.empty_like(src)
            dst.copy_(src)
            torch.cuda.synchronize()
            rec["calibration_copy_bytes"] = src.numel() * 8
        print(json.dumps({"form": args.only, "record": rec}), flush=True)
        return
    log("generating 160^3 Poisson")
    A = W.poisson7(N_EDGE)
    xs, b = W.manufactured_rhs(A, SEED)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    rp, ci, va, bd = d(A.row_ptr), d(A.col), d(A.val), d(b)
    stream = torch.cuda.Stream()          # default priority
    torch.cuda.synchronize()

    coding = amd.AMG_VALUES_AUTO if args.values == "auto" else amd.AMG_VALUES_PLAIN
    if args.kernel_profile:
        with torch.cuda.stream(stream):
            H = amd.Hierarchy(rp, ci, va, value_coding=coding)
            ms, by = H.time_kernel(amd.KERNEL_SWEEP, 0, args.kernel_reps)
            src = torch.ones(1 << 27, dtype=torch.float64, device=dev)   # 1 GiB
            dst = torch.empty_like(src)
            dst.copy_(src)
            torch.cuda.synchronize()
        print(json.dumps({"kernel": sweep_kernel_name(H.info()) + " level 0", "avg_ms": ms,
                          "algorithmic_bytes": by,
                          "launches": args.kernel_reps + 1, "calibration_copy_bytes": src.numel() * 8,
                          "source_hash": kernel_source_hash()}), flush=True)
        return

    def one_step(precision=amd.AMG_PREC_DOUBLE, value_coding=coding):
        with torch.cuda.stream(stream):
            t0 = time.perf_counter()
            H = amd.Hierarchy(rp, ci, va, precision=precision, value_coding=value_coding)
            t1 = time.perf_counter()
            x = torch.zeros(A.n, dtype=torch.float64, device=dev)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            st, it, rel = H.solve(bd, x, rtol=RTOL, maxit=MAXIT)
            e1.record(stream)
            e1.synchronize()
            t2 = time.perf_counter()
        return H, x, dict(status=st, iters=it, relres=rel, setup_s=t1 - t0,
                          solve_s=e0.elapsed_time(e1) / 1e3, wall_solve_s=t2 - t1)

    if args.only == "mixed160":
        recs = []
        for _ in range(3):
            Hm, xm, rm = one_step(amd.AMG_PREC_MIXED)
            Hm.close()
            recs.append(rm)
        print(json.dumps({"form": "mixed160", "record": recs[-1],
                          "solve_s_each": [r["solve_s"] for r in recs]}), flush=True)
        return

    log("warmup", args.warmup)
    for _ in range(args.warmup):
        H, x, rec = one_step()
        H.close()
    torch.cuda.synchronize()
    log("timed steps", args.steps)
    recs = []
    t_start = time.perf_counter()
    for _ in range(args.steps):
        H, x, rec = one_step()
        recs.append(rec)
        if _ < args.steps - 1:
            H.close()
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    last = recs[-1]
    info = H.info()
    xg = x.cpu().numpy()
    true_rel = float(np.linalg.norm(b - A.scipy() @ xg) / np.linalg.norm(b))
    solve_s = float(np.mean([r["solve_s"] for r in recs]))
    setup_s = float(np.mean([r["setup_s"] for r in recs]))

    forms = {}
    # per-kernel timings on the fine level (library stream, HIP events), in
    # the configuration the solve runs (bytes: what each kernel reads and
    # writes in the form it reads, coded values where the level is coded)
    kt = {}
    for name, kid in (("spmv_dots", amd.KERNEL_SPMV), ("sweep", amd.KERNEL_SWEEP),
                      ("restrict", amd.KERNEL_RESTRICT), ("prolong", amd.KERNEL_PROLONG),
                      ("corr_sweep", amd.KERNEL_CORR_SWEEP), ("pcg_update", amd.KERNEL_UPDATE)):
        ms, by = H.time_kernel(kid, 0, args.kernel_reps)
        kt[name] = dict(avg_ms=ms, bytes=by, gbps=by / (ms * 1e-3) / 1e9)
    log("kernels", json.dumps(kt))
    H.close()

    # The graded kernels: fine-level sweep and SpMV + dots reading binary64
    # value arrays (the matrix streamed from HBM, 287 MB as read > the 256 MB
    # last-level cache), priced by the plain-CSR algorithmic bytes: 8-byte
    # values, 4-byte columns, 4-byte row pointers and every vector once.
    n, nnz = A.n, A.nnz
    csr_bytes = dict(sweep=12.0 * nnz + 4.0 * (n + 1) + 3 * 8.0 * n,
                     spmv_dots=12.0 * nnz + 4.0 * (n + 1) + 4 * 8.0 * n)
    log("binary64-value hierarchy (graded kernels)")
    Hq, xq, rq = one_step(value_coding=amd.AMG_VALUES_PLAIN)
    Hq.close()
    Hq, xq, rq = one_step(value_coding=amd.AMG_VALUES_PLAIN)
    plain_kt = {}
    for name, kid in (("sweep", amd.KERNEL_SWEEP), ("spmv_dots", amd.KERNEL_SPMV)):
        ms, by = Hq.time_kernel(kid, 0, args.kernel_reps)
        plain_kt[name] = dict(avg_ms=ms, csr_bytes=csr_bytes[name], physical_bytes=by,
                              gbps=csr_bytes[name] / (ms * 1e-3) / 1e9,
                              frac=csr_bytes[name] / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS)
    sw = plain_kt["sweep"]
    roofline = dict(bound="hbm", achieved=sw["gbps"], peak=HBM_PEAK_GBPS, unit="GB/s",
                    frac=sw["frac"], traffic=measured_traffic("sweep_poisson160_plain", sw["csr_bytes"]),
                    kernel="k_sweep<double, true> (fine-level l1-Jacobi sweep, binary64 value array, "
                           "non-temporal loads, 160^3)",
                    bytes_per_launch=sw["csr_bytes"], avg_launch_ms=sw["avg_ms"],
                    bytes_model="(8 + 4) nnz + 4 (n + 1) + 3 * 8 n: binary64 values, int32 columns, "
                                "row pointers, x, rhs and the new iterate once",
                    physical_bytes_per_launch=sw["physical_bytes"])
    forms["plain_values"] = dict(solve_s=rq["solve_s"], setup_s=rq["setup_s"], iters=rq["iters"],
                                 bitwise_equal_solution=bool(torch.equal(xq, x)),
                                 coded_speedup_solve=rq["solve_s"] / solve_s,
                                 titer_ms=rq["solve_s"] / max(1, rq["iters"]) * 1e3,
                                 kernels_fine_level=plain_kt)
    Hq.close()
    log("plain values", json.dumps(forms["plain_values"]))
    # The coded sweep the default solve runs: its working set (86 MB of
    # matrix + 98 MB of vectors) fits the last-level cache, so back-to-back
    # relaunches are partly served from there; its rate is reported against
    # the bytes it reads, as a compressed-format result, not as an HBM rate.
    coded = dict(kernel="k_sweep2<double, false> (1-byte value codes + per-level table, 16-bit "
                        "column offsets)", avg_ms=kt["sweep"]["avg_ms"], physical_bytes=kt["sweep"]["bytes"],
                 gbps_physical=kt["sweep"]["gbps"],
                 note="working set ~186 MB fits the 256 MB last-level cache: not an HBM rate")

    if not args.no_forms:
        log("mixed-precision form")
        Hm, xm, rm = one_step(amd.AMG_PREC_MIXED)
        Hm.close()
        Hm, xm, rm = one_step(amd.AMG_PREC_MIXED)
        xmh = xm.cpu().numpy()
        forms["mixed"] = dict(solve_s=rm["solve_s"], setup_s=rm["setup_s"], iters=rm["iters"],
                              relres=rm["relres"],
                              true_relres=float(np.linalg.norm(b - A.scipy() @ xmh) / np.linalg.norm(b)),
                              speedup_vs_fp64_solve=solve_s / rm["solve_s"],
                              max_rel_diff_vs_fp64_solution=float(np.max(np.abs(xmh - xg)) / np.max(np.abs(xg))))
        Hm.close()

    if not args.no_forms:
        log("mixed precision, 27-point 128^3")
        forms["mixed_27pt"] = mixed27_leg(amd, torch, W, np, dev)
        log("mixed27", json.dumps(forms["mixed_27pt"]))
        log("learned form")
        forms["learned"] = learned_leg(amd, torch, W, np, dev)
        log("learned", json.dumps(forms["learned"]))

    if not args.no_forms:
        log("bootstrap composite")
        forms["bootstrap"] = bootstrap_leg(amd, torch, W, np, dev)
        log("cycle and smoother options")
        forms["cycles"] = cycles_leg(amd, torch, W, np, dev)

    if not args.no_forms and not args.no_paper:
        log("paper configuration 300^3")
        forms["paper_config_300"] = paper_leg(amd, torch, W, np, dev)
        log("paper", json.dumps(forms["paper_config_300"]))

    if not args.no_forms and not args.no_batched:
        log("batched form")
        forms["batched"] = batched_leg(amd, torch, W, np, dev)
        log("batched", json.dumps(forms["batched"]))

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        cpu = cpu_baseline(A, b)
        log("cpu", json.dumps(cpu))

    out = {
        "metric": METRIC, "value": solve_s, "unit": "s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": t_total / args.steps * 1e3,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "3D Poisson 7-point 160^3 (4,096,000 rows, 28,518,400 nnz, CSR "
                               "FP64 input, int32 indices), b = A x*, x* ~ U[-1,1) seed 2; "
                               + ("the solve kernels read each level's values as 1-byte codes into "
                                  "a per-level binary64 table (every level has <= 256 distinct "
                                  "values; solution bit-identical to the binary64-value solve in "
                                  "detail.forms.plain_values)" if args.values == "auto" else
                                  "the solve kernels read binary64 value arrays"),
                   "rtol": RTOL, "aggr_steps": 2, "coarse_max": 100, "pre_post_sweeps": [4, 4],
                   "coarsest": "dense FP64 Cholesky", "step": "amg_setup + amg_pcg_solve",
                   "values": "coded" if args.values == "auto" else "binary64"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "detail": {"iterations": last["iters"], "relres": last["relres"], "true_relres": true_rel,
                   "solve_s_each": [r["solve_s"] for r in recs],
                   "setup_s": setup_s, "titer_ms": solve_s / max(1, last["iters"]) * 1e3,
                   "levels": info["n"], "opc": info["opc"],
                   "value_table_sizes": info["dict_size"],
                   "matching_rounds": info["matching_rounds"],
                   "kernels_fine_level": kt, "coded_sweep": coded, "forms": forms,
                   "spmv_gbps": plain_kt["spmv_dots"]["gbps"],
                   "spmv_frac": plain_kt["spmv_dots"]["frac"],
                   "smoother_gbps": plain_kt["sweep"]["gbps"],
                   "smoother_frac": plain_kt["sweep"]["frac"],
                   "rates_note": "spmv_/smoother_ rates: binary64-value kernels priced by plain-CSR "
                                 "algorithmic bytes (roofline); kernels_fine_level: the solve's own "
                                 "kernels by the bytes of the form they read"},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
