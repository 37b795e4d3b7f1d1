"""Learned smooth vector: training and use of the network behind amg_mpnn_*.

The network predicts log w, w being the smooth vector whose entries enter the
matching weights of the coarsening (Sec. 3.1 leaves the smooth vector's source
open).  Training targets are the method's own relaxation vectors: 20 l1-Jacobi
sweeps on A w = 0 from ones (AMG_SMOOTH_RELAX), computed by the library.
All arithmetic runs in the library's HIP kernels; this module only moves
arrays and loops over training steps.  A trained parameter set is used by
passing it to amg_setup (``Hierarchy(..., model_params=params)``,
AMG_SMOOTH_LEARNED): the library predicts the vector, checks it and falls
back to relaxation by itself.

Command line (writes the model files used by bench.py):
    python -m paper_2303_02352_amd.surrogate --out paper_2303_02352_amd/models/mpnn_lognormal.json
    python -m paper_2303_02352_amd.surrogate --relax-sweeps 640 \
        --out paper_2303_02352_amd/models/mpnn_lognormal_relax640.json
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np

import paper_2303_02352_amd as amd

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_MODEL = os.path.join(HERE, "models", "mpnn_lognormal.json")
# trained on RELAX(640) targets (--relax-sweeps 640), same fields and steps
RELAX640_MODEL = os.path.join(HERE, "models", "mpnn_lognormal_relax640.json")
RELAX_SWEEPS = 20


def init_params(seed: int = 0) -> np.ndarray:
    """He-style uniform initial weights (fan-in), zero biases."""
    rng = np.random.default_rng(seed)
    W1 = rng.uniform(-1, 1, (16, 32)) * np.sqrt(6.0 / 16)
    W2 = rng.uniform(-1, 1, (64, 32)) * np.sqrt(6.0 / 64)
    wh = rng.uniform(-1, 1, 32) * np.sqrt(3.0 / 32)
    return np.concatenate([W1.ravel(), np.zeros(32), W2.ravel(), np.zeros(32), wh, np.zeros(1)]).astype(np.float32)


def device_csr(A, torch):
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    return d(A.row_ptr), d(A.col), d(A.val)


def relax_target(csr, torch, sweeps=RELAX_SWEEPS):
    """The method's relaxation smooth vector (device float64), via amg_setup on one level."""
    rp, ci, va = csr
    H = amd.Hierarchy(rp, ci, va, smooth_vec=amd.AMG_SMOOTH_RELAX, smooth_sweeps=sweeps, max_levels=1)
    w = H.export_level(0)["w"]
    H.close()
    return torch.from_numpy(w).cuda()


def train(net, data, steps, lr, log_every=50, lr_final=None):
    """Adam over the training graphs, one full graph per step (cycling)."""
    hist = []
    lr_final = lr if lr_final is None else lr_final
    for it in range(steps):
        frac = it / max(1, steps - 1)
        lr_t = lr * (lr_final / lr) ** frac
        rp, ci, va, w = data[it % len(data)]
        loss = net.train_step(rp, ci, va, w, lr_t)
        hist.append(loss)
        if log_every and (it % log_every == 0 or it == steps - 1):
            print("[surrogate] step %d loss %.4e lr %.2e" % (it, loss, lr_t), flush=True)
    return hist


def save(path, params, meta):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as f:
        json.dump(dict(meta=meta, params=[float(x) for x in params]), f)


def load_params(path=DEFAULT_MODEL):
    rec = json.load(open(path))
    return np.asarray(rec["params"], dtype=np.float32), rec["meta"]


def main():
    import torch
    import workloads as W
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_MODEL)
    ap.add_argument("--steps", type=int, default=600)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--lr-final", type=float, default=3e-4)
    ap.add_argument("--small", type=int, default=16, help="training fields at 64^3")
    ap.add_argument("--large", type=int, default=2, help="training fields at 128^3")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--relax-sweeps", type=int, default=RELAX_SWEEPS,
                    help="relaxation sweeps of the training targets")
    args = ap.parse_args()
    t0 = time.time()
    data, seeds = [], []
    for k in range(args.small):
        seeds.append((64, 100 + k))
    for k in range(args.large):
        seeds.append((128, 200 + k))
    for N, sd in seeds:
        A = W.lognormal7(N, sd)
        csr = device_csr(A, torch)
        data.append(csr + (relax_target(csr, torch, args.relax_sweeps),))
        print("[surrogate] field %d^3 seed %d ready" % (N, sd), flush=True)
    t1 = time.time()
    net = amd.SmoothVectorNet(init_params(args.seed))
    hist = train(net, data, args.steps, args.lr, lr_final=args.lr_final)
    torch.cuda.synchronize()
    t2 = time.time()
    meta = dict(fields=seeds, steps=args.steps, lr=args.lr, lr_final=args.lr_final,
                relax_sweeps=args.relax_sweeps, sigma2=2.0, ell=8.0, final_loss=hist[-1],
                first_loss=hist[0], data_s=t1 - t0, train_s=t2 - t1,
                note="targets: %d l1-Jacobi sweeps on A w = 0 from ones; loss: MSE of log w"
                     % args.relax_sweeps)
    save(args.out, net.params(), meta)
    print(json.dumps(meta), flush=True)


if __name__ == "__main__":
    main()
