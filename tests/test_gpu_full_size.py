"""GPU parity at the full workload sizes, in the launch configuration bench.py
times (the same library calls on the same resident inputs).

The oracle cannot rerun these inside a test, so
``tests/golden/oracle_full_size.json`` -- written by
``tests/golden/make_oracle_golden.py`` from the oracle alone -- holds its
results: hierarchy sizes, PCG iterations and residuals, SHA-256 digests of
every level's arrays and of one whole V-cycle output (binary64 and the binary32
cycle) on a seeded residual, and sampled entries of those outputs.

Bars: every level's CSR arrays, l1 diagonal, smooth vector, aggregate map and
P values bit-identical to the oracle's (digests); the whole V-cycle output
bit-identical (digest; the sampled entries within 1e-12 relative, binary64, or
1e-6, binary32 cycle, are reported first as the diagnostic); PCG iterations
within +-1 of the oracle's, recurrence and true relative residual <= 1e-6;
fine-level SpMV bit-exact against the oracle's SpMV over the whole vector.

The batched workload (64 systems, edges 17-94, 16 right-hand sides, binary32
V-cycle inside binary64 PCG) has its own record,
``tests/golden/oracle_batched64x16.json``, from the same script: every pair
must reach a true relative residual <= 1e-6, and sampled pairs must take the
oracle's iterations +-1 and match its binary32 V-cycle on sampled rows within
1e-6.
"""
import json
import os

import numpy as np
import pytest

import oracle
import workloads as W

from gpu_helpers import (assert_level_digests, bits, dev, digest, gpu_hierarchy, host, require_gpu,
                         say, torch)

pytestmark = pytest.mark.gpu

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "oracle_full_size.json")))
BATCH = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "oracle_batched64x16.json")))
MAKE = {"poisson7_160": lambda: W.poisson7(160), "diffusion27_128": lambda: W.diffusion27(128, 3)}


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def _check_samples(z, rec, tol):
    rows = np.asarray(rec["rows"], dtype=np.int64)
    ref = np.array([float.fromhex(h) for h in rec["z"]])
    got = z[rows]
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    say("  sampled V-cycle rel err %.2e, bitwise %s" % (err, np.array_equal(bits(got), bits(ref))))
    assert err <= tol
    if "sha256" in rec:
        same = digest(z, np.float64) == rec["sha256"]
        say("  whole V-cycle output bit-identical: %s" % same)
        assert same


@pytest.mark.parametrize("name", list(MAKE))
def test_full_size_against_oracle(name):
    import paper_2303_02352_amd as amd
    g = GOLDEN[name]
    A = MAKE[name]()
    say("full size", name, "n=%d nnz=%d" % (A.n, A.nnz))
    params = g["params"]
    for prec in (amd.AMG_PREC_DOUBLE, amd.AMG_PREC_MIXED):
        Hg = gpu_hierarchy(A, precision=prec, **params)
        inf = Hg.info()
        assert [[n, z] for n, z in zip(inf["n"], inf["nnz"])] == g["levels"]
        if prec == amd.AMG_PREC_DOUBLE:
            assert_level_digests(Hg, g["level_sha256"])
        r = W.uniform_pm1(g["vcycle"]["r_seed"], A.n)
        z = torch.empty(A.n, dtype=torch.float64, device="cuda")
        Hg.vcycle(dev(r), z)
        if prec == amd.AMG_PREC_DOUBLE:
            _check_samples(host(z), g["vcycle"], 1e-12)
        else:
            _check_samples(host(z), g["vcycle_f32"], 1e-6)
        xs, b = W.manufactured_rhs(A, g["seed"])
        x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
        st, it, rel = Hg.solve(dev(b), x, rtol=1e-6)
        ref_it = g["iterations"] if prec == amd.AMG_PREC_DOUBLE else g["mixed"]["iterations"]
        say("  precision %d: its %d (oracle %d), relres %.3e" % (prec, it, ref_it, rel))
        assert st == 0 and abs(it - ref_it) <= 1 and rel <= 1e-6
        xg = host(x)
        assert np.linalg.norm(b - A.scipy() @ xg) / np.linalg.norm(b) <= 1e-6 * 1.01
        Hg.close()


def test_full_size_plain_values_streamed():
    """160^3 with binary64 value arrays (bench.py --values plain): every level
    is read from plain values and the fine level (287 MB as read) takes the
    non-temporal path; the sampled V-cycle and the iteration count are the
    oracle's, as for the coded default."""
    import paper_2303_02352_amd as amd
    g = GOLDEN["poisson7_160"]
    A = MAKE["poisson7_160"]()
    say("full size plain values, poisson7_160")
    Hg = gpu_hierarchy(A, value_coding=amd.AMG_VALUES_PLAIN, **g["params"])
    assert Hg.info()["dict_size"] == [0] * Hg.info()["levels"]
    r = W.uniform_pm1(g["vcycle"]["r_seed"], A.n)
    z = torch.empty(A.n, dtype=torch.float64, device="cuda")
    Hg.vcycle(dev(r), z)
    _check_samples(host(z), g["vcycle"], 1e-12)
    xs, b = W.manufactured_rhs(A, g["seed"])
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    st, it, rel = Hg.solve(dev(b), x, rtol=1e-6)
    say("  its %d (oracle %d), relres %.3e" % (it, g["iterations"], rel))
    assert st == 0 and abs(it - g["iterations"]) <= 1 and rel <= 1e-6
    Hg.close()


def test_full_size_fine_spmv_bit_exact():
    A = MAKE["poisson7_160"]()
    Hg = gpu_hierarchy(A)
    x = W.uniform_pm1(91, A.n)
    y = torch.empty(A.n, dtype=torch.float64, device="cuda")
    Hg.spmv(0, dev(x), y)
    assert np.array_equal(bits(host(y)), bits(oracle.spmv(A, x)))


def test_full_size_batched_against_oracle():
    import paper_2303_02352_amd as amd
    g = BATCH
    edges = W.batched_edges(g["nsys"], g["edges_seed"])
    assert [int(e) for e in edges] == g["edges"]
    nrhs = g["nrhs"]
    systems = [W.poisson7(N) for N in edges]
    ntot = sum(A.n for A in systems)
    say("batched full size: %d systems, %d rows x %d right-hand sides" % (len(systems), ntot, nrhs))
    bt = amd.Batch([(dev(A.row_ptr), dev(A.col), dev(A.val)) for A in systems],
                   precision=amd.AMG_PREC_MIXED)
    bs = [np.ascontiguousarray(A.scipy() @ W.batched_rhs(s, A.n, nrhs).T) for s, A in enumerate(systems)]
    Bd = dev(np.concatenate([b.reshape(-1) for b in bs]))
    X = torch.zeros(ntot * nrhs, dtype=torch.float64, device="cuda")
    st, its, rel, pst = bt.solve(Bd, X, nrhs, rtol=1e-6, maxit=1000)
    assert st == 0 and np.all(pst == 0) and np.all(rel <= 1e-6)
    Xh = host(X)
    offs = np.cumsum([0] + [A.n * nrhs for A in systems])
    worst = 0.0
    for s, A in enumerate(systems):
        blk = Xh[offs[s]:offs[s + 1]].reshape(A.n, nrhs)
        tr = np.linalg.norm(bs[s] - A.scipy() @ blk, axis=0) / np.linalg.norm(bs[s], axis=0)
        worst = max(worst, float(tr.max()))
    say("  worst true relative residual %.2e, iterations %d-%d" % (worst, its.min(), its.max()))
    assert worst <= 1e-6 * 1.01
    for p in g["pairs"]:
        assert abs(int(its[p["system"], p["column"]]) - p["iterations"]) <= 1, p["system"]
    del bs, Xh, X, Bd
    R = np.concatenate([W.uniform_pm1(g["r_seed"] + s, A.n * nrhs) for s, A in enumerate(systems)])
    Rd = dev(R)
    Z = torch.zeros(ntot * nrhs, dtype=torch.float64, device="cuda")
    bt.vcycle(Rd, Z, nrhs)
    Zh = host(Z)
    for p in g["pairs"]:
        s, c = p["system"], p["column"]
        _check_samples(Zh[offs[s]:offs[s + 1]].reshape(-1, nrhs)[:, c], p, 1e-6)
    bt.close()
