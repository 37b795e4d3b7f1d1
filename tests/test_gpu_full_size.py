"""GPU parity at the full workload sizes, in the launch configuration bench.py
times (the same library calls on the same resident inputs).

The oracle cannot rerun these inside a test, so
``tests/golden/oracle_full_size.json`` -- written by
``tests/golden/make_oracle_golden.py`` from the oracle alone -- holds its
results: hierarchy sizes, PCG iterations and residuals, and sampled entries of
one V-cycle (binary64 and the binary32 cycle) on a seeded residual.

Bars: level sizes and nonzeros equal; PCG iterations within +-1 of the
oracle's, recurrence and true relative residual <= 1e-6; sampled V-cycle
entries within 1e-12 relative (binary64) and 1e-6 (binary32 cycle) of the
oracle's (bit-exact expected); fine-level SpMV bit-exact against the oracle's
SpMV over the whole vector.
"""
import json
import os

import numpy as np
import pytest

import oracle
import workloads as W

from gpu_helpers import bits, dev, gpu_hierarchy, host, require_gpu, say, torch

pytestmark = pytest.mark.gpu

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "oracle_full_size.json")))
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


def test_full_size_fine_spmv_bit_exact():
    A = MAKE["poisson7_160"]()
    Hg = gpu_hierarchy(A)
    x = W.uniform_pm1(91, A.n)
    y = torch.empty(A.n, dtype=torch.float64, device="cuda")
    Hg.spmv(0, dev(x), y)
    assert np.array_equal(bits(host(y)), bits(oracle.spmv(A, x)))
