"""GPU parity of decoupled aggregation (Sec. 4.1): n_parts row blocks, each
matched on its own subgraph.

Bars: every level's aggregate map, P values, coarse pattern and values, l1
diagonal and smooth vector bit-identical to the oracle's; V-cycle output
bit-identical (<= 1e-12 relative is the stated bound); PCG iterations +-1 of
the oracle at rtol.  Sizes: small grids with ragged blocks, and the paper's
weak-scaling per-GPU size 130^3 in the paper configuration (s = 3, coarsest
<= 40 nd by 20 sweeps) for 2, 8 and 64 blocks.
"""
import numpy as np
import pytest

import oracle
import workloads as W

from gpu_helpers import (assert_same_hierarchy, bits, dev, gpu_hierarchy, host, oracle_params,
                         require_gpu, say, torch)

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


CASES = {
    "lognormal14_np2": (lambda: W.lognormal7(14, 7, ell=3.0), dict(n_parts=2, smooth_vec=1, smooth_sweeps=10)),
    "lognormal14_np5": (lambda: W.lognormal7(14, 7, ell=3.0), dict(n_parts=5, smooth_vec=1, smooth_sweeps=10)),
    "poisson33_np64": (lambda: W.poisson7(33), dict(n_parts=64)),
    "poisson16_planes_s3": (lambda: W.poisson7(16), dict(n_parts=16, aggr_steps=3, coarse_max=40 * 16,
                                                         coarse_solver=1, coarse_sweeps=20)),
    "diffusion27_12_np3_mixed": (lambda: W.diffusion27(12, 3), dict(n_parts=3, smooth_vec=1, precision=1)),
    "poisson3_np64_one_level": (lambda: W.poisson7(3), dict(n_parts=64, coarse_max=1)),
}


@pytest.mark.parametrize("case", list(CASES))
def test_decoupled_parity(case):
    make, params = CASES[case]
    A = make()
    say("decoupled parity", case, "n=%d" % A.n, params)
    Ho = oracle.Hierarchy(A, oracle_params(**params))
    Hg = gpu_hierarchy(A, **params)
    inf = assert_same_hierarchy(Hg, Ho)
    assert abs(inf["opc"] - Ho.opc()) <= 1e-15 * Ho.opc()
    r = W.uniform_pm1(21, A.n)
    z = torch.empty(A.n, dtype=torch.float64, device="cuda")
    Hg.vcycle(dev(r), z)
    mixed = params.get("precision", 0) == 1
    zo = Ho.vcycle_f32(r) if mixed else Ho.vcycle(r)
    zg = host(z)
    err = np.max(np.abs(zg - zo)) / max(1e-300, np.max(np.abs(zo)))
    say("  levels", inf["n"], "vcycle rel err %.2e" % err)
    assert err <= (1e-6 if mixed else 1e-12), err
    xs, b = W.manufactured_rhs(A, 4)
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    st, it, rel = Hg.solve(dev(b), x, rtol=1e-6)
    xo, ito, relo, sto = Ho.pcg(b, rtol=1e-6, mixed=mixed)
    say("  iterations gpu %d oracle %d" % (it, ito))
    assert st == 0 and sto == oracle.OK and abs(it - ito) <= 1 and rel <= 1e-6


@pytest.mark.parametrize("nparts", [2, 8, 64])
def test_decoupled_paper_config_130(nparts):
    """130^3, s = 3, coarsest <= 40 * 130 rows by 20 l1-Jacobi sweeps, f = 1:
    hierarchy bit-identical to the oracle's, iterations +-1."""
    nd = 130
    A = W.poisson7(nd)
    params = dict(n_parts=nparts, aggr_steps=3, coarse_max=40 * nd, coarse_solver=1, coarse_sweeps=20)
    say("decoupled 130^3 n_parts=%d" % nparts)
    Ho = oracle.Hierarchy(A, oracle_params(**params))
    Hg = gpu_hierarchy(A, **params)
    inf = assert_same_hierarchy(Hg, Ho)
    b = np.ones(A.n)
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    st, it, rel = Hg.solve(dev(b), x, rtol=1e-6)
    xo, ito, relo, sto = Ho.pcg(b, rtol=1e-6)
    say("  levels", inf["n"], "opc %.4f" % inf["opc"], "iterations gpu %d oracle %d" % (it, ito))
    assert st == 0 and abs(it - ito) <= 1 and rel <= 1e-6
