"""GPU parity of the cycle and smoother options (Appendix A: cycle_type
V/H/W; relax_type / coarse_relax Jacobi, FGS/BGS, symmetrized GS,
l1-Jacobi), binary64.

Bars: the preconditioner output bit-identical to the oracle's (<= 1e-12
relative stated), PCG iterations +-1 at rtol.  Gauss-Seidel passes run as
level schedules: levels of at most 65536 rows in one workgroup, larger ones
one launch per schedule level; both sizes are covered.
"""
import numpy as np
import pytest

import oracle
import workloads as W

from gpu_helpers import dev, gpu_hierarchy, host, oracle_params, require_gpu, say, torch

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def _check(A, params, seed=3):
    Ho = oracle.Hierarchy(A, oracle_params(**params))
    Hg = gpu_hierarchy(A, **params)
    r = W.uniform_pm1(seed, A.n)
    z = torch.empty(A.n, dtype=torch.float64, device="cuda")
    Hg.vcycle(dev(r), z)
    zo = Ho.vcycle(r)
    err = np.max(np.abs(host(z) - zo)) / np.max(np.abs(zo))
    xs, b = W.manufactured_rhs(A, seed + 1)
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    st, it, rel = Hg.solve(dev(b), x, rtol=1e-6)
    xo, ito, relo, sto = Ho.pcg(b, rtol=1e-6)
    say("  levels", Hg.info()["n"], "cycle err %.2e" % err, "iterations gpu %d oracle %d" % (it, ito))
    assert err <= 1e-12, err
    assert st == 0 and sto == oracle.OK and abs(it - ito) <= 1 and rel <= 1e-6


@pytest.mark.parametrize("cycle", [0, 1, 2])
@pytest.mark.parametrize("relax", [0, 1, 3, 4])
def test_cycle_and_smoother(cycle, relax):
    A = W.lognormal7(20, 7, ell=4.0)
    params = dict(cycle_type=cycle, relax_type=relax, smooth_vec=1, pre_sweeps=2, post_sweeps=2)
    say("cycle", cycle, "relax", relax, "n=%d" % A.n)
    _check(A, params)


@pytest.mark.parametrize("crelax", [0, 1, 3, 4])
def test_coarsest_sweeps(crelax):
    A = W.poisson7(24)
    params = dict(cycle_type=2, relax_type=1, coarse_solver=1, coarse_relax=crelax, coarse_sweeps=8,
                  coarse_max=600)
    say("coarse relax", crelax)
    _check(A, params)


@pytest.mark.parametrize("cycle", [1, 2])
@pytest.mark.parametrize("coarse_solver", [0, 1])
def test_l1_cycles_in_the_coarse_tail(cycle, coarse_solver):
    """H/W-cycles with l1-Jacobi everywhere run their levels below 1024 rows
    in one workgroup (the general cycle's tail), with a direct or an
    l1-Jacobi coarsest solve."""
    A = W.poisson7(26)
    params = dict(cycle_type=cycle, relax_type=4, coarse_solver=coarse_solver, coarse_relax=4,
                  coarse_sweeps=6, coarse_max=300, pre_sweeps=3, post_sweeps=2)
    say("tail cycle", cycle, "coarse solver", coarse_solver)
    _check(A, params)


@pytest.mark.parametrize("relax", [1, 3])
def test_gauss_seidel_multi_launch_levels(relax):
    """48^3 = 110592 rows on the fine level: one launch per schedule level."""
    A = W.lognormal7(48, 5, ell=6.0)
    params = dict(cycle_type=1, relax_type=relax, smooth_vec=1, pre_sweeps=1, post_sweeps=1)
    say("GS multi-launch, relax", relax)
    _check(A, params)


def test_binary32_cycle_refuses_other_options():
    import paper_2303_02352_amd as amd
    A = W.poisson7(8)
    with pytest.raises(amd.AMGError) as e:
        gpu_hierarchy(A, cycle_type=2, precision=1)
    assert e.value.code == amd.AMG_ERR_UNSUPPORTED
