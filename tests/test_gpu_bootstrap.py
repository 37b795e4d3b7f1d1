"""GPU parity of the bootstrap composite AMG (Appendix A: bootstrap_type,
max_hrc, desired convergence rate).

Bars: the same number of hierarchies as the oracle; every hierarchy of the
composite bit-identical to the oracle's (its smooth vector is the
bootstrap's iterate, so this also checks the rate-estimate iterations bit
for bit); rate estimates within 1e-10 relative (their dot products are tree
reductions on the GPU, left folds in the oracle); composite preconditioner
output <= 1e-12 relative (binary64) or <= 1e-6 (binary32 cycles); PCG
iterations +-1 at rtol.
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
    "lognormal16_mult": (lambda: W.lognormal7(16, 7, ell=4.0), dict(bootstrap_type=0)),
    "lognormal16_symm": (lambda: W.lognormal7(16, 7, ell=4.0), dict(bootstrap_type=1)),
    "lognormal16_add": (lambda: W.lognormal7(16, 7, ell=4.0), dict(bootstrap_type=2)),
    "poisson21_symm_mixed": (lambda: W.poisson7(21), dict(bootstrap_type=1, precision=1)),
    "diffusion27_12_mult_relax": (lambda: W.diffusion27(12, 3), dict(bootstrap_type=0, smooth_vec=1)),
    "lognormal24_mult_np4": (lambda: W.lognormal7(24, 5, ell=4.0), dict(bootstrap_type=0, n_parts=4)),
}


@pytest.mark.parametrize("case", list(CASES))
def test_bootstrap_parity(case):
    make, extra = CASES[case]
    A = make()
    params = dict(max_hrc=3, bootstrap_rate=0.05, bootstrap_its=8, **extra)
    say("bootstrap parity", case, "n=%d" % A.n, params)
    Ho = oracle.Hierarchy(A, oracle_params(**params))
    Hg = gpu_hierarchy(A, **params)
    inf = Hg.info()
    assert inf["nhrc"] == Ho.nhrc == 3, (inf["nhrc"], Ho.nhrc)
    ro = Ho.rates()
    say("  rates gpu", np.round(inf["rates"], 6), "oracle", np.round(ro, 6))
    assert len(inf["rates"]) == len(ro)
    assert np.all(np.abs(np.array(inf["rates"]) - ro) <= 1e-10 * ro)
    for j in range(Ho.nhrc):
        assert_same_hierarchy(Hg.component(j), Ho.component(j))
    mixed = params.get("precision", 0) == 1
    r = W.uniform_pm1(17, A.n)
    z = torch.empty(A.n, dtype=torch.float64, device="cuda")
    Hg.vcycle(dev(r), z)
    zo = Ho.vcycle_f32(r) if mixed else Ho.vcycle(r)
    err = np.max(np.abs(host(z) - zo)) / np.max(np.abs(zo))
    say("  composite cycle rel err %.2e" % err)
    assert err <= (1e-6 if mixed else 1e-12), err
    # a component's own V-cycle through its borrowed handle
    z1 = torch.empty(A.n, dtype=torch.float64, device="cuda")
    Hg.component(1).vcycle(dev(r), z1)
    zo1 = Ho.component(1).vcycle(r, single=True)
    if not mixed:
        assert np.max(np.abs(host(z1) - zo1)) <= 1e-12 * np.max(np.abs(zo1))
    xs, b = W.manufactured_rhs(A, 6)
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    st, it, rel = Hg.solve(dev(b), x, rtol=1e-6)
    xo, ito, relo, sto = Ho.pcg(b, rtol=1e-6, mixed=mixed)
    say("  iterations gpu %d oracle %d" % (it, ito))
    assert st == 0 and sto == oracle.OK and abs(it - ito) <= 1 and rel <= 1e-6
    # the allocation-free solve runs the same composite
    x2 = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    st2, it2, rel2 = Hg.solve_noalloc(dev(b), x2, rtol=1e-6)
    assert (st2, it2, rel2) == (st, it, rel)
    assert np.array_equal(bits(host(x2)), bits(host(x)))


def test_bootstrap_stops_at_the_desired_rate():
    """The paper's desired rate 0.8: one V-cycle on Poisson already converges
    faster, so one hierarchy is kept and one rate estimated, as in the oracle."""
    A = W.poisson7(24)
    params = dict(max_hrc=4, bootstrap_rate=0.8)
    Ho = oracle.Hierarchy(A, oracle_params(**params))
    Hg = gpu_hierarchy(A, **params)
    inf = Hg.info()
    assert inf["nhrc"] == Ho.nhrc == 1
    assert len(inf["rates"]) == 1 and abs(inf["rates"][0] - Ho.rates()[0]) <= 1e-10 * Ho.rates()[0]


def test_bootstrap_64_cube():
    """64^3 log-normal field, two hierarchies, symmetrized composite."""
    A = W.lognormal7(64, 7)
    params = dict(max_hrc=2, bootstrap_rate=0.05, bootstrap_type=1, smooth_vec=1)
    Ho = oracle.Hierarchy(A, oracle_params(**params))
    Hg = gpu_hierarchy(A, **params)
    assert Hg.info()["nhrc"] == Ho.nhrc == 2
    for j in range(2):
        assert_same_hierarchy(Hg.component(j), Ho.component(j))
    xs, b = W.manufactured_rhs(A, 8)
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    st, it, rel = Hg.solve(dev(b), x, rtol=1e-6)
    xo, ito, relo, sto = Ho.pcg(b, rtol=1e-6)
    say("bootstrap 64^3: iterations gpu %d oracle %d" % (it, ito))
    assert st == 0 and abs(it - ito) <= 1
