"""amg_pcg_solve_noalloc (the solve for callers that cannot allocate) against
amg_pcg_solve, through the C ABI.

Bar: the two solves run the same kernels in the same order, so the solutions
are bit-identical and the iteration counts and residuals equal.  Two calls in
a row share the device's scratch: the second, on a smaller hierarchy, must
not see the first call's state.  The oracle check of amg_pcg_solve itself is
in test_gpu_parity.py; here the no-alloc solve is also held to the oracle's
iterations (+-1) and rtol.
"""
import numpy as np
import pytest

import oracle
import workloads as W

from gpu_helpers import bits, dev, gpu_hierarchy, host, oracle_params, require_gpu, say, torch


def test_max_rows_is_the_scratch_limit():
    import paper_2303_02352_amd as amd
    # (4 MiB - 256 B) / (3 partial sums x 8 B) workgroups of 512 rows
    assert amd.load().amg_pcg_solve_noalloc_max_rows() == (4 * 2 ** 20 - 256) // 24 * 512


CASES = [
    ("poisson40", lambda: W.poisson7(40), {}),
    ("poisson21_ragged", lambda: W.poisson7(21), {}),
]


def _pair(A, params, seed):
    import paper_2303_02352_amd as amd
    xs, b = W.manufactured_rhs(A, seed)
    H = gpu_hierarchy(A, **params)
    bd = dev(b)
    x_ref = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    st_r, it_r, rel_r = H.solve(bd, x_ref, rtol=1e-6)
    x_na = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    st_n, it_n, rel_n = H.solve_noalloc(bd, x_na, rtol=1e-6)
    torch.cuda.synchronize()
    out = (st_r, it_r, rel_r, host(x_ref)), (st_n, it_n, rel_n, host(x_na)), b
    H.close()
    return out


@pytest.mark.gpu
@pytest.mark.parametrize("precision", [0, 1])
def test_noalloc_matches_solve_twice_second_smaller(precision):
    """Two calls in a row (40^3, then the smaller ragged 21^3), in binary64
    and with the binary32 V-cycle: solution bits, iterations, residual and
    status equal to amg_pcg_solve's on the same hierarchy."""
    require_gpu()
    import paper_2303_02352_amd as amd
    for name, make, params in CASES:
        A = make()
        params = dict(params, precision=precision)
        say("no-alloc solve", name, "n=%d" % A.n, params)
        (st_r, it_r, rel_r, x_r), (st_n, it_n, rel_n, x_n), b = _pair(A, params, 11)
        assert st_r == st_n == amd.AMG_OK, (st_r, st_n)
        assert it_n == it_r and rel_n == rel_r, (it_n, it_r, rel_n, rel_r)
        assert np.array_equal(bits(x_n), bits(x_r)), name
        Ho = oracle.Hierarchy(A, oracle_params(**params))
        xo, ito, relo, sto = Ho.pcg(b, rtol=1e-6)
        assert abs(it_n - ito) <= 1 and rel_n <= 1e-6, (it_n, ito, rel_n)


@pytest.mark.gpu
def test_noalloc_zero_rhs_and_maxit():
    """Edge cases through the same path: b = 0 gives 0 iterations; maxit = 2
    stops with NOT_CONVERGED after 2 iterations, as amg_pcg_solve does."""
    require_gpu()
    import paper_2303_02352_amd as amd
    A = W.poisson7(24)
    H = gpu_hierarchy(A)
    z = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    assert H.solve_noalloc(z, x) == (amd.AMG_OK, 0, 0.0)
    xs, b = W.manufactured_rhs(A, 3)
    bd = dev(b)
    xa = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    xb = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    ra = H.solve(bd, xa, rtol=1e-12, maxit=2)
    rb = H.solve_noalloc(bd, xb, rtol=1e-12, maxit=2)
    assert ra == rb and ra[0] == amd.AMG_NOT_CONVERGED and ra[1] == 2, (ra, rb)
    assert np.array_equal(bits(host(xa)), bits(host(xb)))
    H.close()
