"""Pins for the oracle's bootstrap composite AMG (Appendix A: bootstrap_type,
max_hrc, desired convergence rate), CPU only.

  * max_hrc = 1 is the plain preconditioner, bit for bit, with no estimate;
  * on a tiny problem each hierarchy's preconditioner is taken as a dense
    matrix B_j (its V-cycle applied to unit vectors), and the composite must
    equal the operator its rule defines:
      multiplicative  B = (I - (I - B_m A) ... (I - B_1 A)) A^-1,
      symmetrized     the same with E = (I-B_1 A)..(I-B_m A)..(I-B_1 A),
      additive        B = (B_1 + ... + B_m) / m;
  * the symmetrized and additive composites are symmetric positive definite,
    the multiplicative one is not symmetric;
  * the rate estimate equals (||E^its x0||_A / ||x0||_A)^(1/its) with the
    dense error propagator and a start vector drawn here from the published
    SplitMix64 definition, and the next hierarchy's smooth vector is E^its x0
    scaled by its largest magnitude;
  * the stop rule: a desired rate of 1 keeps one hierarchy; a tiny one builds
    max_hrc hierarchies and estimates max_hrc rates;
  * PCG with each composite reaches rtol on the true residual.
"""
import numpy as np
import pytest

import oracle
import workloads as W


def _bits(a):
    return np.ascontiguousarray(a, np.float64).view(np.uint64)


def _dense_b(H, single=False):
    n = H.n
    B = np.empty((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        B[:, j] = H.vcycle(e, single=single)
    return B


def _start_vector(n, seed, j):
    base = ((16 * seed + j) & 0xFFFFFFFF) << 32
    with np.errstate(over="ignore"):
        bits = W.splitmix64(np.uint64(base) + np.arange(n, dtype=np.uint64))
    return 2.0 * ((bits >> np.uint64(11)).astype(np.float64) * 2.0 ** -53) - 1.0


def test_one_hierarchy_is_the_plain_preconditioner():
    A = W.lognormal7(10, 4, ell=3.0)
    H1 = oracle.Hierarchy(A, oracle.AMGParams())
    H2 = oracle.Hierarchy(A, oracle.AMGParams(max_hrc=1, bootstrap_type=1, bootstrap_rate=0.01))
    assert H2.nhrc == 1 and len(H2.rates()) == 0
    r = W.uniform_pm1(5, A.n)
    assert np.array_equal(_bits(H1.vcycle(r)), _bits(H2.vcycle(r)))


PARAMS = dict(max_hrc=3, bootstrap_rate=1e-3, bootstrap_its=6, coarse_max=6, smooth_vec=1, smooth_sweeps=3)


@pytest.fixture(scope="module")
def tiny():
    A = W.lognormal7(5, 9, ell=2.0)
    return A, A.scipy().toarray()


@pytest.mark.parametrize("btype", [0, 1, 2])
def test_composite_equals_its_dense_operator(tiny, btype):
    A, Ad = tiny
    H = oracle.Hierarchy(A, oracle.AMGParams(bootstrap_type=btype, **PARAMS))
    m = H.nhrc
    assert m == 3
    Bs = [_dense_b(H.component(j), single=True) for j in range(m)]
    I = np.eye(A.n)
    if btype == 2:
        B = sum(Bs) / m
    else:
        order = list(range(m)) if btype == 0 else list(range(m)) + list(range(m - 2, -1, -1))
        E = I
        for j in order:                       # applied first = rightmost factor
            E = (I - Bs[j] @ Ad) @ E
        B = (I - E) @ np.linalg.inv(Ad)
    Bc = _dense_b(H)
    assert np.max(np.abs(Bc - B)) <= 1e-10 * np.max(np.abs(B))
    sym = np.max(np.abs(Bc - Bc.T)) / np.max(np.abs(Bc))
    if btype in (1, 2):
        assert sym <= 1e-12
        assert np.min(np.linalg.eigvalsh((Bc + Bc.T) / 2)) > 0
    else:
        assert sym > 1e-6


@pytest.mark.parametrize("btype", [0, 1])
def test_rate_estimate_and_next_smooth_vector(tiny, btype):
    A, Ad = tiny
    p = oracle.AMGParams(bootstrap_type=btype, **PARAMS)
    H = oracle.Hierarchy(A, p)
    rates = H.rates()
    assert len(rates) == 3
    I = np.eye(A.n)
    for m in (1, 2, 3):
        # dense error propagator of the first m hierarchies' composite
        sub = oracle.Hierarchy(A, oracle.AMGParams(**dict(vars(p), max_hrc=m)))
        assert sub.nhrc == m
        Em = I - _dense_b(sub) @ Ad
        x0 = _start_vector(A.n, p.bootstrap_seed, m)
        x = np.linalg.matrix_power(Em, p.bootstrap_its) @ x0
        want = (np.sqrt(x @ Ad @ x) / np.sqrt(x0 @ Ad @ x0)) ** (1.0 / p.bootstrap_its)
        assert abs(rates[m - 1] - want) <= 1e-9 * want, (m, rates[m - 1], want)
        if m < 3:
            w = H.component(m).level(0)["w"]
            assert np.max(np.abs(w - x / np.max(np.abs(x)))) <= 1e-9


def test_stop_rule():
    A = W.poisson7(12)
    H = oracle.Hierarchy(A, oracle.AMGParams(max_hrc=4, bootstrap_rate=1.0))
    assert H.nhrc == 1 and len(H.rates()) == 1 and H.rates()[0] <= 1.0
    H = oracle.Hierarchy(A, oracle.AMGParams(max_hrc=3, bootstrap_rate=1e-6))
    assert H.nhrc == 3 and len(H.rates()) == 3


@pytest.mark.parametrize("btype", [0, 1, 2])
def test_composite_pcg_converges(btype):
    A = W.lognormal7(16, 7, ell=4.0)
    xs, b = W.manufactured_rhs(A, 3)
    plain = oracle.Hierarchy(A, oracle.AMGParams())
    _, it1, _, _ = plain.pcg(b, rtol=1e-6)
    H = oracle.Hierarchy(A, oracle.AMGParams(max_hrc=3, bootstrap_type=btype, bootstrap_rate=0.05))
    assert H.nhrc == 3
    for mixed in (False, True):
        x, it, rel, st = H.pcg(b, rtol=1e-6, mixed=mixed)
        assert st == oracle.OK and rel <= 1e-6
        assert np.linalg.norm(b - A.scipy() @ x) / np.linalg.norm(b) <= 1.01e-6
        assert it <= it1
