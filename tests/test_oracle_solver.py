"""Pins for the oracle's V-cycle and flexible CG (CPU only).

  * V-cycle: equals the dense operator B^k of Sec. 3.1 built from the
    hierarchy's matrices (the printed formula for one sweep, its
    nu-sweep generalisation for more), is symmetric and positive definite,
    and with a single level is A^{-1}.
  * Flexible CG (Sec. 3, Alg. 1): with B = I it reproduces textbook
    Hestenes-Stiefel CG (a different recurrence, written in the test) step
    for step; a single-level hierarchy converges in one iteration; the true
    residual and the error against a direct solve respect rtol and
    kappa * rtol; degenerate and failure cases return the documented codes.
  * Mixed-precision form (the same V-cycle evaluated in binary32): within a
    few units of binary32 rounding of the dense binary64 B^k, and clearly
    not a binary64 evaluation; exact under scaling by powers of two; the
    binary64 flexible CG around it meets rtol on the true residual with
    about the iteration count of the binary64 cycle.
  * Hierarchy facts the paper prints for its own parameter set (Sec. 5):
    4 levels at 130^3 on one node, 5 levels at 300^3, operator complexity
    about 1.14 (tests/golden/paper_hierarchy.json).
"""
import json
import os

import numpy as np
import pytest

import oracle
import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_hierarchy.json")


def _dense_P(Lk, nc):
    P = np.zeros((Lk["n"], nc))
    P[np.arange(Lk["n"]), Lk["agg"]] = Lk["pval"]
    return P


def _smoother_from_zero(A, D, nu):
    """Matrix S with x = S r after nu l1-Jacobi sweeps started from x = 0."""
    n = A.shape[0]
    S = np.zeros((n, n))
    E = np.eye(n) - D @ A
    T = np.eye(n)
    for _ in range(nu):
        S = S + T @ D
        T = E @ T
    return S


def _dense_B(H, pre, post, coarse_sweeps=0):
    """B^k recursively: pre-smooth, coarse correction, post-smooth (Sec. 3.1);
    at the coarsest level A^-1, or coarse_sweeps l1-Jacobi sweeps from zero."""
    levels = [H.level(k) for k in range(H.nlevels)]
    mats = [W.CSR(L["n"], L["row_ptr"], L["col"], L["val"]).scipy().toarray() for L in levels]
    if coarse_sweeps:
        B = _smoother_from_zero(mats[-1], np.diag(levels[-1]["dinv"]), coarse_sweeps)
    else:
        B = np.linalg.inv(mats[-1])
    for k in range(H.nlevels - 2, -1, -1):
        A = mats[k]
        D = np.diag(levels[k]["dinv"])
        P = _dense_P(levels[k], mats[k + 1].shape[0])
        Q = P @ B @ P.T
        S1 = _smoother_from_zero(A, D, pre)
        S2 = _smoother_from_zero(A, D, post)
        C = S1 + Q @ (np.eye(A.shape[0]) - A @ S1)
        B = C + S2 @ (np.eye(A.shape[0]) - A @ C)
    return B, mats, levels


def test_vcycle_equals_printed_operator_one_sweep():
    A = W.poisson7(4)
    H = oracle.Hierarchy(A, oracle.AMGParams(aggr_steps=2, coarse_max=16, pre_sweeps=1,
                                             post_sweeps=1))
    assert H.nlevels == 2
    levels = [H.level(k) for k in range(2)]
    A0 = A.scipy().toarray()
    A1 = W.CSR(levels[1]["n"], levels[1]["row_ptr"], levels[1]["col"], levels[1]["val"]).scipy().toarray()
    Mi = np.diag(levels[0]["dinv"])
    P = _dense_P(levels[0], levels[1]["n"])
    I = np.eye(A.n)
    # B^k = M^-T + M^-1 - M^-T A M^-1 + (I - M^-T A) P B^{k+1} P^T (I - A M^-1)
    Bref = Mi.T + Mi - Mi.T @ A0 @ Mi + (I - Mi.T @ A0) @ P @ np.linalg.inv(A1) @ P.T @ (I - A0 @ Mi)
    Bgot = np.column_stack([H.vcycle(e) for e in np.eye(A.n)])
    assert np.max(np.abs(Bgot - Bref)) <= 1e-13 * np.max(np.abs(Bref))


@pytest.mark.parametrize("maker", ["poisson", "diffusion27"])
def test_vcycle_equals_dense_recursion_multilevel(maker):
    A = W.poisson7(6) if maker == "poisson" else W.diffusion27(5, 3)
    H = oracle.Hierarchy(A, oracle.AMGParams(aggr_steps=2, coarse_max=6))
    assert H.nlevels >= 3
    B, _, _ = _dense_B(H, 4, 4)
    Bgot = np.column_stack([H.vcycle(e) for e in np.eye(A.n)])
    assert np.max(np.abs(Bgot - B)) <= 1e-11 * np.max(np.abs(B))
    # symmetric positive definite operator
    assert np.max(np.abs(Bgot - Bgot.T)) <= 1e-12 * np.max(np.abs(Bgot))
    assert np.min(np.linalg.eigvalsh(0.5 * (Bgot + Bgot.T))) > 0


U32 = 2.0 ** -24   # unit roundoff of binary32


@pytest.mark.parametrize("maker", ["poisson", "diffusion27", "lognormal7"])
@pytest.mark.parametrize("steps,pre,post", [(2, 4, 4), (1, 1, 2)])
def test_binary32_vcycle_within_rounding_of_dense_operator(maker, steps, pre, post):
    """B_32 r against B^k r (binary64, dense): the binary32 cycle rounds the
    matrices, the l1 diagonal, P and r to binary32 and every operation after;
    on these sizes that moves the result by about one unit of binary32
    rounding (measured 0.9-1.7 u), so 64 u bounds it, while a dropped term,
    a wrong sign or index moves it by O(1).  It must also differ from the
    binary64 cycle (whose error is ~1e-16) by more than 1e-9: a binary32
    evaluation really happened."""
    A = {"poisson": lambda: W.poisson7(6), "diffusion27": lambda: W.diffusion27(5, 3),
         "lognormal7": lambda: W.lognormal7(6, 7, ell=2.0)}[maker]()
    H = oracle.Hierarchy(A, oracle.AMGParams(aggr_steps=steps, coarse_max=6, pre_sweeps=pre,
                                             post_sweeps=post))
    assert H.nlevels >= 4
    B, _, _ = _dense_B(H, pre, post)
    for seed in (77, 78):
        r = W.uniform_pm1(seed, A.n)
        ref = B @ r
        err = np.max(np.abs(H.vcycle_f32(r) - ref)) / np.max(np.abs(ref))
        assert 1e-9 < err <= 64 * U32
        # scaling by a power of two commutes with every binary32 rounding
        s = 2.0 ** -5
        assert np.array_equal(H.vcycle_f32(r * s), H.vcycle_f32(r) * s)


@pytest.mark.parametrize("maker", ["poisson", "diffusion27"])
def test_binary32_vcycle_with_sweeps_at_the_coarsest_level(maker):
    """Coarsest level solved by 20 l1-Jacobi sweeps (the paper's setting):
    the binary32 cycle against the dense binary64 operator whose coarsest
    block is the 20-sweep polynomial, same 64 u bound; the binary64 cycle
    equals that operator to 1e-12."""
    A = {"poisson": lambda: W.poisson7(6), "diffusion27": lambda: W.diffusion27(5, 3)}[maker]()
    H = oracle.Hierarchy(A, oracle.AMGParams(aggr_steps=2, coarse_max=12, coarse_solver=1,
                                             coarse_sweeps=20))
    assert H.nlevels >= 3 and not H.coarse_dense
    B, _, _ = _dense_B(H, 4, 4, coarse_sweeps=20)
    for seed in (77, 78):
        r = W.uniform_pm1(seed, A.n)
        ref = B @ r
        assert np.max(np.abs(H.vcycle(r) - ref)) <= 1e-12 * np.max(np.abs(ref))
        err = np.max(np.abs(H.vcycle_f32(r) - ref)) / np.max(np.abs(ref))
        assert 1e-9 < err <= 64 * U32


@pytest.mark.parametrize("maker,N", [("poisson", 16), ("diffusion27", 10), ("lognormal7", 12)])
def test_mixed_pcg_meets_rtol(maker, N):
    """Alg. 1 in binary64 around the binary32 cycle: the true residual
    b - A x (scipy) meets rtol, and the flexible iteration count is within two
    of the count with the binary64 cycle."""
    A = {"poisson": lambda: W.poisson7(N), "diffusion27": lambda: W.diffusion27(N, 3),
         "lognormal7": lambda: W.lognormal7(N, 7, ell=3.0)}[maker]()
    xs, b = W.manufactured_rhs(A, 5)
    H = oracle.Hierarchy(A, oracle.AMGParams(smooth_vec=1 if maker != "poisson" else 0))
    assert H.nlevels >= 2
    rtol = 1e-6
    x, it, rel, st = H.pcg(b, rtol=rtol, mixed=True)
    x64, it64, rel64, st64 = H.pcg(b, rtol=rtol)
    assert st == oracle.OK and st64 == oracle.OK
    assert rel <= rtol
    assert np.linalg.norm(b - A.scipy() @ x) / np.linalg.norm(b) <= rtol * 1.01
    assert abs(it - it64) <= 2


def test_vcycle_symmetry_and_positivity_32():
    A = W.poisson7(32)
    H = oracle.Hierarchy(A)
    x, y = W.uniform_pm1(31, A.n), W.uniform_pm1(32, A.n)
    Bx, By = H.vcycle(x), H.vcycle(y)
    assert abs(Bx @ y - x @ By) <= 1e-13 * abs(Bx @ y) + 1e-14 * np.linalg.norm(Bx) * np.linalg.norm(y)
    assert Bx @ x > 0


def test_single_level_is_exact_inverse():
    A = W.poisson7(4)                               # 64 rows <= coarse_max = 100
    H = oracle.Hierarchy(A)
    assert H.nlevels == 1 and H.coarse_dense
    r = W.uniform_pm1(41, A.n)
    z = H.vcycle(r)
    zr = np.linalg.solve(A.scipy().toarray(), r)
    assert np.max(np.abs(z - zr)) <= 1e-13 * np.max(np.abs(zr)) * 10
    xs, b = W.manufactured_rhs(A, 1)
    x, it, rel, st = H.pcg(b)
    assert st == oracle.OK and it == 1


def _textbook_cg(S, b, rtol, maxit):
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rr = r @ r
    nr0 = np.sqrt(rr)
    it = 0
    while np.sqrt(rr) > rtol * nr0 and it < maxit:
        Ap = S @ p
        a = rr / (p @ Ap)
        x += a * p
        r -= a * Ap
        it += 1
        rr_new = r @ r
        p = r + (rr_new / rr) * p
        rr = rr_new
    return x, it


def test_identity_preconditioner_is_textbook_cg():
    A = W.poisson7(10)
    xs, b = W.manufactured_rhs(A, 3)
    H = oracle.Hierarchy(A, oracle.AMGParams(precond=0))
    x, it, rel, st = H.pcg(b, rtol=1e-8)
    xr, itr = _textbook_cg(A.scipy(), b, 1e-8, 1000)
    assert st == oracle.OK
    assert abs(it - itr) <= 1
    assert np.max(np.abs(x - xr)) <= 1e-7 * np.max(np.abs(xr))


def test_cg_on_tiny_system_finishes_within_n_steps():
    A = W.poisson7(3)        # 27 unknowns, distinct eigenvalues <= 27
    xs, b = W.manufactured_rhs(A, 4)
    H = oracle.Hierarchy(A, oracle.AMGParams(precond=0))
    x, it, rel, st = H.pcg(b, rtol=1e-12)
    assert st == oracle.OK and it <= 27


@pytest.mark.parametrize("maker,N", [("poisson", 16), ("diffusion27", 10), ("lognormal7", 12)])
def test_pcg_meets_rtol_and_direct_solution(maker, N):
    import scipy.sparse.linalg as spla
    A = {"poisson": lambda: W.poisson7(N), "diffusion27": lambda: W.diffusion27(N, 3),
         "lognormal7": lambda: W.lognormal7(N, 7, ell=3.0)}[maker]()
    xs, b = W.manufactured_rhs(A, 5)
    H = oracle.Hierarchy(A, oracle.AMGParams(smooth_vec=1 if maker != "poisson" else 0))
    rtol = 1e-6
    x, it, rel, st = H.pcg(b, rtol=rtol)
    assert st == oracle.OK
    S = A.scipy()
    true_rel = np.linalg.norm(b - S @ x) / np.linalg.norm(b)
    assert rel <= rtol
    assert true_rel <= rtol * 1.01
    xd = spla.spsolve(S.tocsc(), b)
    ev = np.linalg.eigvalsh(S.toarray()) if A.n <= 2000 else None
    kappa = ev[-1] / ev[0] if ev is not None else 1e4
    assert np.linalg.norm(x - xd) <= kappa * rtol * np.linalg.norm(xd)


def test_pcg_iteration_counts_32():
    """Iteration count at 32^3 (configuration of the small parity workload)."""
    A = W.poisson7(32)
    xs, b = W.manufactured_rhs(A, 1)
    H = oracle.Hierarchy(A)
    assert [s[0] for s in H.sizes()] == [32768, 8192, 2048, 512, 128, 64]
    x, it, rel, st = H.pcg(b)
    assert st == oracle.OK and rel <= 1e-6
    assert 5 <= it <= 15


def test_pcg_failure_codes():
    A = W.poisson7(6)
    xs, b = W.manufactured_rhs(A, 1)
    H = oracle.Hierarchy(A)
    x, it, rel, st = H.pcg(b, rtol=1e-30, maxit=3)
    assert st == oracle.NOT_CONVERGED and it == 3
    bb = b.copy(); bb[3] = np.nan
    x, it, rel, st = H.pcg(bb)
    assert st == oracle.NONFINITE
    x, it, rel, st = H.pcg(np.zeros(A.n))
    assert st == oracle.OK and it == 0
    # symmetric with positive diagonal but indefinite: 2x2 block [[1, 2], [2, 1]] pattern
    n = 4
    D = np.array([[1.0, 2.0, 0, 0], [2.0, 1.0, 0, 0], [0, 0, 1.0, 0], [0, 0, 0, 1.0]])
    import scipy.sparse as sp
    Sx = sp.csr_matrix(D)
    Ai = W.CSR(n, Sx.indptr.astype(np.int32), Sx.indices.astype(np.int32), Sx.data.copy())
    with pytest.raises(oracle.OracleError) as e:
        oracle.Hierarchy(Ai)        # single level: Cholesky of an indefinite matrix
    assert e.value.status == oracle.NOT_SPD
    Hn = oracle.Hierarchy(Ai, oracle.AMGParams(precond=0))
    x, it, rel, st = Hn.pcg(np.array([1.0, -1.0, 0.0, 0.0]))
    assert st == oracle.NOT_SPD


def test_relaxed_smooth_vector_is_normalised():
    A = W.lognormal7(8, 7, ell=2.0)
    H = oracle.Hierarchy(A, oracle.AMGParams(smooth_vec=1, smooth_sweeps=20))
    w = H.level(0)["w"]
    assert np.max(np.abs(w)) == 1.0
    # twenty sweeps of x + dinv (0 - A x) from ones, written densely
    S = A.scipy().toarray()
    d = oracle.l1_dinv(A)
    x = np.ones(A.n)
    for _ in range(20):
        x = x - d * (S @ x)
    assert np.allclose(w, x / np.max(np.abs(x)), rtol=1e-12, atol=1e-14)


def _paper_params(nd):
    g = json.load(open(GOLDEN))["params"]
    return oracle.AMGParams(aggr_steps=g["aggr_steps"], coarse_max=g["coarse_max_per_nd"] * nd,
                            max_levels=g["max_levels"], coarse_solver=1,
                            coarse_sweeps=g["coarse_sweeps"], pre_sweeps=g["pre_sweeps"],
                            post_sweeps=g["post_sweeps"])


def test_paper_hierarchy_130():
    g = json.load(open(GOLDEN))
    nd = g["weak_scaling_130"]["nd"]
    A = W.poisson7(nd)
    H = oracle.Hierarchy(A, _paper_params(nd))
    assert H.nlevels == g["weak_scaling_130"]["levels_on_one_node"]
    assert abs(H.opc() - g["operator_complexity"]["value"]) <= g["operator_complexity"]["tolerance"]


@pytest.mark.slow
def test_paper_hierarchy_300():
    g = json.load(open(GOLDEN))
    nd = g["strong_scaling_300"]["nd"]
    A = W.poisson7(nd)
    H = oracle.Hierarchy(A, _paper_params(nd))
    assert H.nlevels == g["strong_scaling_300"]["levels"]
    assert abs(H.opc() - g["operator_complexity"]["value"]) <= g["operator_complexity"]["tolerance"]


def test_coarse_inverse_against_numpy():
    """The coarsest direct solve multiplies by A_c^-1, whose columns come from
    the Cholesky factor; it must agree with numpy's inverse."""
    A = W.diffusion27(6, 3)
    H = oracle.Hierarchy(A, oracle.AMGParams(coarse_max=60))
    assert H.coarse_dense
    lv = H.level(H.nlevels - 1)
    Ac = W.CSR(lv["n"], lv["row_ptr"], lv["col"], lv["val"]).scipy().toarray()
    Ai = H.coarse_inverse()
    ref = np.linalg.inv(Ac)
    assert np.max(np.abs(Ai - ref)) <= 1e-13 * np.linalg.cond(Ac) * np.max(np.abs(ref))
    assert np.max(np.abs(Ai @ Ac - np.eye(lv["n"]))) <= 1e-12
