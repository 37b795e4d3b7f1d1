"""Pins for the oracle's cycle and smoother options (Appendix A: cycle_type
V/H/W; relax_type and coarse_relax Jacobi, FGS/BGS, symmetrized GS,
l1-Jacobi), CPU only.

The preconditioner is rebuilt here as a dense matrix from the textbook
multigrid recursion, written independently of the oracle's loops:
  B_nl = A_nl^-1 (direct) or (I - S_c) A_nl^-1 for coarsest sweeps,
  E_k  = S_post^nu2 (I - P_k Bt_{k+1} P_k^T A_k) S_pre^nu1,  B_k = (I - E_k) A_k^-1,
  Bt_{k+1} = (I - (I - B_{k+1} A_{k+1})^g_k) A_{k+1}^-1   (g_k coarse cycles),
with the smoothers' error propagators
  Jacobi I - D^-1 A, l1-Jacobi I - M^-1 A, forward GS I - (D + L)^-1 A,
  backward GS I - (D + U)^-1 A, symmetrized GS the backward after the forward,
and g_k = 1 (V), 2 (W), 2 on odd levels and 1 on even ones (H).  The
oracle's cycle applied to unit vectors must equal it; the Gauss-Seidel
cycles are symmetric (forward before, backward after the correction); PCG
reaches rtol with every option.
"""
import numpy as np
import pytest

import oracle
import workloads as W


def _dense(level):
    import scipy.sparse as sp
    n = level["n"]
    return sp.csr_matrix((level["val"], level["col"], level["row_ptr"]), shape=(n, n)).toarray()


def _smoother_e(A, typ, where):
    """Error propagator of one sweep; where: 'pre', 'post' or a coarsest pass index."""
    D = np.diag(np.diag(A))
    I = np.eye(A.shape[0])
    L = np.tril(A, -1)
    U = np.triu(A, 1)
    if typ == 4:
        return I - np.diag(1.0 / np.abs(A).sum(axis=1)) @ A
    if typ == 0:
        return I - np.linalg.inv(D) @ A
    EF = I - np.linalg.inv(D + L) @ A
    EB = I - np.linalg.inv(D + U) @ A
    if typ == 3:
        return EB @ EF
    if where == "pre":
        return EF
    if where == "post":
        return EB
    return EF if where % 2 == 0 else EB


def _dense_b(H, p):
    nl = H.nlevels
    lev = [H.level(k) for k in range(nl)]
    A = [_dense(l) for l in lev]

    def g(k):
        return {0: 1, 2: 2, 1: 2 if k % 2 == 1 else 1}[p.cycle_type]

    def B(k):
        Ak = A[k]
        I = np.eye(Ak.shape[0])
        Ainv = np.linalg.inv(Ak)
        if k == nl - 1:
            if H.coarse_dense:
                return Ainv
            E = I
            for q in range(p.coarse_sweeps):
                E = _smoother_e(Ak, p.coarse_relax, q) @ E
            return (I - E) @ Ainv
        n, nc = Ak.shape[0], A[k + 1].shape[0]
        P = np.zeros((n, nc))
        P[np.arange(n), lev[k]["agg"]] = lev[k]["pval"]
        Bc = B(k + 1)
        Ic = np.eye(nc)
        Bt = (Ic - np.linalg.matrix_power(Ic - Bc @ A[k + 1], g(k))) @ np.linalg.inv(A[k + 1])
        Spre = np.linalg.matrix_power(_smoother_e(Ak, p.relax_type, "pre"), p.pre_sweeps)
        Spost = np.linalg.matrix_power(_smoother_e(Ak, p.relax_type, "post"), p.post_sweeps)
        E = Spost @ (I - P @ Bt @ P.T @ Ak) @ Spre
        return (I - E) @ Ainv

    return B(0)


def _oracle_b(H):
    n = H.n
    M = np.empty((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        M[:, j] = H.vcycle(e)
    return M


@pytest.fixture(scope="module")
def tiny():
    return W.lognormal7(5, 11, ell=2.0)


@pytest.mark.parametrize("cycle", [0, 1, 2])
@pytest.mark.parametrize("relax", [0, 1, 3, 4])
def test_cycle_equals_dense_recursion(tiny, cycle, relax):
    A = tiny
    p = oracle.AMGParams(cycle_type=cycle, relax_type=relax, coarse_max=4, aggr_steps=1,
                         pre_sweeps=2, post_sweeps=1, smooth_vec=1, smooth_sweeps=3)
    H = oracle.Hierarchy(A, p)
    assert H.nlevels >= 4
    Bd = _dense_b(H, p)
    Bo = _oracle_b(H)
    assert np.max(np.abs(Bo - Bd)) <= 1e-11 * np.max(np.abs(Bd)), (cycle, relax)


@pytest.mark.parametrize("crelax", [0, 1, 3, 4])
def test_coarsest_sweeps_each_type(tiny, crelax):
    A = tiny
    p = oracle.AMGParams(cycle_type=2, relax_type=3, coarse_relax=crelax, coarse_solver=1, coarse_sweeps=6,
                         coarse_max=20, aggr_steps=2)
    H = oracle.Hierarchy(A, p)
    assert not H.coarse_dense and H.nlevels >= 2
    Bd = _dense_b(H, p)
    assert np.max(np.abs(_oracle_b(H) - Bd)) <= 1e-11 * np.max(np.abs(Bd))


@pytest.mark.parametrize("cycle,relax", [(0, 1), (2, 1), (1, 3), (2, 0)])
def test_symmetric_cycles(cycle, relax):
    A = W.poisson7(10)
    H = oracle.Hierarchy(A, oracle.AMGParams(cycle_type=cycle, relax_type=relax, coarse_max=20))
    x, y = W.uniform_pm1(1, A.n), W.uniform_pm1(2, A.n)
    bx, by = H.vcycle(x), H.vcycle(y)
    assert abs(bx @ y - x @ by) <= 1e-12 * abs(bx @ y)
    assert bx @ x > 0


def test_gauss_seidel_pass_is_a_triangular_solve():
    """One forward pass from zero solves (D + L) x = r; one backward pass (D + U) x = r."""
    A = W.lognormal7(4, 3, ell=2.0)
    Ad = A.scipy().toarray()
    r = W.uniform_pm1(7, A.n)
    for relax, M in ((1, np.tril(Ad)), ):
        p = oracle.AMGParams(relax_type=relax, coarse_max=A.n, coarse_solver=1, coarse_relax=1,
                             coarse_sweeps=1, max_levels=1)
        H = oracle.Hierarchy(A, p)
        assert H.nlevels == 1
        assert np.max(np.abs(H.vcycle(r) - np.linalg.solve(M, r))) <= 1e-13 * np.max(np.abs(r))


@pytest.mark.parametrize("cycle", [0, 1, 2])
@pytest.mark.parametrize("relax", [0, 1, 3, 4])
def test_pcg_converges_with_every_option(cycle, relax):
    A = W.lognormal7(16, 7, ell=4.0)
    xs, b = W.manufactured_rhs(A, 2)
    H = oracle.Hierarchy(A, oracle.AMGParams(cycle_type=cycle, relax_type=relax, smooth_vec=1))
    x, it, rel, st = H.pcg(b, rtol=1e-6)
    assert st == oracle.OK and rel <= 1e-6, (st, it, rel)
    assert np.linalg.norm(b - A.scipy() @ x) / np.linalg.norm(b) <= 1.01e-6
