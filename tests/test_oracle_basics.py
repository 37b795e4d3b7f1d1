"""Pins for the oracle's building blocks (CPU only).

Each pin compares the oracle with something other than itself:
  * SplitMix64: the published first outputs of the stream with state 0.
  * 7-point generator: nnz = 7N^3 - 6N^2, zero interior row sums, symmetry.
  * SpMV: the closed-form eigenpairs of the discrete Laplacian
    (lambda = 6 - 2cos(p pi/(N+1)) - 2cos(q pi/(N+1)) - 2cos(r pi/(N+1)),
    sine-product eigenvectors) and exact integer arithmetic on integer x.
  * l1 diagonal (Sec. 3.1): Poisson row -> 6 + number of in-domain neighbours.
  * Matching weights: the closed form 7/6 on Poisson with w = 1, invariance
    under w -> c w, the M-matrix bound >= 1, and an independent formulation
    as the energy ratio v^T A_2 v / v^T D_2 v of the 2x2 principal block on
    v = (w_i, -w_j).
  * Cholesky: numpy.linalg.cholesky and numpy.linalg.solve.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W


def test_splitmix64_published_stream():
    z = W.splitmix64(np.array([0, 0x9E3779B97F4A7C15], dtype=np.uint64))
    assert int(z[0]) == 0xE220A8397B1DCDAF
    assert int(z[1]) == 0x6E789E6AA1B965F4


@pytest.mark.parametrize("N", [1, 2, 3, 5, 8])
def test_poisson7_structure(N):
    A = W.poisson7(N)
    assert A.nnz == 7 * N ** 3 - 6 * N ** 2
    assert oracle.validate(A) == oracle.OK
    S = A.scipy()
    assert (S - S.T).nnz == 0
    # interior rows sum to zero, boundary rows to the number of missing neighbours
    rs = np.asarray(S.sum(axis=1)).ravel()
    idx = np.arange(N ** 3)
    x, y, z = idx % N, (idx // N) % N, idx // (N * N)
    missing = sum(((c == 0).astype(int) + (c == N - 1).astype(int)) for c in (x, y, z))
    assert np.array_equal(rs, missing.astype(float))


def _laplacian_eigpair(N, p, q, r):
    h = math.pi / (N + 1)
    lam = 6 - 2 * math.cos(p * h) - 2 * math.cos(q * h) - 2 * math.cos(r * h)
    i = np.arange(1, N + 1)
    sx, sy, sz = np.sin(p * h * i), np.sin(q * h * i), np.sin(r * h * i)
    v = (sz[:, None, None] * sy[None, :, None] * sx[None, None, :]).ravel()
    return lam, v


@pytest.mark.parametrize("N,pqr", [(6, (1, 1, 1)), (7, (2, 5, 3)), (9, (9, 1, 4))])
def test_spmv_closed_form_eigenpairs(N, pqr):
    A = W.poisson7(N)
    lam, v = _laplacian_eigpair(N, *pqr)
    y = oracle.spmv(A, v)
    assert np.max(np.abs(y - lam * v)) <= 1e-13 * np.max(np.abs(v)) * 12


def test_spmv_integer_exact():
    A = W.poisson7(7)
    x = np.round(W.uniform_pm1(11, A.n) * 1000)
    y = oracle.spmv(A, x)
    # exact reference in Python integers, row by row
    rp, ci, va = A.row_ptr, A.col, A.val
    for i in range(A.n):
        s = sum(int(va[k]) * int(x[ci[k]]) for k in range(rp[i], rp[i + 1]))
        assert y[i] == float(s)


def test_l1_diagonal_poisson():
    N = 5
    A = W.poisson7(N)
    d = oracle.l1_dinv(A)
    idx = np.arange(N ** 3)
    x, y, z = idx % N, (idx // N) % N, idx // (N * N)
    nb = sum(((c > 0).astype(int) + (c < N - 1).astype(int)) for c in (x, y, z))
    assert np.array_equal(1.0 / d, 6.0 + nb)


def test_weights_poisson_closed_form():
    A = W.poisson7(4)
    wt = oracle.edge_weights(A, np.ones(A.n))
    off = A.col != np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    assert np.all(np.abs(wt[off] - 7.0 / 6.0) <= 2.0 ** -52 * 2)
    assert np.all(np.isnan(wt[~off]))


def _spd_random(n, seed, density=0.3):
    u = W.uniform(seed, n * n).reshape(n, n)
    vals = W.uniform_pm1(seed + 1, n * n).reshape(n, n)
    M = np.where(u < density, vals, 0.0)
    M = np.triu(M, 1)
    M = M + M.T
    np.fill_diagonal(M, np.abs(M).sum(axis=1) + 0.5)
    return M


def _dense_to_csr(D):
    import scipy.sparse as sp
    S = sp.csr_matrix(D)
    S.sort_indices()
    # keep the diagonal even when it is the only entry
    return W.CSR(D.shape[0], S.indptr.astype(np.int32), S.indices.astype(np.int32),
                 S.data.astype(np.float64))


def test_weights_energy_ratio_and_invariance():
    D = _spd_random(30, 3)
    A = _dense_to_csr(D)
    w = W.uniform_pm1(5, 30) + 1.5
    wt = oracle.edge_weights(A, w)
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    for k in range(A.nnz):
        i, j = rows[k], A.col[k]
        if i == j:
            continue
        A2 = np.array([[D[i, i], D[i, j]], [D[j, i], D[j, j]]])
        v = np.array([w[i], -w[j]])
        ratio = v @ A2 @ v / (v @ np.diag(np.diag(A2)) @ v)
        assert abs(wt[k] - ratio) <= 1e-14 * max(1.0, abs(ratio))
    wt3 = oracle.edge_weights(A, 3.0 * w)
    off = rows != A.col
    assert np.allclose(wt3[off], wt[off], rtol=1e-14, atol=0)


def test_weights_m_matrix_at_least_one():
    A = W.diffusion27(5, 3)
    w = 0.5 + W.uniform(9, A.n)
    wt = oracle.edge_weights(A, w)
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    assert np.all(wt[rows != A.col] >= 1.0)


def test_cholesky_against_numpy():
    D = _spd_random(40, 21)
    st, L = oracle.cholesky(D)
    assert st == oracle.OK
    Lref = np.linalg.cholesky(D)
    assert np.max(np.abs(L - Lref)) <= 1e-13 * np.max(np.abs(Lref))
    r = W.uniform_pm1(22, 40)
    x = oracle.chol_solve(L, r)
    xr = np.linalg.solve(D, r)
    assert np.max(np.abs(x - xr)) <= 1e-13 * np.max(np.abs(xr)) * np.linalg.cond(D)


def test_cholesky_rejects_indefinite():
    D = np.array([[1.0, 2.0], [2.0, 1.0]])
    st, _ = oracle.cholesky(D)
    assert st == oracle.NOT_SPD


def test_validate_rejects_bad_inputs():
    A = W.poisson7(3)
    assert oracle.validate(A) == oracle.OK
    B = W.CSR(A.n, A.row_ptr.copy(), A.col.copy(), A.val.copy())
    B.val[0] = -B.val[0]            # diagonal of row 0 is its first entry
    assert oracle.validate(B) == oracle.NOT_SPD
    B = W.CSR(A.n, A.row_ptr.copy(), A.col.copy(), A.val.copy())
    B.val[1] = np.nan
    assert oracle.validate(B) == oracle.NONFINITE
    B = W.CSR(A.n, A.row_ptr.copy(), A.col.copy(), A.val.copy())
    B.val[1] = -0.5                 # breaks bitwise symmetry
    assert oracle.validate(B) == oracle.INVALID
    B = W.CSR(A.n, A.row_ptr.copy(), A.col.copy(), A.val.copy())
    B.col[[0, 1]] = B.col[[1, 0]]   # unsorted row
    assert oracle.validate(B) == oracle.INVALID
