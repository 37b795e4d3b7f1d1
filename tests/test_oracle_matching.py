"""Pins for the oracle's matching, aggregation and Galerkin product (CPU only).

  * Matching (Sec. 4.1, 1/2-approximate MWM): exhaustive maximum weight
    matching on random graphs with <= 12 vertices; the oracle's matching is
    valid, maximal over eligible edges, locally dominant, weighs >= 1/2 of
    the optimum, and the independent sequential Suitor gives the same mate[]
    for random proposal orders.
  * Aggregates: on Poisson with even N and w = 1 the first pairwise step
    pairs (2m, 2m+1) along x; two steps give 2x2x1 boxes.
  * Prolongator: P^T P = I and P w_c = w (P built densely in the test).
  * Galerkin (Sec. 3.1): A_c equals the dense product P^T A P, is bitwise
    symmetric, and matches the closed-form coarse stencils of the box
    aggregates (first step: diagonal 5, x -1/2, y/z -1; after two steps:
    diagonal 4, x/y -1/2, z -1).
"""
import itertools

import numpy as np
import pytest

import oracle
import workloads as W


def _random_graph(n, seed, density=0.45, ties=False):
    u = W.uniform(seed, n * n).reshape(n, n)
    vals = -(0.1 + W.uniform(seed + 1, n * n).reshape(n, n))
    if ties:
        vals = -np.round(1 + 2 * W.uniform(seed + 1, n * n).reshape(n, n))
    M = np.triu(np.where(u < density, vals, 0.0), 1)
    M = M + M.T
    np.fill_diagonal(M, np.abs(M).sum(axis=1) + 1.0)
    import scipy.sparse as sp
    S = sp.csr_matrix(M)
    S.sort_indices()
    return M, W.CSR(n, S.indptr.astype(np.int32), S.indices.astype(np.int32), S.data.copy())


def _eligible_edges(M, w):
    n = M.shape[0]
    E = {}
    for i in range(n):
        for j in range(i + 1, n):
            if M[i, j] != 0.0:
                v = np.array([w[i], -w[j]])
                A2 = M[np.ix_([i, j], [i, j])]
                wt = v @ A2 @ v / (v @ np.diag(np.diag(A2)) @ v)
                if wt > 0:
                    E[(i, j)] = wt
    return E


def _brute_mwm(n, E):
    best = [0.0]
    edges = sorted(E)

    def rec(k, used, acc):
        if acc + sum(E[e] for e in edges[k:]) <= best[0]:
            return
        if k == len(edges):
            best[0] = max(best[0], acc)
            return
        i, j = edges[k]
        if i not in used and j not in used:
            rec(k + 1, used | {i, j}, acc + E[(i, j)])
        rec(k + 1, used, acc)

    rec(0, frozenset(), 0.0)
    return best[0]


@pytest.mark.parametrize("seed", range(12))
def test_matching_half_approx_and_valid(seed):
    n = 6 + seed % 7
    M, A = _random_graph(n, 100 + seed, ties=(seed % 3 == 0))
    w = 0.5 + W.uniform(300 + seed, n)
    mate = oracle.match_greedy(A, w)
    E = _eligible_edges(M, w)
    # valid: symmetric pairing over eligible edges
    for i in range(n):
        j = mate[i]
        if j >= 0:
            assert mate[j] == i and j != i
            assert (min(i, j), max(i, j)) in E
    # maximal: no eligible edge joins two free vertices
    for (i, j) in E:
        assert mate[i] >= 0 or mate[j] >= 0
    # weight within 1/2 of the exhaustive optimum
    got = sum(E[(i, mate[i])] for i in range(n) if mate[i] > i)
    opt = _brute_mwm(n, E)
    assert got >= 0.5 * opt - 1e-12
    # locally dominant under the key (weight, max id, min id)
    key = {e: (E[e], e[1], e[0]) for e in E}
    for i in range(n):
        j = mate[i]
        if j > i:
            k = key[(i, j)]
            for e in E:
                if (i in e or j in e):
                    other = e[0] if e[1] in (i, j) else e[1]
                    # edges to vertices matched by a heavier edge may be heavier
                    if mate[other] >= 0 and key[(min(other, mate[other]), max(other, mate[other]))] > k:
                        continue
                    assert key[e] <= k


@pytest.mark.parametrize("seed", range(8))
def test_suitor_equals_greedy(seed):
    n = 40
    M, A = _random_graph(n, 500 + seed, density=0.2, ties=(seed % 2 == 0))
    w = np.ones(n) if seed % 2 == 0 else 0.2 + W.uniform(600 + seed, n)
    g = oracle.match_greedy(A, w)
    for t in range(4):
        order = np.argsort(W.uniform(700 + 10 * seed + t, n)).astype(np.int32)
        s = oracle.match_suitor(A, w, order)
        assert np.array_equal(g, s)


def _dense_P(n, nc, agg, pval):
    P = np.zeros((n, nc))
    P[np.arange(n), agg] = pval
    return P


def test_first_step_pairs_along_x():
    N = 6
    A = W.poisson7(N)
    st = oracle.pairwise_step(A, np.ones(A.n))
    idx = np.arange(A.n)
    assert np.array_equal(st["mate"], np.where(idx % 2 == 0, idx + 1, idx - 1))
    assert st["nc"] == A.n // 2
    assert np.all(st["pval"] == 1.0 / np.sqrt(2.0))


def test_galerkin_dense_and_symmetry_and_stencil():
    N = 6
    A = W.poisson7(N)
    w = np.ones(A.n)
    st = oracle.pairwise_step(A, w)
    P = _dense_P(A.n, st["nc"], st["agg"], st["pval"])
    assert np.allclose(P.T @ P, np.eye(st["nc"]), atol=1e-15, rtol=0)
    assert np.allclose(P @ st["wc"], w, atol=1e-15, rtol=0)
    Ac = W.CSR(st["nc"], st["row_ptr"], st["col"], st["val"])
    dense = A.scipy().toarray()
    ref = P.T @ dense @ P
    got = Ac.scipy().toarray()
    assert np.max(np.abs(got - ref)) <= 1e-14
    assert oracle.validate(Ac) == oracle.OK      # includes bitwise symmetry
    # coarse stencil of x-pairs: diagonal 5, x-neighbour -1/2, y/z neighbours -1
    nx = N // 2
    I = 1 + nx * 2 + nx * N * 2        # an interior coarse point
    row = got[I]
    assert row[I] == pytest.approx(5.0, abs=4e-15)
    assert row[I - 1] == pytest.approx(-0.5, abs=4e-16) and row[I + 1] == pytest.approx(-0.5, abs=4e-16)
    for off in (nx, nx * N):
        assert row[I - off] == pytest.approx(-1.0, abs=1e-15)
        assert row[I + off] == pytest.approx(-1.0, abs=1e-15)


def test_two_steps_give_boxes_and_box_stencil():
    N = 8
    A = W.poisson7(N)
    H = oracle.Hierarchy(A, oracle.AMGParams(aggr_steps=2, coarse_max=10, max_levels=2))
    assert H.nlevels == 2
    L0 = H.level(0)
    idx = np.arange(A.n)
    x, y, z = idx % N, (idx // N) % N, idx // (N * N)
    box = (x // 2) + (N // 2) * (y // 2) + (N // 2) ** 2 * z
    # aggregate ids follow the box ids (numbered by smallest member, ascending)
    assert np.array_equal(L0["agg"], box)
    assert np.allclose(L0["pval"], 0.5, rtol=0, atol=1e-16)
    L1 = H.level(1)
    Ac = W.CSR(L1["n"], L1["row_ptr"], L1["col"], L1["val"]).scipy().toarray()
    m = N // 2
    I = 1 + m * 1 + m * m * 3
    assert Ac[I, I] == pytest.approx(4.0, abs=1e-14)
    for off, v in ((1, -0.5), (m, -0.5), (m * m, -1.0)):
        assert Ac[I, I - off] == pytest.approx(v, abs=1e-14)
        assert Ac[I, I + off] == pytest.approx(v, abs=1e-14)
    # composite P against the dense product of the two pairwise prolongators
    s1 = oracle.pairwise_step(A, np.ones(A.n))
    A1 = W.CSR(s1["nc"], s1["row_ptr"], s1["col"], s1["val"])
    s2 = oracle.pairwise_step(A1, s1["wc"])
    Pbar = _dense_P(A.n, s1["nc"], s1["agg"], s1["pval"]) @ _dense_P(s1["nc"], s2["nc"], s2["agg"], s2["pval"])
    assert np.allclose(_dense_P(A.n, L1["n"], L0["agg"], L0["pval"]), Pbar, atol=1e-16, rtol=0)
    assert np.allclose(Ac, Pbar.T @ A.scipy().toarray() @ Pbar, atol=1e-13, rtol=0)


@pytest.mark.parametrize("maker", ["diffusion27", "lognormal7", "hubs"])
def test_galerkin_dense_variable_coefficients(maker):
    if maker == "diffusion27":
        A = W.diffusion27(5, 3)
    elif maker == "lognormal7":
        A = W.lognormal7(6, 7, ell=2.0)
    else:   # two long rows (108 and 72 entries) on a 7-point grid
        A = W.with_hubs(W.poisson7(6), [(10, 2), (150, 3)])
        assert np.diff(A.row_ptr).max() >= 100
        S = A.scipy()
        assert abs(S - S.T).max() == 0.0
        d = S.diagonal()
        assert np.all(d >= np.asarray(abs(S).sum(axis=1)).ravel() - d - 1e-12)
    H = oracle.Hierarchy(A, oracle.AMGParams(aggr_steps=2, coarse_max=8, smooth_vec=1,
                                             smooth_sweeps=5))
    assert H.nlevels >= 3
    for k in range(H.nlevels - 1):
        Lk, Lk1 = H.level(k), H.level(k + 1)
        Ak = W.CSR(Lk["n"], Lk["row_ptr"], Lk["col"], Lk["val"])
        Ak1 = W.CSR(Lk1["n"], Lk1["row_ptr"], Lk1["col"], Lk1["val"])
        assert oracle.validate(Ak1) == oracle.OK
        P = _dense_P(Lk["n"], Lk1["n"], Lk["agg"], Lk["pval"])
        ref = P.T @ Ak.scipy().toarray() @ P
        assert np.max(np.abs(Ak1.scipy().toarray() - ref)) <= 1e-13 * np.max(np.abs(ref))
        assert np.allclose(P.T @ P, np.eye(Lk1["n"]), atol=1e-14, rtol=0)
        assert np.allclose(P @ Lk1["w"], Lk["w"], atol=1e-14, rtol=0)
        assert np.bincount(Lk["agg"]).max() <= 4
