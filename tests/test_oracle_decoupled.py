"""Pins for the oracle's decoupled aggregation (Sec. 4.1), CPU only.

Every task owns a block of consecutive rows and runs the matching on the
subgraph of its own rows only; edges between blocks are ignored, so the
prolongator is block diagonal and a coarse row belongs to the block of its
aggregate.  Pins, none of which re-evaluates the oracle's own formulas:
  * the row blocks are the consecutive split with sizes differing by <= 1;
  * one block, or blocks aligned with the components of a disconnected
    matrix, change nothing (bit-identical hierarchy);
  * the decoupled matching equals the union of the plain matchings of the
    diagonal blocks taken as separate graphs (local row numbering);
  * aggregates never leave their block; coarse blocks are inherited and
    consecutive;
  * P is block diagonal and A_c equals the dense P^T A P;
  * closed form on 7-point Poisson 8^3, w = 1, s = 3: one block gives 2x2x2
    boxes, one block per z-plane gives 4x2x1 boxes (z couplings are cut, so
    the third step pairs boxes along x);
  * more blocks than rows: no pair is formed, one level, one PCG iteration;
  * the V-cycle stays symmetric and PCG reaches rtol.
"""
import numpy as np
import pytest

import oracle
import workloads as W


def _bits(a):
    return np.ascontiguousarray(a, np.float64).view(np.uint64)


def _same_hierarchy(H1, H2):
    assert H1.nlevels == H2.nlevels
    for k in range(H1.nlevels):
        a, b = H1.level(k), H2.level(k)
        assert a["n"] == b["n"] and a["nnz"] == b["nnz"], k
        assert np.array_equal(a["row_ptr"], b["row_ptr"]) and np.array_equal(a["col"], b["col"]), k
        assert np.array_equal(_bits(a["val"]), _bits(b["val"])), k
        assert np.array_equal(_bits(a["w"]), _bits(b["w"])), k
        if k < H1.nlevels - 1:
            assert np.array_equal(a["agg"], b["agg"]), k
            assert np.array_equal(_bits(a["pval"]), _bits(b["pval"])), k


@pytest.mark.parametrize("n,np_", [(10, 3), (7, 7), (5, 9), (1000, 64), (65, 2)])
def test_row_blocks_are_the_consecutive_split(n, np_):
    part = oracle.row_blocks(n, np_)
    assert np.all(np.diff(part) >= 0)
    for p in range(np_):
        rows = np.nonzero(part == p)[0]
        assert len(rows) in (n // np_, n // np_ + 1)
        if len(rows):
            assert rows[0] == (p * n) // np_
            assert np.array_equal(rows, np.arange(rows[0], rows[0] + len(rows)))


def test_one_block_changes_nothing():
    A = W.lognormal7(12, 3, ell=3.0)
    p = dict(smooth_vec=1, smooth_sweeps=5)
    _same_hierarchy(oracle.Hierarchy(A, oracle.AMGParams(**p)),
                    oracle.Hierarchy(A, oracle.AMGParams(n_parts=1, **p)))


def _block_diag(blocks):
    import scipy.sparse as sp
    S = sp.block_diag([b.scipy() for b in blocks], format="csr")
    S.sort_indices()
    return W.CSR(S.shape[0], S.indptr.astype(np.int32), S.indices.astype(np.int32), S.data.copy())


def test_blocks_aligned_with_components_change_nothing():
    """Four disconnected copies of a 6^3 log-normal operator, four row blocks
    exactly on the copies: no edge crosses a block, so decoupling is moot."""
    comps = [W.lognormal7(6, 10 + c, ell=2.0) for c in range(4)]
    A = _block_diag(comps)
    assert np.array_equal(oracle.row_blocks(A.n, 4), np.repeat(np.arange(4), comps[0].n))
    p = dict(smooth_vec=1, smooth_sweeps=4, coarse_max=20)
    _same_hierarchy(oracle.Hierarchy(A, oracle.AMGParams(**p)),
                    oracle.Hierarchy(A, oracle.AMGParams(n_parts=4, **p)))


def _submatrix(A, lo, hi):
    S = A.scipy()[lo:hi, lo:hi].tocsr()
    S.sort_indices()
    return W.CSR(hi - lo, S.indptr.astype(np.int32), S.indices.astype(np.int32), S.data.copy())


@pytest.mark.parametrize("np_", [2, 3, 7])
def test_decoupled_matching_is_union_of_local_matchings(np_):
    A = W.lognormal7(9, 5, ell=3.0)
    w = 0.5 + W.uniform(41, A.n)
    part = oracle.row_blocks(A.n, np_)
    got = oracle.pairwise_step(A, w, part)["mate"]
    want = np.full(A.n, -1, np.int32)
    for p in range(np_):
        rows = np.nonzero(part == p)[0]
        lo, hi = int(rows[0]), int(rows[-1]) + 1
        m = oracle.match_greedy(_submatrix(A, lo, hi), w[lo:hi])
        want[lo:hi] = np.where(m >= 0, m + lo, -1)
    assert np.array_equal(got, want)
    # and it differs from the coupled matching (some pair crossed a block)
    assert not np.array_equal(got, oracle.pairwise_step(A, w)["mate"])


def test_aggregates_stay_in_blocks_and_blocks_are_inherited():
    A = W.lognormal7(14, 8, ell=3.0)
    H = oracle.Hierarchy(A, oracle.AMGParams(n_parts=5, smooth_vec=1, smooth_sweeps=6, coarse_max=30))
    assert H.nlevels >= 3
    for k in range(H.nlevels):
        pk = H.part(k)
        assert np.all(np.diff(pk) >= 0) and pk.min() >= 0 and pk.max() <= 4
        if k < H.nlevels - 1:
            agg = H.level(k)["agg"]
            pc = H.part(k + 1)
            assert np.array_equal(pc[agg], pk), k
    assert np.array_equal(H.part(0), oracle.row_blocks(A.n, 5))


def test_block_diagonal_p_and_galerkin_product():
    A = W.lognormal7(5, 2, ell=2.0)
    H = oracle.Hierarchy(A, oracle.AMGParams(n_parts=3, aggr_steps=2, smooth_vec=1, smooth_sweeps=3,
                                             coarse_max=8))
    Ad = A.scipy().toarray()
    for k in range(H.nlevels - 1):
        lk, lc = H.level(k), H.level(k + 1)
        n, nc = lk["n"], lc["n"]
        P = np.zeros((n, nc))
        P[np.arange(n), lk["agg"]] = lk["pval"]
        pk, pc = H.part(k), H.part(k + 1)
        rr, cc = np.nonzero(P)
        assert np.all(pk[rr] == pc[cc]), k
        import scipy.sparse as sp
        Ak = sp.csr_matrix((lk["val"], lk["col"], lk["row_ptr"]), shape=(n, n)).toarray()
        Ac = sp.csr_matrix((lc["val"], lc["col"], lc["row_ptr"]), shape=(nc, nc)).toarray()
        ref = P.T @ Ak @ P
        assert np.max(np.abs(Ac - ref)) <= 1e-13 * np.max(np.abs(ref)), k
        if k == 0:
            assert np.array_equal(Ak, Ad)


def _boxes(N, bx, by, bz):
    z, y, x = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
    nx, ny = N // bx, N // by
    return ((x // bx) + nx * (y // by) + nx * ny * (z // bz)).reshape(-1).astype(np.int32)


def test_poisson_planes_closed_form():
    N = 8
    A = W.poisson7(N)
    one = oracle.Hierarchy(A, oracle.AMGParams(aggr_steps=3, coarse_max=1))
    assert np.array_equal(one.level(0)["agg"], _boxes(N, 2, 2, 2))
    planes = oracle.Hierarchy(A, oracle.AMGParams(aggr_steps=3, coarse_max=1, n_parts=N))
    assert np.array_equal(planes.level(0)["agg"], _boxes(N, 4, 2, 1))
    assert np.array_equal(planes.part(1), np.repeat(np.arange(N), (N // 4) * (N // 2)))


def test_more_blocks_than_rows():
    A = W.poisson7(3)
    H = oracle.Hierarchy(A, oracle.AMGParams(n_parts=64, coarse_max=1))
    assert H.nlevels == 1
    xs, b = W.manufactured_rhs(A, 2)
    x, it, rel, st = H.pcg(b, rtol=1e-10)
    assert st == oracle.OK and it == 1


@pytest.mark.parametrize("np_", [1, 4, 16])
def test_decoupled_vcycle_symmetric_and_pcg_converges(np_):
    A = W.poisson7(16)
    H = oracle.Hierarchy(A, oracle.AMGParams(n_parts=np_))
    x, y = W.uniform_pm1(3, A.n), W.uniform_pm1(4, A.n)
    bx, by = H.vcycle(x), H.vcycle(y)
    assert abs(bx @ y - x @ by) <= 1e-13 * abs(bx @ y)
    assert bx @ x > 0
    xs, b = W.manufactured_rhs(A, 5)
    u, it, rel, st = H.pcg(b, rtol=1e-6)
    assert st == oracle.OK and rel <= 1e-6
    true = np.linalg.norm(b - A.scipy() @ u) / np.linalg.norm(b)
    assert true <= 1.01e-6
