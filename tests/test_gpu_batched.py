"""GPU parity of the batched form (many systems x several right-hand sides).

Every (system, right-hand side) pair must behave as its own single-system
solve: the batched V-cycle column equals the oracle's V-cycle of that system
(binary64: <= 1e-12 relative; the coarsest block product runs on the FP64
matrix cores, whose sums round in their own order, so the columns agree to
the binary64 unit rather than bit for bit; mixed: against the oracle's
binary32 cycle, <= 1e-6), and the batched PCG reaches rtol with the oracle's
iteration count +-1 for every pair.  The batch mixes grid edges so that
systems have different depths, one system is a single level, and one edge is
odd (ragged slices).
"""
import numpy as np
import pytest

import oracle
import workloads as W

from gpu_helpers import bits, dev, host, require_gpu, say, torch

pytestmark = pytest.mark.gpu

EDGES = [8, 12, 5, 10, 4, 7, 9]


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def _stack(blocks):
    return np.ascontiguousarray(np.concatenate([b.reshape(-1) for b in blocks]))


def _batch(systems, **params):
    import paper_2303_02352_amd as amd
    return amd.Batch([(dev(A.row_ptr), dev(A.col), dev(A.val)) for A in systems], **params)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("nrhs", [2, 4, 8, 16])
def test_batched_vcycle_matches_oracle(nrhs, precision):
    systems = [W.poisson7(N) for N in EDGES]
    say("batched vcycle", nrhs, precision)
    bt = _batch(systems, precision=precision)
    R = [W.uniform_pm1(900 + s, A.n * nrhs).reshape(A.n, nrhs) for s, A in enumerate(systems)]
    Z = torch.zeros(sum(A.n for A in systems) * nrhs, dtype=torch.float64, device="cuda")
    bt.vcycle(dev(_stack(R)), Z, nrhs)
    Zh = host(Z)
    off = 0
    worst = 0.0
    for s, A in enumerate(systems):
        Ho = oracle.Hierarchy(A)
        blk = Zh[off:off + A.n * nrhs].reshape(A.n, nrhs)
        off += A.n * nrhs
        for c in range(nrhs):
            ref = Ho.vcycle_f32(R[s][:, c]) if precision == 1 else Ho.vcycle(R[s][:, c])
            err = np.max(np.abs(blk[:, c] - ref)) / np.max(np.abs(ref))
            worst = max(worst, err)
            assert err <= (1e-6 if precision == 1 else 1e-12), (s, c, err)
    say("  worst rel err %.2e" % worst)
    inf = bt.info()
    # the autotuner's pick is timing-dependent: any width that divides nrhs
    for k in range(inf["levels"]):
        if inf["n_smoothed"][k] > 0:
            for cpl in (inf["cols_per_lane"][k], inf["cols_per_lane_corr"][k]):
                assert cpl in (1, 2, 4, 8, 16) and nrhs % cpl == 0
    assert inf["tile_rows"] in (128, 256, 512, 1024)
    assert inf["spmm_cols"] in (1, 2, 4) and nrhs % inf["spmm_cols"] == 0


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("nrhs", [1, 16])
def test_batched_pcg_matches_oracle(nrhs, precision):
    systems = [W.poisson7(N) for N in EDGES]
    say("batched pcg", nrhs, precision)
    bt = _batch(systems, precision=precision)
    xs = [W.batched_rhs(s, A.n, nrhs).T for s, A in enumerate(systems)]        # (n, nrhs)
    bs = [np.ascontiguousarray((A.scipy() @ x)) for A, x in zip(systems, xs)]
    X = torch.zeros(sum(A.n for A in systems) * nrhs, dtype=torch.float64, device="cuda")
    st, its, rel, pst = bt.solve(dev(_stack(bs)), X, nrhs, rtol=1e-6)
    assert st == 0 and np.all(pst == 0)
    Xh = host(X)
    off = 0
    for s, A in enumerate(systems):
        Ho = oracle.Hierarchy(A)
        blk = Xh[off:off + A.n * nrhs].reshape(A.n, nrhs)
        off += A.n * nrhs
        for c in range(nrhs):
            xo, ito, relo, sto = Ho.pcg(bs[s][:, c], mixed=(precision == 1))
            assert abs(int(its[s, c]) - ito) <= 1, (s, c, its[s, c], ito)
            assert rel[s, c] <= 1e-6
            tr = np.linalg.norm(bs[s][:, c] - A.scipy() @ blk[:, c]) / np.linalg.norm(bs[s][:, c])
            assert tr <= 1e-6 * 1.01
    say("  iterations per system (col 0):", list(its[:, 0]))


def test_batched_masks_keep_converged_pairs_frozen():
    """A zero right-hand side converges at once (0 iterations) while the other
    columns keep iterating; repeated solves are bitwise identical."""
    systems = [W.poisson7(N) for N in (9, 6)]
    bt = _batch(systems)
    nrhs = 4
    bs = []
    for s, A in enumerate(systems):
        x = W.batched_rhs(s, A.n, nrhs).T.copy()
        x[:, 2] = 0.0
        bs.append(np.ascontiguousarray(A.scipy() @ x))
    outs = []
    for _ in range(2):
        X = torch.zeros(sum(A.n for A in systems) * nrhs, dtype=torch.float64, device="cuda")
        st, its, rel, pst = bt.solve(dev(_stack(bs)), X, nrhs)
        outs.append((its.copy(), bits(host(X))))
        assert st == 0 and np.all(its[:, 2] == 0) and np.all(its[:, [0, 1, 3]] > 0)
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def test_batched_solve_with_one_vector_per_system():
    """amg_batch_solve_systems (B[s], X[s] apart) gives the bits of amg_batch_solve
    on the stacked block, with initial guesses taken from X[s]."""
    systems = [W.poisson7(N) for N in (9, 6, 5)]
    bt = _batch(systems, precision=1)
    nrhs = 8
    bs = [np.ascontiguousarray(A.scipy() @ W.batched_rhs(s, A.n, nrhs).T) for s, A in enumerate(systems)]
    x0 = [0.1 * W.uniform_pm1(30 + s, A.n * nrhs) for s, A in enumerate(systems)]
    X = dev(_stack(x0))
    st, its, rel, pst = bt.solve(dev(_stack(bs)), X, nrhs)
    Xs = [dev(x) for x in x0]
    st2, its2, rel2, pst2 = bt.solve_systems([dev(b) for b in bs], Xs, nrhs)
    say("  stacked %s, per system %s" % (its.max(), its2.max()))
    assert st == st2 == 0
    assert np.array_equal(its, its2) and np.array_equal(rel, rel2) and np.array_equal(pst, pst2)
    assert np.array_equal(bits(host(X)), bits(np.concatenate([host(x) for x in Xs])))


def test_batched_errors():
    import paper_2303_02352_amd as amd
    systems = [W.poisson7(N) for N in (6, 5)]
    bt = _batch(systems)
    X = torch.zeros(sum(A.n for A in systems) * 3, dtype=torch.float64, device="cuda")
    st, its, rel, pst = bt.solve(X.clone(), X, 3, check=False)
    assert st == amd.AMG_ERR_UNSUPPORTED
    X2 = X[:sum(A.n for A in systems) * 2].contiguous()
    st, its, rel, pst = bt.solve(torch.zeros_like(X2), X2, 2)       # zero right-hand sides
    assert st == 0 and np.all(its == 0) and np.all(rel == 0.0)
    b = torch.from_numpy(W.uniform_pm1(5, X2.numel())).cuda()
    st, its, rel, pst = bt.solve(b, torch.zeros_like(X2), 2, rtol=1e-30, maxit=2, check=False)
    assert st == amd.AMG_NOT_CONVERGED and np.all(its == 2) and np.all(pst == amd.AMG_NOT_CONVERGED)
    with pytest.raises(amd.AMGError) as e:
        _batch(systems, coarse_solver=1)
    assert e.value.code == amd.AMG_ERR_UNSUPPORTED
