"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Bars (stated per test):
  * setup: aggregate maps, coarse sparsity patterns, coarse values, P values,
    smooth vectors and l1 diagonals bit-exact on every level;
  * SpMV and sweeps: bit-exact (both sides fold each row in CSR order);
  * V-cycle output: relative max error <= 1e-12 (bit-exact expected);
  * PCG: iteration count within +-1 and relative residual <= rtol.
Inputs are the seeded generators of ``workloads``; sizes span several tiles
with ragged tails (odd grid edges, slices not multiple of 64 rows).
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
    "poisson32": (lambda: W.poisson7(32), {}),
    "poisson33_ragged": (lambda: W.poisson7(33), {}),
    "poisson17_s3_jacobi": (lambda: W.poisson7(17), dict(aggr_steps=3, coarse_max=40 * 17,
                                                          coarse_solver=1, coarse_sweeps=20)),
    "diffusion27_14_relax": (lambda: W.diffusion27(14, 3), dict(smooth_vec=1, smooth_sweeps=20)),
    "lognormal7_20_relax": (lambda: W.lognormal7(20, 7, ell=4.0), dict(smooth_vec=1, smooth_sweeps=20)),
    "poisson16_pre1_post2": (lambda: W.poisson7(16), dict(pre_sweeps=1, post_sweeps=2, aggr_steps=1)),
    "poisson12_maxlev2": (lambda: W.poisson7(12), dict(max_levels=2)),
    # coarsest level of 2000 rows: above the direct-solve limit, so solved by
    # sweeps (in binary64 also inside the binary32 cycle)
    "poisson20_maxlev2": (lambda: W.poisson7(20), dict(max_levels=2)),
    "poisson4_single_level": (lambda: W.poisson7(4), {}),
    "poisson1_n1": (lambda: W.poisson7(1), {}),
    # rows past 70304 shuffled: slot groups spanning more than 16 bits of
    # column offsets next to compact ones
    "poisson52_halfperm": (lambda: W.permute_tail(W.poisson7(52), 9, 52 ** 3 // 2), {}),
    # long rows: coarse rows of more than 512 Galerkin terms (one-thread
    # sort), of 17..512 (wavefront sort) and of at most 16 (registers)
    "poisson12_hubs": (lambda: W.with_hubs(W.poisson7(12), [(100, 2), (900, 5), (1500, 13)]), {}),
}


@pytest.mark.parametrize("case", list(CASES))
def test_setup_bit_exact(case):
    make, params = CASES[case]
    A = make()
    say("setup parity", case, "n=%d nnz=%d" % (A.n, A.nnz), params)
    Ho = oracle.Hierarchy(A, oracle_params(**params))
    Hg = gpu_hierarchy(A, **params)
    inf = assert_same_hierarchy(Hg, Ho)
    assert abs(inf["opc"] - Ho.opc()) <= 1e-15 * Ho.opc()
    assert inf["coarse_dense"] == Ho.coarse_dense


@pytest.mark.parametrize("case", ["poisson33_ragged", "diffusion27_14_relax", "lognormal7_20_relax",
                                  "poisson52_halfperm"])
def test_spmv_and_sweep_bit_exact_every_level(case):
    make, params = CASES[case]
    A = make()
    Ho = oracle.Hierarchy(A, oracle_params(**params))
    Hg = gpu_hierarchy(A, **params)
    for k in range(Ho.nlevels):
        lv = Ho.level(k)
        Ak = W.CSR(lv["n"], lv["row_ptr"], lv["col"], lv["val"])
        x = W.uniform_pm1(100 + k, Ak.n)
        r = W.uniform_pm1(200 + k, Ak.n)
        say("spmv/sweep parity", case, "level", k, "n", Ak.n)
        y = torch.empty(Ak.n, dtype=torch.float64, device="cuda")
        Hg.spmv(k, dev(x), y)
        assert np.array_equal(bits(host(y)), bits(oracle.spmv(Ak, x)))
        xn = torch.empty_like(y)
        Hg.sweep(k, dev(r), dev(x), xn)
        ref = x + lv["dinv"] * (r - oracle.spmv(Ak, x))
        assert np.array_equal(bits(host(xn)), bits(ref))


@pytest.mark.parametrize("case", [c for c in CASES if c != "poisson1_n1"])
def test_vcycle_matches_oracle(case):
    make, params = CASES[case]
    A = make()
    say("vcycle parity", case)
    Ho = oracle.Hierarchy(A, oracle_params(**params))
    Hg = gpu_hierarchy(A, **params)
    r = W.uniform_pm1(77, A.n)
    zo = Ho.vcycle(r)
    z = torch.empty(A.n, dtype=torch.float64, device="cuda")
    Hg.vcycle(dev(r), z)
    zg = host(z)
    err = np.max(np.abs(zg - zo)) / np.max(np.abs(zo))
    say("  max rel err", err, "bitwise", np.array_equal(bits(zg), bits(zo)))
    assert err <= 1e-12


@pytest.mark.parametrize("case", [c for c in CASES if c != "poisson1_n1"])
def test_pcg_matches_oracle(case):
    make, params = CASES[case]
    A = make()
    xs, b = W.manufactured_rhs(A, 1)
    say("pcg parity", case)
    Ho = oracle.Hierarchy(A, oracle_params(**params))
    xo, ito, relo, sto = Ho.pcg(b, rtol=1e-6)
    Hg = gpu_hierarchy(A, **params)
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    st, it, rel = Hg.solve(dev(b), x, rtol=1e-6)
    say("  oracle its %d rel %.3e | gpu its %d rel %.3e" % (ito, relo, it, rel))
    assert sto == 0 and st == 0
    assert abs(it - ito) <= 1
    assert rel <= 1e-6
    xg = host(x)
    true_rel = np.linalg.norm(b - A.scipy() @ xg) / np.linalg.norm(b)
    assert true_rel <= 1e-6 * 1.01
    assert np.linalg.norm(xg - xo) <= 1e-5 * np.linalg.norm(xo)


def test_plain_cg_identity_preconditioner():
    A = W.poisson7(12)
    xs, b = W.manufactured_rhs(A, 3)
    Ho = oracle.Hierarchy(A, oracle.AMGParams(precond=0))
    xo, ito, relo, sto = Ho.pcg(b, rtol=1e-8)
    Hg = gpu_hierarchy(A, precond=0)
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    st, it, rel = Hg.solve(dev(b), x, rtol=1e-8)
    assert st == 0 and abs(it - ito) <= 1 and rel <= 1e-8


def test_nonzero_initial_guess_and_zero_rhs():
    A = W.poisson7(16)
    xs, b = W.manufactured_rhs(A, 5)
    Hg = gpu_hierarchy(A)
    x0 = W.uniform_pm1(9, A.n)
    Ho = oracle.Hierarchy(A)
    xo, ito, relo, sto = Ho.pcg(b, x0=x0)
    x = dev(x0)
    st, it, rel = Hg.solve(dev(b), x)
    assert st == 0 and abs(it - ito) <= 1
    z = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    st, it, rel = Hg.solve(torch.zeros_like(z), z)
    assert st == 0 and it == 0 and rel == 0.0


def test_repeat_solves_are_bitwise_identical():
    A = W.poisson7(24)
    xs, b = W.manufactured_rhs(A, 2)
    Hg = gpu_hierarchy(A)
    outs = []
    for _ in range(3):
        x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
        st, it, rel = Hg.solve(dev(b), x)
        outs.append((it, rel, bits(host(x))))
    for o in outs[1:]:
        assert o[0] == outs[0][0] and o[1] == outs[0][1] and np.array_equal(o[2], outs[0][2])
    H2 = gpu_hierarchy(A)
    assert_same_hierarchy(H2, oracle.Hierarchy(A))


def test_maxit_and_error_codes():
    import paper_2303_02352_amd as amd
    A = W.poisson7(10)
    xs, b = W.manufactured_rhs(A, 1)
    Hg = gpu_hierarchy(A)
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    st, it, rel = Hg.solve(dev(b), x, rtol=1e-30, maxit=3, check=False)
    assert st == amd.AMG_NOT_CONVERGED and it == 3
    bb = b.copy()
    bb[5] = np.nan
    st, it, rel = Hg.solve(dev(bb), torch.zeros_like(x), check=False)
    assert st == amd.AMG_ERR_NONFINITE
    # malformed / unsymmetric / non-SPD inputs are rejected by amg_setup
    bad = W.CSR(A.n, A.row_ptr.copy(), A.col.copy(), A.val.copy())
    bad.col[[0, 1]] = bad.col[[1, 0]]
    with pytest.raises(amd.AMGError) as e:
        gpu_hierarchy(bad)
    assert e.value.code == amd.AMG_ERR_INVALID
    bad = W.CSR(A.n, A.row_ptr.copy(), A.col.copy(), A.val.copy())
    bad.val[1] = -0.5
    with pytest.raises(amd.AMGError) as e:
        gpu_hierarchy(bad)
    assert e.value.code == amd.AMG_ERR_INVALID
    bad = W.CSR(A.n, A.row_ptr.copy(), A.col.copy(), A.val.copy())
    bad.val[0] = -6.0
    with pytest.raises(amd.AMGError) as e:
        gpu_hierarchy(bad)
    assert e.value.code == amd.AMG_ERR_NOT_SPD
    bad = W.CSR(A.n, A.row_ptr.copy(), A.col.copy(), A.val.copy())
    bad.val[2] = np.inf
    with pytest.raises(amd.AMGError) as e:
        gpu_hierarchy(bad)
    assert e.value.code == amd.AMG_ERR_NONFINITE
    # indefinite single-level system: non-positive Cholesky pivot
    import scipy.sparse as sp
    D = np.array([[1.0, 2.0, 0, 0], [2.0, 1.0, 0, 0], [0, 0, 1.0, 0], [0, 0, 0, 1.0]])
    S = sp.csr_matrix(D)
    Ai = W.CSR(4, S.indptr.astype(np.int32), S.indices.astype(np.int32), S.data.copy())
    with pytest.raises(amd.AMGError) as e:
        gpu_hierarchy(Ai)
    assert e.value.code == amd.AMG_ERR_NOT_SPD
    Hn = gpu_hierarchy(Ai, precond=0)
    st, it, rel = Hn.solve(dev(np.array([1.0, -1.0, 0.0, 0.0])), torch.zeros(4, dtype=torch.float64,
                                                                            device="cuda"), check=False)
    assert st == amd.AMG_ERR_NOT_SPD


def test_host_csr_input_equals_device_input():
    import paper_2303_02352_amd as amd
    A = W.poisson7(20)
    Hd = gpu_hierarchy(A)
    Hh = amd.Hierarchy(A.row_ptr, A.col, A.val)
    for k in range(Hd.info()["levels"]):
        a, b = Hd.export_level(k), Hh.export_level(k)
        assert np.array_equal(bits(a["val"]), bits(b["val"]))


MIXED_CASES = ["poisson32", "poisson33_ragged", "diffusion27_14_relax", "lognormal7_20_relax",
               "poisson17_s3_jacobi", "poisson20_maxlev2"]


@pytest.mark.parametrize("case", MIXED_CASES)
def test_mixed_precision_vcycle_and_pcg(case):
    """Mixed form: binary32 V-cycle, binary64 PCG.  The GPU cycle is compared
    with the oracle's binary32 cycle (relative 1e-6, bit-exact expected) and
    its distance to the binary64 cycle is reported; PCG reaches the same rtol
    with the oracle's mixed iteration count +-1."""
    import paper_2303_02352_amd as amd
    make, params = CASES[case]
    A = make()
    say("mixed parity", case)
    Ho = oracle.Hierarchy(A, oracle_params(**params))
    Hg = gpu_hierarchy(A, precision=amd.AMG_PREC_MIXED, **params)
    assert_same_hierarchy(Hg, Ho)        # setup stays binary64
    r = W.uniform_pm1(78, A.n)
    z = torch.empty(A.n, dtype=torch.float64, device="cuda")
    Hg.vcycle(dev(r), z)
    zg = host(z)
    z32 = Ho.vcycle_f32(r)
    z64 = Ho.vcycle(r)
    err32 = np.max(np.abs(zg - z32)) / np.max(np.abs(z32))
    err64 = np.max(np.abs(zg - z64)) / np.max(np.abs(z64))
    say("  vs oracle binary32 %.2e (bitwise %s), vs binary64 %.2e" %
        (err32, np.array_equal(bits(zg), bits(z32)), err64))
    assert err32 <= 1e-6
    assert err64 <= 1e-5
    xs, b = W.manufactured_rhs(A, 1)
    xo, ito, relo, sto = Ho.pcg(b, mixed=True)
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    st, it, rel = Hg.solve(dev(b), x)
    say("  pcg oracle-mixed its %d | gpu-mixed its %d rel %.2e" % (ito, it, rel))
    assert st == 0 and sto == 0 and abs(it - ito) <= 1 and rel <= 1e-6
    xg = host(x)
    assert np.linalg.norm(b - A.scipy() @ xg) / np.linalg.norm(b) <= 1e-6 * 1.01


def test_time_kernel_ids_and_byte_model():
    """amg_time_kernel: every kernel id runs on a level that has it, reports a
    positive duration, and its algorithmic bytes follow the stated model
    (sweep: the matrix in its compact form plus three vectors)."""
    import paper_2303_02352_amd as amd
    A = W.poisson7(24)
    Hg = gpu_hierarchy(A)
    for kid in (amd.KERNEL_SPMV, amd.KERNEL_SWEEP, amd.KERNEL_RESTRICT, amd.KERNEL_PROLONG,
                amd.KERNEL_UPDATE, amd.KERNEL_CORR_SWEEP):
        ms, by = Hg.time_kernel(kid, 0, 3)
        say("  kernel", kid, "ms %.4f bytes %.0f" % (ms, by))
        assert ms > 0 and by > 0
    nnz, n = A.nnz, A.n
    nslices = -(-n // 64)
    # n = 13824 < 65536: every slice is compact (2-byte offsets + one base per
    # 64 slots); values plain (8 bytes) or coded (1 byte + the table: the
    # 7-point matrix holds 6, -1 and the padding 0)
    assert Hg.info()["dict_size"][0] == 3
    ms, sweep_bytes = Hg.time_kernel(amd.KERNEL_SWEEP, 0, 1)
    lo = 1 * nnz + 8 * 3 + 2 * nnz + 24 * n
    assert lo < sweep_bytes <= lo + 4 * 7 * nslices + 4 * (nslices + 1)
    Hp = gpu_hierarchy(A, value_coding=amd.AMG_VALUES_PLAIN)
    assert Hp.info()["dict_size"][0] == 0
    ms, sweep_bytes = Hp.time_kernel(amd.KERNEL_SWEEP, 0, 1)
    lo = 8 * nnz + 2 * nnz + 24 * n
    assert lo < sweep_bytes <= lo + 4 * 7 * nslices + 4 * (nslices + 1)
    for bad in (-1, 6):
        with pytest.raises(amd.AMGError):
            Hg.time_kernel(bad, 0, 1)
    last = Hg.info()["levels"] - 1
    with pytest.raises(amd.AMGError):
        Hg.time_kernel(amd.KERNEL_CORR_SWEEP, last, 1)


@pytest.mark.parametrize("case", ["poisson33_ragged", "lognormal7_20_relax", "poisson12_hubs"])
@pytest.mark.parametrize("precision", [0, 1])
def test_coded_values_equal_plain_values(case, precision):
    """Levels whose values take at most 256 bit patterns are read as one-byte
    codes into a table: V-cycle and PCG give the same bits as the plain
    value arrays, and the table holds exactly the distinct values (padding
    zero included) of the level."""
    import paper_2303_02352_amd as amd
    make, params = CASES[case]
    A = make()
    say("coded vs plain values", case, "precision", precision)
    Hc = gpu_hierarchy(A, precision=precision, **params)
    Hp = gpu_hierarchy(A, precision=precision, value_coding=amd.AMG_VALUES_PLAIN, **params)
    ic, ip = Hc.info(), Hp.info()
    assert ip["dict_size"] == [0] * ip["levels"]
    for k in range(ic["levels"]):
        vals = Hc.export_level(k)["val"]
        distinct = np.unique(bits(np.concatenate((vals, [0.0])))).size
        # the padding zero is present unless every slice is exactly full
        assert ic["dict_size"][k] in ((distinct, distinct - 1) if distinct <= 256 else (0,))
    if case.startswith("poisson"):
        assert ic["dict_size"][0] > 0
    else:
        assert ic["dict_size"][0] == 0
    r = dev(W.uniform_pm1(31, A.n))
    z = [torch.empty(A.n, dtype=torch.float64, device="cuda") for _ in range(2)]
    Hc.vcycle(r, z[0])
    Hp.vcycle(r, z[1])
    assert np.array_equal(bits(host(z[0])), bits(host(z[1])))
    xs, b = W.manufactured_rhs(A, 2)
    outs = []
    for H in (Hc, Hp):
        x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
        st, it, rel = H.solve(dev(b), x)
        outs.append((st, it, rel, host(x)))
    assert outs[0][:3] == outs[1][:3]
    assert np.array_equal(bits(outs[0][3]), bits(outs[1][3]))


def _k_valued(N, K):
    """7-point pattern on N^3 with K distinct off-diagonal values
    -(0.5 + 0.5 ((i + j) mod K) / K) (symmetric), diagonal 6.5: diagonally
    dominant, and K + 1 distinct stored values (K + 2 slot values with the
    padding zero of the boundary rows)."""
    A = W.poisson7(N)
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    off = rows != A.col
    val = np.full(A.nnz, 6.5)
    val[off] = -(0.5 + 0.5 * ((rows[off] + A.col[off]) % K) / K)
    return W.CSR(A.n, A.row_ptr, A.col, val)


@pytest.mark.parametrize("K,table", [(62, 64), (63, 65), (254, 256), (255, 0)])
@pytest.mark.parametrize("precision", [0, 1])
def test_value_table_limit(K, table, precision):
    """A level with exactly 256 distinct slot values is coded, one with 257
    is not; tables of 64 and 65 entries sit on either side of the switch
    from one register per lane to a copied table.  Every case gives the
    plain path's bits and the oracle's V-cycle (binary64 within 1e-12, the
    binary32 cycle within 1e-6)."""
    import paper_2303_02352_amd as amd
    A = _k_valued(12, K)
    say("value table limit K=%d precision %d" % (K, precision))
    Hc = gpu_hierarchy(A, precision=precision)
    assert Hc.info()["dict_size"][0] == table
    Hp = gpu_hierarchy(A, precision=precision, value_coding=amd.AMG_VALUES_PLAIN)
    Ho = oracle.Hierarchy(A, oracle_params())
    r = W.uniform_pm1(5, A.n)
    zo = Ho.vcycle(r) if precision == 0 else Ho.vcycle_f32(r)
    z = [torch.empty(A.n, dtype=torch.float64, device="cuda") for _ in range(2)]
    Hc.vcycle(dev(r), z[0])
    Hp.vcycle(dev(r), z[1])
    assert np.array_equal(bits(host(z[0])), bits(host(z[1])))
    tol = 1e-12 if precision == 0 else 1e-6
    assert np.max(np.abs(host(z[0]) - zo)) <= tol * np.max(np.abs(zo))


def test_caller_stream_gives_the_same_bits():
    """A hierarchy and a batch built and used on a stream of the caller's
    (amg_params.stream) give the bits of the library-stream runs."""
    import paper_2303_02352_amd as amd
    A = W.poisson7(20)
    xs, b = W.manufactured_rhs(A, 4)
    r = W.uniform_pm1(12, A.n)
    systems = [W.poisson7(N) for N in (9, 6)]
    nr = 4
    Bh = W.uniform_pm1(13, sum(S.n for S in systems) * nr)

    def run():
        out = []
        for prec in (amd.AMG_PREC_DOUBLE, amd.AMG_PREC_MIXED):
            H = gpu_hierarchy(A, precision=prec)
            z = torch.empty(A.n, dtype=torch.float64, device="cuda")
            H.vcycle(dev(r), z)
            x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
            st, it, rel = H.solve(dev(b), x)
            out += [bits(host(z)), bits(host(x)), (st, it)]
            H.close()
        bt = amd.Batch([(dev(S.row_ptr), dev(S.col), dev(S.val)) for S in systems])
        X = torch.zeros(Bh.size, dtype=torch.float64, device="cuda")
        st, its, rel, pst = bt.solve(dev(Bh), X, nr)
        out += [bits(host(X)), its.tolist()]
        bt.close()
        return out

    ref = run()                       # torch's default stream: the library's own stream
    s = torch.cuda.Stream()           # default priority
    with torch.cuda.stream(s):
        got = run()
        s.synchronize()
    for a, c in zip(ref, got):
        assert np.array_equal(np.asarray(a), np.asarray(c))


def test_hierarchies_on_concurrent_host_threads():
    """Different hierarchies and batches may be built and solved from
    different host threads at the same time (one thread per object): each
    thread gets the bits a sequential run gives."""
    from concurrent.futures import ThreadPoolExecutor
    import paper_2303_02352_amd as amd
    mats = [W.poisson7(22), W.diffusion27(12, 3), W.poisson7(19), W.lognormal7(14, 5, ell=3.0)]

    def work(i):
        A = mats[i]
        xs, b = W.manufactured_rhs(A, 20 + i)
        H = amd.Hierarchy(A.row_ptr, A.col, A.val, precision=i % 2)   # host CSR: library stream
        out = []
        for _ in range(3):
            x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
            st, it, rel = H.solve(torch.from_numpy(b).cuda(), x)
            torch.cuda.current_stream().synchronize()
            out.append((st, it, bits(x.cpu().numpy())))
        H.close()
        if i % 2:   # a batch too: its solve captures a graph of its own
            systems = [W.poisson7(N) for N in (6 + i, 5)]
            bt = amd.Batch([(S.row_ptr, S.col, S.val) for S in systems])
            nr = 2
            Bb = torch.from_numpy(W.uniform_pm1(40 + i, sum(S.n for S in systems) * nr)).cuda()
            X = torch.zeros_like(Bb)
            st, its, rel, pst = bt.solve(Bb, X, nr)
            torch.cuda.current_stream().synchronize()
            out.append((st, int(its.sum()), bits(X.cpu().numpy())))
            bt.close()
        return out

    ref = [work(i) for i in range(len(mats))]
    with ThreadPoolExecutor(len(mats)) as ex:
        got = list(ex.map(work, range(len(mats))))
    for r, g in zip(ref, got):
        for (s0, i0, x0), (s1, i1, x1) in zip(r, g):
            assert s0 == s1 == 0 and i0 == i1 and np.array_equal(x0, x1)


def test_repeated_setup_and_destroy_hold_memory_steady():
    """Hierarchies and batches built, used and destroyed in a loop: after the
    first cycle (the pool's steady state) the device's free memory does not
    shrink, and every hierarchy reports the same device footprint."""
    import paper_2303_02352_amd as amd
    A = W.poisson7(24)
    xs, b = W.manufactured_rhs(A, 3)
    bd = dev(b)
    systems = [W.poisson7(N) for N in (7, 5)]

    def cycle():
        sizes = []
        for prec in (amd.AMG_PREC_DOUBLE, amd.AMG_PREC_MIXED):
            H = gpu_hierarchy(A, precision=prec)
            x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
            st, it, rel = H.solve(bd, x)
            assert st == 0
            sizes.append(H.info()["device_bytes"])
            H.close()
        bt = amd.Batch([(dev(S.row_ptr), dev(S.col), dev(S.val)) for S in systems])
        X = torch.zeros(sum(S.n for S in systems) * 4, dtype=torch.float64, device="cuda")
        st, its, rel, pst = bt.solve(torch.ones_like(X), X, 4)
        assert st == 0
        bt.close()
        torch.cuda.synchronize()
        return sizes

    first = cycle()
    free0 = torch.cuda.mem_get_info()[0]
    for _ in range(30):
        assert cycle() == first
    free1 = torch.cuda.mem_get_info()[0]
    say("free device memory after 1 / 31 cycles: %d / %d MiB" % (free0 >> 20, free1 >> 20))
    assert free1 >= free0 - (64 << 20)


def test_slot_count_limit_is_refused():
    """The first row of every slice is a hub coupled to all other hubs (a
    dense, diagonally dominant block); the other rows are the identity.  nnz
    stays far below 2^31, but the SELL form would need 5793 slices x 64 x
    5793 slots >= 2^31, past the int32 slot offsets: amg_setup must refuse it
    (AMG_ERR_UNSUPPORTED) before any slot is written, and leave no hierarchy."""
    import paper_2303_02352_amd as amd
    S, eps = 5793, 1e-3
    n = 64 * S
    hubs = np.arange(S, dtype=np.int64) * 64
    lens = np.ones(n, dtype=np.int64)
    lens[hubs] = S
    rp = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(lens, out=rp[1:])
    col = np.arange(n, dtype=np.int32)[np.repeat(np.arange(n), lens)]     # the diagonal of plain rows
    val = np.ones(rp[-1])
    at = (rp[hubs][:, None] + np.arange(S)[None, :]).reshape(-1)
    col[at] = np.tile(hubs.astype(np.int32), S)
    val[at] = -eps
    val[rp[hubs] + np.arange(S)] = 1.0 + (S - 1) * eps                    # hub k's diagonal is its k-th entry
    A = W.CSR(n, rp.astype(np.int32), col, val)
    say("slot limit: n=%d nnz=%d" % (A.n, A.nnz))
    assert A.nnz < 2 ** 26 and S * 64 * S >= 2 ** 31
    with pytest.raises(amd.AMGError) as e:
        gpu_hierarchy(A)
    assert e.value.code == amd.AMG_ERR_UNSUPPORTED
