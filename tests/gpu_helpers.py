"""Shared helpers for the GPU tests (marshalling between numpy and torch)."""
import hashlib
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")


def require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")


def say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def gpu_hierarchy(A, **params):
    import paper_2303_02352_amd as amd
    return amd.Hierarchy(dev(A.row_ptr), dev(A.col), dev(A.val), **params)


def oracle_params(**kw):
    import oracle
    keep = {k: v for k, v in kw.items() if k in oracle.AMGParams.__dataclass_fields__}
    return oracle.AMGParams(**keep)


def bits(a):
    return np.ascontiguousarray(a, dtype=np.float64).view(np.uint64)


def assert_same_hierarchy(Hg, Ho):
    """Aggregate maps, coarse patterns and values, P values, smooth vectors,
    l1 diagonals: identical bit for bit on every level."""
    inf = Hg.info()
    assert inf["levels"] == Ho.nlevels, (inf["n"], Ho.sizes())
    for k in range(Ho.nlevels):
        g = Hg.export_level(k)
        o = Ho.level(k)
        assert g["n"] == o["n"] and g["nnz"] == o["nnz"], k
        assert np.array_equal(g["row_ptr"], o["row_ptr"]), k
        assert np.array_equal(g["col"], o["col"]), k
        assert np.array_equal(bits(g["val"]), bits(o["val"])), k
        assert np.array_equal(bits(g["dinv"]), bits(o["dinv"])), k
        assert np.array_equal(bits(g["w"]), bits(o["w"])), k
        if k < Ho.nlevels - 1:
            assert np.array_equal(g["agg"], o["agg"]), k
            assert np.array_equal(bits(g["pval"]), bits(o["pval"])), k
    return inf


def digest(a, dtype):
    """SHA-256 of the array's little-endian bytes as `dtype` (the digests the
    oracle's golden records hold)."""
    return hashlib.sha256(np.ascontiguousarray(a, dtype=np.dtype(dtype).newbyteorder("<")).tobytes()).hexdigest()


def assert_level_digests(Hg, recs):
    """Every level of the GPU hierarchy hashes to the oracle's stored digests
    (CSR arrays, l1 diagonal, smooth vector, aggregate map, P values)."""
    inf = Hg.info()
    assert inf["levels"] == len(recs), (inf["n"], len(recs))
    for k, rec in enumerate(recs):
        g = Hg.export_level(k)
        got = dict(row_ptr=digest(g["row_ptr"], np.int32), col=digest(g["col"], np.int32),
                   val=digest(g["val"], np.float64), dinv=digest(g["dinv"], np.float64),
                   w=digest(g["w"], np.float64))
        if g["agg"] is not None:
            got["agg"] = digest(g["agg"], np.int32)
            got["pval"] = digest(g["pval"], np.float64)
        bad = [f for f in rec if rec[f] != got.get(f)]
        say("  level %d (n=%d): %s" % (k, g["n"], "all arrays bit-identical" if not bad else "DIFFER: %s" % bad))
        assert not bad, (k, bad)
        del g
