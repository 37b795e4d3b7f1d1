"""Shared helpers for the GPU tests (marshalling between numpy and torch)."""
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
