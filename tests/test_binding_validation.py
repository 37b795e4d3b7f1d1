"""The Python binding refuses malformed array arguments before their
addresses cross the C ABI (CPU only: every case raises ValueError without a
library call that could touch a device).

Covered: wrong dtype, wrong length, non-contiguous arrays, arrays split
between host and device memory, host vectors where the solve needs device
memory, and the batched and network entry points' block sizes.
"""
import numpy as np
import pytest

import paper_2303_02352_amd as amd
import workloads as W

torch = pytest.importorskip("torch")


class _FakeCuda:
    """Stands in for a CUDA tensor in the memory-space checks (no device is
    touched: the check raises before any address is used)."""

    def __init__(self, a, index=0):
        self._a = a
        self.dtype = torch.from_numpy(a).dtype
        self.shape = a.shape
        self.is_cuda = True
        self.device = type("D", (), {"index": index})()

    def data_ptr(self):
        return 0

    def is_contiguous(self):
        return True

    def numel(self):
        return self._a.size


def _csr():
    A = W.poisson7(3)
    return A.row_ptr.copy(), A.col.copy(), A.val.copy()


@pytest.mark.parametrize("case", ["rp_dtype", "col_dtype", "val_dtype", "val_short", "col_short",
                                  "noncontig", "mixed_space", "smooth_len", "smooth_space"])
def test_setup_refuses_bad_csr(case):
    rp, ci, va = _csr()
    kw = {}
    if case == "rp_dtype":
        rp = rp.astype(np.int64)
    elif case == "col_dtype":
        ci = ci.astype(np.int64)
    elif case == "val_dtype":
        va = va.astype(np.float32)
    elif case == "val_short":
        va = va[:-1].copy()
    elif case == "col_short":
        ci = ci[:-1].copy()
    elif case == "noncontig":
        va = np.repeat(va, 2)[::2]
    elif case == "mixed_space":
        va = _FakeCuda(va)
    elif case == "smooth_len":
        kw["smooth_vector"] = np.ones(rp.size)
    elif case == "smooth_space":
        kw["smooth_vector"] = _FakeCuda(np.ones(rp.size - 1))
    with pytest.raises(ValueError):
        amd.Hierarchy(rp, ci, va, **kw)


def _fake_hierarchy(sizes=(27, 4)):
    H = amd.Hierarchy.__new__(amd.Hierarchy)
    H.h = None
    H.sizes = list(sizes)
    H.device = 0
    return H


@pytest.mark.parametrize("case", ["host", "dtype", "short", "long", "other_device"])
def test_solve_and_vcycle_refuse_bad_vectors(case):
    H = _fake_hierarchy()
    n = H.sizes[0]
    good = _FakeCuda(np.zeros(n))
    bad = {"host": np.zeros(n), "dtype": _FakeCuda(np.zeros(n, np.float32)),
           "short": _FakeCuda(np.zeros(n - 1)), "long": _FakeCuda(np.zeros(n + 1)),
           "other_device": _FakeCuda(np.zeros(n), index=1)}[case]
    with pytest.raises(ValueError):
        H.solve(good, bad)
    with pytest.raises(ValueError):
        H.solve(bad, good)
    with pytest.raises(ValueError):
        H.vcycle(bad, good)
    with pytest.raises(ValueError):
        H.vcycle(good, bad)


def test_level_calls_check_level_and_size():
    H = _fake_hierarchy()
    with pytest.raises(ValueError):
        H.spmv(2, _FakeCuda(np.zeros(4)), _FakeCuda(np.zeros(4)))
    with pytest.raises(ValueError):        # level-1 call given level-0 sized vectors
        H.spmv(1, _FakeCuda(np.zeros(27)), _FakeCuda(np.zeros(27)))
    with pytest.raises(ValueError):
        H.sweep(1, _FakeCuda(np.zeros(4)), _FakeCuda(np.zeros(4)), _FakeCuda(np.zeros(3)))


def test_batch_refuses_bad_blocks():
    B = amd.Batch.__new__(amd.Batch)
    B.h = None
    B.sizes = [27, 64]
    B.device = 0
    ok = _FakeCuda(np.zeros(91 * 4))
    with pytest.raises(ValueError):
        B.solve(ok, _FakeCuda(np.zeros(91 * 4 - 1)), 4)
    with pytest.raises(ValueError):
        B.solve(ok, ok, 0)
    with pytest.raises(ValueError):
        B.vcycle(ok, np.zeros(91 * 4), 4)       # host output
    with pytest.raises(ValueError):
        amd.Batch([])
    rp, ci, va = _csr()
    with pytest.raises(ValueError):             # systems in different memory spaces
        amd.Batch([(rp, ci, va), (_FakeCuda(rp), _FakeCuda(ci), _FakeCuda(va))])


def test_network_refuses_bad_arguments():
    with pytest.raises(ValueError):
        amd.SmoothVectorNet(np.zeros(amd.AMG_MPNN_NPARAMS + 1, np.float32))
    net = amd.SmoothVectorNet.__new__(amd.SmoothVectorNet)
    net.h = None
    rp, ci, va = _csr()
    with pytest.raises(ValueError):             # host CSR
        net.features(rp, ci, va)
    d = [_FakeCuda(a) for a in (rp, ci, va)]
    with pytest.raises(ValueError):
        net.predict(*d, w_out=_FakeCuda(np.zeros(26)))
    with pytest.raises(ValueError):
        net.train_step(*d, w_target=np.ones(27), lr=0.0)
