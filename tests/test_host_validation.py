"""Host-side argument checks of the C ABI (CPU only: every case below is
rejected before the library touches a device).

Empty and malformed CSR headers, NULL arguments and out-of-range parameters
must come back as AMG_ERR_INVALID with a message and no hierarchy; the status
strings cover every code the header defines.
"""
import ctypes as C

import numpy as np
import pytest

import paper_2303_02352_amd as amd


def _setup(A, p):
    h = C.c_void_p()
    st = amd.load().amg_setup(C.byref(A), C.byref(p), C.byref(h))
    return st, h


def _csr(n, nnz, arrays=True):
    # the header is rejected before any array is read: small arrays suffice
    rp = np.zeros(max(n, 0) + 1, dtype=np.int32)
    ci = np.zeros(8, dtype=np.int32)
    va = np.ones(8)
    keep = (rp, ci, va)
    if not arrays:
        return amd.amg_csr(n, nnz, None, None, None, 0), keep
    return amd.amg_csr(n, nnz, rp.ctypes.data, ci.ctypes.data, va.ctypes.data, 0), keep


@pytest.mark.parametrize("n,nnz,arrays", [(0, 0, True), (-3, 0, True), (4, 3, True), (4, 4, False),
                                          (4, 2 ** 31, True)])
def test_bad_csr_header_is_invalid(n, nnz, arrays):
    A, keep = _csr(n, nnz, arrays)
    st, h = _setup(A, amd.default_params())
    assert st == amd.AMG_ERR_INVALID and not h.value
    assert amd.load().amg_last_error().decode()


@pytest.mark.parametrize("field,value", [("aggr_steps", 0), ("max_levels", 0), ("coarse_max", 0),
                                         ("coarse_sweeps", 0), ("pre_sweeps", -1), ("post_sweeps", -1),
                                         ("smooth_sweeps", -1), ("coarse_solver", 7), ("smooth_vec", 5),
                                         ("smooth_vec", amd.AMG_SMOOTH_GIVEN), ("precision", 3),
                                         ("precond", 2), ("value_coding", 2), ("value_coding", -1),
                                         ("smooth_vec", amd.AMG_SMOOTH_LEARNED), ("n_parts", 0),
                                         ("n_parts", 2 ** 24 + 1), ("cycle_type", 3), ("relax_type", 2),
                                         ("coarse_relax", 5), ("max_hrc", 0), ("max_hrc", 17),
                                         ("bootstrap_type", 3), ("bootstrap_its", 0),
                                         ("bootstrap_rate", 0.0), ("bootstrap_rate", 1.5)])
def test_bad_parameter_is_invalid(field, value):
    A, keep = _csr(1, 1)
    p = amd.default_params()
    setattr(p, field, value)
    st, h = _setup(A, p)
    assert st == amd.AMG_ERR_INVALID and not h.value
    assert amd.load().amg_last_error().decode()


def test_default_parameters():
    p = amd.default_params()
    assert (p.aggr_steps, p.max_levels, p.coarse_max, p.pre_sweeps, p.post_sweeps) == (2, 40, 100, 4, 4)
    assert p.value_coding == amd.AMG_VALUES_AUTO and p.precision == amd.AMG_PREC_DOUBLE
    assert (p.n_parts, p.cycle_type, p.relax_type, p.coarse_relax) == (1, amd.AMG_CYCLE_V,
                                                                      amd.AMG_RELAX_L1_JACOBI,
                                                                      amd.AMG_RELAX_L1_JACOBI)
    assert (p.max_hrc, p.bootstrap_type, p.bootstrap_its, p.bootstrap_seed) == (1, amd.AMG_BOOTSTRAP_MULT, 15, 1)
    assert p.bootstrap_rate == 0.8 and not p.model_params and not p.smooth_vector


def test_binary32_cycle_with_other_options_is_unsupported():
    A, keep = _csr(1, 1)
    for field, value in (("cycle_type", amd.AMG_CYCLE_W), ("relax_type", amd.AMG_RELAX_GS),
                         ("coarse_relax", amd.AMG_RELAX_SYM_GS)):
        p = amd.default_params(precision=amd.AMG_PREC_MIXED)
        setattr(p, field, value)
        st, h = _setup(A, p)
        assert st == amd.AMG_ERR_UNSUPPORTED and not h.value, field


def test_unknown_parameter_name_is_refused():
    with pytest.raises(TypeError):
        amd.default_params(n_part=2)


def test_null_arguments():
    L = amd.load()
    A, keep = _csr(1, 1)
    p = amd.default_params()
    h = C.c_void_p()
    assert L.amg_setup(None, C.byref(p), C.byref(h)) == amd.AMG_ERR_INVALID
    assert L.amg_setup(C.byref(A), None, C.byref(h)) == amd.AMG_ERR_INVALID
    assert L.amg_setup(C.byref(A), C.byref(p), None) == amd.AMG_ERR_INVALID
    assert L.amg_params_default(None) == amd.AMG_ERR_INVALID


def test_status_strings_cover_every_code():
    L = amd.load()
    codes = [amd.AMG_OK, amd.AMG_NOT_CONVERGED, amd.AMG_ERR_INVALID, amd.AMG_ERR_NOT_SPD,
             amd.AMG_ERR_NONFINITE, amd.AMG_ERR_NOMEM, amd.AMG_ERR_DEVICE, amd.AMG_ERR_UNSUPPORTED,
             amd.AMG_ERR_MODEL]
    msgs = [L.amg_strerror(c).decode() for c in codes]
    assert all(msgs) and len(set(msgs)) == len(codes)


def test_valid_system_without_a_device_fails_loudly():
    """With no GPU the library has no fallback: a well-formed system is
    refused with AMG_ERR_DEVICE and a message, and no hierarchy is made."""
    import torch
    if torch.cuda.device_count() > 0:
        pytest.skip("a GPU is visible")
    import workloads as W
    A = W.poisson7(4)
    csr = amd.amg_csr(A.n, A.nnz, A.row_ptr.ctypes.data, A.col.ctypes.data, A.val.ctypes.data, 0)
    st, h = _setup(csr, amd.default_params())
    assert st == amd.AMG_ERR_DEVICE and not h.value
    assert "device" in amd.load().amg_last_error().decode()
