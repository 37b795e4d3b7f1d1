"""Python binding of libamg355 (MI355X AMG-preconditioned flexible CG).

Argument marshalling only: every step of setup and solve runs in the HIP
kernels of ``libamg355.so`` behind the C ABI of ``include/amg355.h``.  The
functions keep the C names (``amg_setup``, ``amg_pcg_solve``, ...); the
``Hierarchy`` class is a convenience wrapper over them.  torch tensors supply
device memory and the stream; there is no CPU fallback, and importing the
package raises if the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libamg355.so")

AMG_OK, AMG_NOT_CONVERGED = 0, 1
AMG_ERR_INVALID, AMG_ERR_NOT_SPD, AMG_ERR_NONFINITE = -1, -2, -3
AMG_ERR_NOMEM, AMG_ERR_DEVICE, AMG_ERR_UNSUPPORTED, AMG_ERR_MODEL = -4, -5, -6, -7
AMG_COARSE_CHOLESKY, AMG_COARSE_JACOBI = 0, 1
AMG_SMOOTH_ONES, AMG_SMOOTH_RELAX, AMG_SMOOTH_GIVEN, AMG_SMOOTH_LEARNED = 0, 1, 2, 3
AMG_PREC_DOUBLE, AMG_PREC_MIXED = 0, 1
AMG_VALUES_PLAIN, AMG_VALUES_AUTO = 0, 1
AMG_CYCLE_V, AMG_CYCLE_H, AMG_CYCLE_W = 0, 1, 2
AMG_RELAX_JACOBI, AMG_RELAX_GS, AMG_RELAX_SYM_GS, AMG_RELAX_L1_JACOBI = 0, 1, 3, 4
AMG_BOOTSTRAP_MULT, AMG_BOOTSTRAP_SYMMULT, AMG_BOOTSTRAP_ADD = 0, 1, 2
AMG_MAX_LEVELS = 64
KERNEL_SPMV, KERNEL_SWEEP, KERNEL_RESTRICT, KERNEL_PROLONG, KERNEL_UPDATE, KERNEL_CORR_SWEEP = 0, 1, 2, 3, 4, 5


class amg_csr(C.Structure):
    _fields_ = [("n", C.c_int32), ("nnz", C.c_int64), ("row_ptr", C.c_void_p),
                ("col_idx", C.c_void_p), ("val", C.c_void_p), ("on_device", C.c_int32)]


class amg_params(C.Structure):
    _fields_ = [(f, C.c_int32) for f in (
        "aggr_steps", "max_levels", "coarse_max", "coarse_solver", "coarse_sweeps",
        "pre_sweeps", "post_sweeps", "smooth_vec", "smooth_sweeps", "precond", "precision",
        "value_coding", "n_parts", "cycle_type", "relax_type", "coarse_relax", "max_hrc",
        "bootstrap_type", "bootstrap_its", "bootstrap_seed")] + [
        ("bootstrap_rate", C.c_double), ("smooth_vector", C.c_void_p),
        ("model_params", C.c_void_p), ("model_path", C.c_char_p), ("stream", C.c_void_p)]


class amg_info_t(C.Structure):
    _fields_ = [("levels", C.c_int32), ("n", C.c_int32 * AMG_MAX_LEVELS),
                ("nnz", C.c_int64 * AMG_MAX_LEVELS), ("opc", C.c_double),
                ("coarse_dense", C.c_int32), ("matching_rounds", C.c_int32),
                ("setup_ms", C.c_double), ("setup_match_ms", C.c_double),
                ("setup_rap_ms", C.c_double), ("device_bytes", C.c_int64),
                ("dict_size", C.c_int32 * AMG_MAX_LEVELS), ("setup_smooth_ms", C.c_double),
                ("nhrc", C.c_int32), ("nrates", C.c_int32), ("rates", C.c_double * 16),
                ("setup_bootstrap_ms", C.c_double), ("smooth_status", C.c_int32)]


class amg_batch_info_t(C.Structure):
    _fields_ = [("nsys", C.c_int32), ("levels", C.c_int32), ("n", C.c_int32 * AMG_MAX_LEVELS),
                ("n_smoothed", C.c_int32 * AMG_MAX_LEVELS), ("nnz", C.c_int64 * AMG_MAX_LEVELS),
                ("cols_per_lane", C.c_int32 * AMG_MAX_LEVELS), ("setup_ms", C.c_double),
                ("tune_ms", C.c_double), ("cols_per_lane_corr", C.c_int32 * AMG_MAX_LEVELS),
                ("tile_rows", C.c_int32), ("spmm_cols", C.c_int32)]


EXPORTS = {
    "amg_params_default": (C.c_int, [C.POINTER(amg_params)]),
    "amg_setup": (C.c_int, [C.POINTER(amg_csr), C.POINTER(amg_params), C.POINTER(C.c_void_p)]),
    "amg_pcg_solve": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_int32,
                                C.POINTER(C.c_int32), C.POINTER(C.c_double)]),
    "amg_pcg_solve_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_int32,
                                        C.POINTER(C.c_int32), C.POINTER(C.c_double)]),
    "amg_pcg_solve_noalloc_max_rows": (C.c_int64, []),
    "amg_destroy": (None, [C.c_void_p]),
    "amg_strerror": (C.c_char_p, [C.c_int]),
    "amg_last_error": (C.c_char_p, []),
    "amg_info": (C.c_int, [C.c_void_p, C.POINTER(amg_info_t)]),
    "amg_export_level": (C.c_int, [C.c_void_p, C.c_int32] + [C.c_void_p] * 7),
    "amg_component": (C.c_void_p, [C.c_void_p, C.c_int32]),
    "amg_vcycle": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "amg_spmv": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
    "amg_sweep": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
    "amg_time_kernel": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32,
                                  C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "amg_batch_setup": (C.c_int, [C.c_int32, C.POINTER(amg_csr), C.POINTER(amg_params),
                                  C.POINTER(C.c_void_p)]),
    "amg_batch_solve": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_double,
                                  C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
    "amg_batch_solve_systems": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_double,
                                          C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
    "amg_batch_vcycle": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
    "amg_batch_info": (C.c_int, [C.c_void_p, C.POINTER(amg_batch_info_t)]),
    "amg_batch_destroy": (None, [C.c_void_p]),
    "amg_mpnn_create": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(C.c_void_p)]),
    "amg_mpnn_read_params": (C.c_int, [C.c_char_p, C.c_void_p]),
    "amg_mpnn_get_params": (C.c_int, [C.c_void_p, C.c_void_p]),
    "amg_mpnn_features": (C.c_int, [C.c_void_p, C.POINTER(amg_csr), C.c_void_p]),
    "amg_mpnn_predict": (C.c_int, [C.c_void_p, C.POINTER(amg_csr), C.c_void_p, C.c_void_p]),
    "amg_mpnn_train_step": (C.c_int, [C.c_void_p, C.POINTER(amg_csr), C.c_void_p, C.c_float,
                                      C.POINTER(C.c_float), C.c_void_p]),
    "amg_mpnn_destroy": (None, [C.c_void_p]),
}
AMG_MPNN_NPARAMS = 2657

_lib = None


def load():
    """Load libamg355.so; raises if it is missing (no fallback path exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libamg355.so is not built: run `python -m paper_2303_02352_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class AMGError(RuntimeError):
    def __init__(self, code, where):
        L = load()
        msg = L.amg_last_error().decode() or L.amg_strerror(code).decode()
        super().__init__("%s: status %d (%s)" % (where, code, msg))
        self.code = code


def _ptr(a):
    """Device or host address of a torch tensor / numpy array (contiguous)."""
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        if not a.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return C.c_void_p(a.data_ptr())
    if not a.flags["C_CONTIGUOUS"]:
        raise ValueError("array must be C-contiguous")
    return C.c_void_p(a.ctypes.data)


def _on_device(a):
    return 1 if (hasattr(a, "is_cuda") and a.is_cuda) else 0


_DTYPES = {"float64": ("float64", "torch.float64"), "int32": ("int32", "torch.int32"),
           "float32": ("float32", "torch.float32")}


def _space(a):
    """('cuda', index) for a device tensor, ('host', None) for host memory."""
    if hasattr(a, "is_cuda") and a.is_cuda:
        return ("cuda", a.device.index)
    return ("host", None)


def _arr(a, name, dtype, numel=None, space=None):
    """Check one array argument before its address crosses the C ABI: a numpy
    array or torch tensor of `dtype`, contiguous, with `numel` elements, in
    `space` (('cuda', index), ('host', None), 'cuda' for any device, or None
    for either).  Raises ValueError; returns the address."""
    if not (hasattr(a, "data_ptr") or isinstance(a, np.ndarray)):
        raise ValueError("%s: expected a numpy array or torch tensor, got %s" % (name, type(a).__name__))
    if str(a.dtype) not in _DTYPES[dtype]:
        raise ValueError("%s: dtype %s, expected %s" % (name, a.dtype, dtype))
    contiguous = a.is_contiguous() if hasattr(a, "data_ptr") else a.flags["C_CONTIGUOUS"]
    if not contiguous:
        raise ValueError("%s: must be contiguous" % name)
    size = a.numel() if hasattr(a, "data_ptr") else a.size
    if numel is not None and size != numel:
        raise ValueError("%s: %d elements, expected %d" % (name, size, numel))
    sp = _space(a)
    if space == "cuda":
        if sp[0] != "cuda":
            raise ValueError("%s: must be device memory (a CUDA tensor)" % name)
    elif space is not None and sp != space:
        raise ValueError("%s: in %s, expected %s (all arrays of a call share one memory space "
                         "and device)" % (name, _where(sp), _where(space)))
    return _ptr(a)


def _where(sp):
    return "host memory" if sp[0] == "host" else "cuda:%s" % sp[1]


def default_params(**overrides) -> amg_params:
    p = amg_params()
    load().amg_params_default(C.byref(p))
    names = {f[0] for f in amg_params._fields_}
    for k, v in overrides.items():
        if k not in names:
            raise TypeError("unknown amg_params field %r" % k)
        setattr(p, k, v)
    return p


def current_stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _csr_args(row_ptr, col, val):
    """amg_csr for three arrays in one memory space (checked), and n, nnz."""
    sp = _space(val)
    if not hasattr(row_ptr, "shape") or len(row_ptr.shape) != 1 or row_ptr.shape[0] < 1:
        raise ValueError("row_ptr: expected a 1-D array of n + 1 entries")
    n = int(row_ptr.shape[0]) - 1
    nnz = int(col.shape[0]) if hasattr(col, "shape") and len(col.shape) == 1 else -1
    if nnz < 0:
        raise ValueError("col: expected a 1-D array")
    prp = _arr(row_ptr, "row_ptr", "int32", n + 1, sp)
    pci = _arr(col, "col", "int32", nnz, sp)
    pva = _arr(val, "val", "float64", nnz, sp)
    return amg_csr(n, nnz, prp, pci, pva, 1 if sp[0] == "cuda" else 0), n, nnz


def _device_of(a):
    """Device index of a CUDA tensor, else the current device."""
    if _on_device(a):
        return a.device.index
    import torch
    return torch.cuda.current_device()


class Hierarchy:
    """AMG hierarchy built by ``amg_setup``.

    ``row_ptr`` (int32), ``col`` (int32), ``val`` (float64): torch CUDA
    tensors or host numpy arrays.  Keyword arguments override fields of
    ``amg_params`` (e.g. ``aggr_steps=3``, ``precision=AMG_PREC_MIXED``);
    ``smooth_vector`` is an array of n doubles in the CSR's memory space.
    """

    def __init__(self, row_ptr, col, val, stream=None, smooth_vector=None, model_params=None,
                 model_path=None, **params):
        L = load()
        A, self.n, self.nnz = _csr_args(row_ptr, col, val)
        p = default_params(**params)
        if smooth_vector is not None:
            p.smooth_vec = AMG_SMOOTH_GIVEN
            p.smooth_vector = _arr(smooth_vector, "smooth_vector", "float64", self.n, _space(val))
        theta = None
        if model_params is not None:
            theta = np.ascontiguousarray(model_params, dtype=np.float32)
            if theta.shape != (AMG_MPNN_NPARAMS,):
                raise ValueError("model_params: shape %s, expected (%d,)" % (theta.shape, AMG_MPNN_NPARAMS))
            p.smooth_vec = AMG_SMOOTH_LEARNED
            p.model_params = theta.ctypes.data
        path = None
        if model_path is not None:
            path = os.fsencode(model_path)
            p.smooth_vec = AMG_SMOOTH_LEARNED
            p.model_path = path
        p.stream = stream if stream is not None else (current_stream() if A.on_device else None)
        self.params = p
        h = C.c_void_p()
        st = L.amg_setup(C.byref(A), C.byref(p), C.byref(h))
        p.smooth_vector = None   # read during amg_setup only
        p.model_params = None
        p.model_path = None
        if st != AMG_OK:
            raise AMGError(st, "amg_setup")
        self.h = h
        self.device = _device_of(val)
        self.sizes = self.info()["n"]

    def _vec(self, a, name, k=0):
        """A device vector of level k's size on the hierarchy's device."""
        return _arr(a, name, "float64", self.sizes[k], ("cuda", self.device))

    def _level(self, k):
        if not 0 <= int(k) < len(self.sizes):
            raise ValueError("level %d out of range [0, %d)" % (k, len(self.sizes)))
        return int(k)

    def close(self):
        if getattr(self, "_borrowed", False):
            return
        if getattr(self, "h", None) and self.h.value:
            load().amg_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, b, x, rtol=1e-6, maxit=1000, check=True):
        """Flexible PCG; x (device) holds x0 on entry.  Returns (status, iters, relres)."""
        it, rel = C.c_int32(), C.c_double()
        pb, px = self._vec(b, "b"), self._vec(x, "x")
        st = load().amg_pcg_solve(self.h, pb, px, float(rtol), int(maxit), C.byref(it), C.byref(rel))
        if check and st < 0:
            raise AMGError(st, "amg_pcg_solve")
        return st, it.value, rel.value

    def solve_noalloc(self, b, x, rtol=1e-6, maxit=1000, check=True):
        """amg_pcg_solve_noalloc: the same solve with its PCG state in the
        library's static per-device scratch (no allocation during the call).
        Returns (status, iters, relres)."""
        it, rel = C.c_int32(), C.c_double()
        pb, px = self._vec(b, "b"), self._vec(x, "x")
        st = load().amg_pcg_solve_noalloc(self.h, pb, px, float(rtol), int(maxit), C.byref(it),
                                          C.byref(rel))
        if check and st < 0:
            raise AMGError(st, "amg_pcg_solve_noalloc")
        return st, it.value, rel.value

    def info(self) -> dict:
        inf = amg_info_t()
        st = load().amg_info(self.h, C.byref(inf))
        if st != AMG_OK:
            raise AMGError(st, "amg_info")
        L = inf.levels
        return dict(levels=L, n=list(inf.n[:L]), nnz=list(inf.nnz[:L]), opc=inf.opc,
                    coarse_dense=bool(inf.coarse_dense), matching_rounds=inf.matching_rounds,
                    setup_ms=inf.setup_ms, setup_match_ms=inf.setup_match_ms,
                    setup_rap_ms=inf.setup_rap_ms, device_bytes=inf.device_bytes,
                    dict_size=list(inf.dict_size[:L]), setup_smooth_ms=inf.setup_smooth_ms,
                    nhrc=inf.nhrc, rates=list(inf.rates[:inf.nrates]),
                    setup_bootstrap_ms=inf.setup_bootstrap_ms, smooth_status=inf.smooth_status)

    def component(self, j):
        """Hierarchy j of the bootstrap composite (0 = this one) as a borrowed
        view for info / export_level / vcycle / spmv / sweep; it is never
        destroyed on its own and keeps this hierarchy alive."""
        ph = load().amg_component(self.h, int(j))
        if not ph:
            raise AMGError(AMG_ERR_INVALID, "amg_component")
        v = object.__new__(Hierarchy)
        v.h = C.c_void_p(ph)
        v.n, v.nnz, v.params, v.device, v._owner = self.n, self.nnz, self.params, self.device, self
        v._borrowed = True
        v.sizes = v.info()["n"]
        return v

    def export_level(self, k) -> dict:
        inf = self.info()
        n, nnz = inf["n"][k], inf["nnz"][k]
        out = dict(row_ptr=np.empty(n + 1, np.int32), col=np.empty(nnz, np.int32),
                   val=np.empty(nnz), dinv=np.empty(n), w=np.empty(n),
                   agg=np.full(n, -1, np.int32), pval=np.zeros(n))
        st = load().amg_export_level(self.h, k, *[_ptr(out[f]) for f in
                                                  ("row_ptr", "col", "val", "dinv", "w", "agg", "pval")])
        if st != AMG_OK:
            raise AMGError(st, "amg_export_level")
        if k == inf["levels"] - 1:
            out["agg"] = out["pval"] = None
        out["n"], out["nnz"] = n, nnz
        return out

    def vcycle(self, r, z):
        st = load().amg_vcycle(self.h, self._vec(r, "r"), self._vec(z, "z"))
        if st != AMG_OK:
            raise AMGError(st, "amg_vcycle")

    def spmv(self, k, x, y):
        k = self._level(k)
        st = load().amg_spmv(self.h, k, self._vec(x, "x", k), self._vec(y, "y", k))
        if st != AMG_OK:
            raise AMGError(st, "amg_spmv")

    def sweep(self, k, r, x, xn):
        k = self._level(k)
        st = load().amg_sweep(self.h, k, self._vec(r, "r", k), self._vec(x, "x", k), self._vec(xn, "xn", k))
        if st != AMG_OK:
            raise AMGError(st, "amg_sweep")

    def time_kernel(self, kernel, k=0, reps=20):
        ms, by = C.c_double(), C.c_double()
        st = load().amg_time_kernel(self.h, int(kernel), int(k), int(reps), C.byref(ms), C.byref(by))
        if st != AMG_OK:
            raise AMGError(st, "amg_time_kernel")
        return ms.value, by.value


class Batch:
    """Batched hierarchy (``amg_batch_setup``) over several systems.

    ``systems``: list of (row_ptr, col, val) torch CUDA tensors or host numpy
    arrays.  Vectors passed to ``solve``/``vcycle`` are device tensors holding
    the systems one after another, each an n_s x nrhs row-major block.
    """

    def __init__(self, systems, stream=None, **params):
        L = load()
        self._keep = systems
        if not systems:
            raise ValueError("a batch needs at least one system")
        arr = (amg_csr * len(systems))()
        space = _space(systems[0][2])
        for i, (rp, ci, va) in enumerate(systems):
            if _space(va) != space:
                raise ValueError("system %d: every system must be in %s" % (i, _where(space)))
            arr[i] = _csr_args(rp, ci, va)[0]
        self.sizes = [int(s[0].shape[0]) - 1 for s in systems]
        p = default_params(**params)
        p.stream = stream if stream is not None else (current_stream() if arr[0].on_device else None)
        self.params = p
        h = C.c_void_p()
        st = L.amg_batch_setup(len(systems), arr, C.byref(p), C.byref(h))
        if st != AMG_OK:
            raise AMGError(st, "amg_batch_setup")
        self.h = h
        self.device = _device_of(systems[0][2])

    def _block(self, a, name, nrhs):
        # (an unsupported nrhs is the library's to refuse: AMG_ERR_UNSUPPORTED)
        if int(nrhs) < 1:
            raise ValueError("nrhs must be positive")
        return _arr(a, name, "float64", sum(self.sizes) * int(nrhs), ("cuda", self.device))

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            load().amg_batch_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, B, X, nrhs, rtol=1e-6, maxit=1000, check=True):
        """Returns (status, iters[nsys, nrhs], relres[nsys, nrhs], pair_status[nsys, nrhs])."""
        ns = len(self.sizes)
        it = np.zeros(ns * nrhs, np.int32)
        rel = np.zeros(ns * nrhs)
        pst = np.zeros(ns * nrhs, np.int32)
        pB, pX = self._block(B, "B", nrhs), self._block(X, "X", nrhs)
        st = load().amg_batch_solve(self.h, int(nrhs), pB, pX, float(rtol), int(maxit),
                                    _ptr(it), _ptr(rel), _ptr(pst))
        if check and st < 0:
            raise AMGError(st, "amg_batch_solve")
        return st, it.reshape(ns, nrhs), rel.reshape(ns, nrhs), pst.reshape(ns, nrhs)

    def solve_systems(self, Bs, Xs, nrhs, rtol=1e-6, maxit=1000, check=True):
        """One (n_s * nrhs) vector per system for B and X (amg_batch_solve_systems);
        returns as solve()."""
        ns = len(self.sizes)
        if int(nrhs) < 1:
            raise ValueError("nrhs must be positive")
        if len(Bs) != ns or len(Xs) != ns:
            raise ValueError("one B and one X per system expected (%d systems)" % ns)
        pb = (C.c_void_p * ns)(*[_arr(b, "B[%d]" % k, "float64", self.sizes[k] * int(nrhs),
                                      ("cuda", self.device)) for k, b in enumerate(Bs)])
        px = (C.c_void_p * ns)(*[_arr(x, "X[%d]" % k, "float64", self.sizes[k] * int(nrhs),
                                      ("cuda", self.device)) for k, x in enumerate(Xs)])
        it = np.zeros(ns * nrhs, np.int32)
        rel = np.zeros(ns * nrhs)
        pst = np.zeros(ns * nrhs, np.int32)
        st = load().amg_batch_solve_systems(self.h, int(nrhs), pb, px, float(rtol), int(maxit),
                                            _ptr(it), _ptr(rel), _ptr(pst))
        if check and st < 0:
            raise AMGError(st, "amg_batch_solve_systems")
        return st, it.reshape(ns, nrhs), rel.reshape(ns, nrhs), pst.reshape(ns, nrhs)

    def vcycle(self, R, Z, nrhs):
        st = load().amg_batch_vcycle(self.h, int(nrhs), self._block(R, "R", nrhs), self._block(Z, "Z", nrhs))
        if st != AMG_OK:
            raise AMGError(st, "amg_batch_vcycle")

    def info(self) -> dict:
        inf = amg_batch_info_t()
        st = load().amg_batch_info(self.h, C.byref(inf))
        if st != AMG_OK:
            raise AMGError(st, "amg_batch_info")
        L = inf.levels
        return dict(nsys=inf.nsys, levels=L, n=list(inf.n[:L]), n_smoothed=list(inf.n_smoothed[:L]),
                    nnz=list(inf.nnz[:L]), cols_per_lane=list(inf.cols_per_lane[:L]),
                    cols_per_lane_corr=list(inf.cols_per_lane_corr[:L]), tile_rows=inf.tile_rows,
                    spmm_cols=inf.spmm_cols,
                    setup_ms=inf.setup_ms, tune_ms=inf.tune_ms)


def read_model_params(path) -> np.ndarray:
    """The network parameters of a model file, read by the library
    (amg_mpnn_read_params; host only)."""
    out = np.empty(AMG_MPNN_NPARAMS, dtype=np.float32)
    st = load().amg_mpnn_read_params(os.fsencode(path), out.ctypes.data)
    if st != AMG_OK:
        raise AMGError(st, "amg_mpnn_read_params")
    return out


class SmoothVectorNet:
    """Learned smooth-vector network (``amg_mpnn_*``): features, predict, train."""

    def __init__(self, params=None, stream=None):
        L = load()
        theta = None if params is None else np.ascontiguousarray(params, dtype=np.float32)
        if theta is not None and theta.shape != (AMG_MPNN_NPARAMS,):
            raise ValueError("params: shape %s, expected (%d,)" % (theta.shape, AMG_MPNN_NPARAMS))
        h = C.c_void_p()
        st = L.amg_mpnn_create(_ptr(theta), stream, C.byref(h))
        if st != AMG_OK:
            raise AMGError(st, "amg_mpnn_create")
        self.h = h

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            load().amg_mpnn_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _csr(row_ptr, col, val):
        if not _on_device(val):
            raise ValueError("the network reads a CSR in device memory")
        return _csr_args(row_ptr, col, val)[0]

    def params(self):
        out = np.empty(AMG_MPNN_NPARAMS, np.float32)
        st = load().amg_mpnn_get_params(self.h, _ptr(out))
        if st != AMG_OK:
            raise AMGError(st, "amg_mpnn_get_params")
        return out

    def features(self, row_ptr, col, val):
        A = self._csr(row_ptr, col, val)
        X = np.empty((A.n, 8), np.float32)
        st = load().amg_mpnn_features(self.h, C.byref(A), _ptr(X))
        if st != AMG_OK:
            raise AMGError(st, "amg_mpnn_features")
        return X

    def predict(self, row_ptr, col, val, w_out=None, want_y=False):
        """w_out: device float64 tensor of n (exp of the prediction); returns y (host) if asked."""
        A = self._csr(row_ptr, col, val)
        y = np.empty(A.n, np.float32) if want_y else None
        pw = None if w_out is None else _arr(w_out, "w_out", "float64", A.n, _space(val))
        st = load().amg_mpnn_predict(self.h, C.byref(A), pw, _ptr(y))
        if st != AMG_OK:
            raise AMGError(st, "amg_mpnn_predict")
        return y

    def train_step(self, row_ptr, col, val, w_target, lr, want_grad=False):
        A = self._csr(row_ptr, col, val)
        loss = C.c_float()
        g = np.empty(AMG_MPNN_NPARAMS, np.float32) if want_grad else None
        pt = _arr(w_target, "w_target", "float64", A.n, _space(val))
        st = load().amg_mpnn_train_step(self.h, C.byref(A), pt, float(lr), C.byref(loss), _ptr(g))
        if st != AMG_OK:
            raise AMGError(st, "amg_mpnn_train_step")
        return (loss.value, g) if want_grad else loss.value
