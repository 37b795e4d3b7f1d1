"""CPU oracle for the AMG-preconditioned flexible CG -- TEST INFRASTRUCTURE ONLY.

A plain sequential FP64 implementation (``amg_oracle.c``) of what the GPU
library computes, written from the paper's algorithms (arXiv 2303.02352:
Sec. 3 Alg. 1, Sec. 3.1 Alg. 2 / Alg. 3, Sec. 4.1 matching).  Only the tests,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may
import this package.  It shares no code with ``paper_2303_02352_amd``.

Functions pinned by tests in ``tests/test_oracle_*.py``; the pins are listed
in each test module's docstring.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, fields

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "amg_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, NOT_CONVERGED, INVALID, NOT_SPD, NONFINITE, NOMEM = 0, 1, -1, -2, -3, -4

_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")


_LIB_TIMING = os.path.join(_HERE, "liboracle_omp.so")


def _compile(out, flags, force):
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(_SRC):
        tmp = out + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc"] + flags + ["-std=c11", "-ffp-contract=off", "-fno-fast-math",
                                                 "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, out)
    return out


def build(force: bool = False) -> str:
    """Compile ``liboracle.so``, the parity oracle: gcc, sequential, plain C,
    no FMA contraction."""
    return _compile(_LIB, ["-O2"], force)


def build_timing(force: bool = False) -> str:
    """Compile ``liboracle_omp.so``, the CPU-baseline timing build of the same
    source: -O3 -march=native with OpenMP over the rows of SpMV, sweeps,
    residuals, prolongation and PCG updates, per-thread dot partials folded
    in thread order; setup stays sequential.  Used only to time the CPU
    baseline on all host cores, never as the parity reference."""
    return _compile(_LIB_TIMING, ["-O3", "-march=native", "-fopenmp"], force)


class Params(C.Structure):
    _fields_ = [(name, C.c_int32) for name in (
        "aggr_steps", "max_levels", "coarse_max", "coarse_solver", "coarse_sweeps",
        "pre_sweeps", "post_sweeps", "smooth_vec", "smooth_sweeps", "precond", "n_parts",
        "cycle_type", "relax_type", "coarse_relax", "max_hrc", "bootstrap_type", "bootstrap_its",
        "bootstrap_seed")] + [("bootstrap_rate", C.c_double)]


@dataclass
class AMGParams:
    """Method parameters (defaults: s = 2 pairwise steps -> aggregates <= 4,
    coarsest <= 100 rows by dense Cholesky, 4 + 4 l1-Jacobi sweeps, constant
    smooth vector)."""
    aggr_steps: int = 2
    max_levels: int = 40
    coarse_max: int = 100
    coarse_solver: int = 0
    coarse_sweeps: int = 20
    pre_sweeps: int = 4
    post_sweeps: int = 4
    smooth_vec: int = 0
    smooth_sweeps: int = 20
    precond: int = 1
    n_parts: int = 1            # decoupled aggregation over this many row blocks (Sec. 4.1)
    cycle_type: int = 0         # 0 V, 1 H, 2 W
    relax_type: int = 4         # 0 Jacobi, 1 forward/backward GS, 3 symmetrized GS, 4 l1-Jacobi
    coarse_relax: int = 4       # the same codes, for coarse_solver = 1
    max_hrc: int = 1            # bootstrap: most hierarchies in the composite
    bootstrap_type: int = 0     # 0 multiplicative, 1 symmetrized multiplicative, 2 additive
    bootstrap_its: int = 15     # composite iterations on A x = 0 per rate estimate
    bootstrap_seed: int = 1
    bootstrap_rate: float = 0.8  # desired convergence rate of the composite

    def c(self) -> Params:
        return Params(*[float(getattr(self, f.name)) if f.name == "bootstrap_rate"
                        else int(getattr(self, f.name)) for f in fields(self)])


_lib = None
_lib_timing = None


def lib():
    """The parity oracle (sequential)."""
    global _lib
    if _lib is None:
        _lib = _register(C.CDLL(build()))
    return _lib


def lib_timing():
    """The OpenMP timing build (CPU baseline only)."""
    global _lib_timing
    if _lib_timing is None:
        _lib_timing = _register(C.CDLL(build_timing()))
    return _lib_timing


def _register(L):
    if True:
        L.orc_validate.argtypes = [C.c_int32, _i32p, _i32p, _f64p]
        L.orc_spmv.argtypes = [C.c_int32, _i32p, _i32p, _f64p, _f64p, _f64p]
        L.orc_l1_dinv.argtypes = [C.c_int32, _i32p, _i32p, _f64p, _f64p]
        L.orc_edge_weights.argtypes = [C.c_int32, _i32p, _i32p, _f64p, _f64p, _f64p]
        L.orc_match_greedy.argtypes = [C.c_int32, _i32p, _i32p, _f64p, _f64p, _i32p]
        L.orc_match_suitor.argtypes = [C.c_int32, _i32p, _i32p, _f64p, _f64p, _i32p, _i32p]
        L.orc_cholesky.argtypes = [C.c_int32, _f64p, _f64p]
        L.orc_chol_solve.argtypes = [C.c_int32, _f64p, _f64p, _f64p]
        L.orc_setup.restype = C.c_void_p
        L.orc_setup.argtypes = [C.c_int32, _i32p, _i32p, _f64p, C.POINTER(Params), C.c_void_p,
                                C.POINTER(C.c_int)]
        L.orc_free.argtypes = [C.c_void_p]
        L.orc_nlevels.argtypes = [C.c_void_p]
        L.orc_coarse_dense.argtypes = [C.c_void_p]
        L.orc_level_size.argtypes = [C.c_void_p, C.c_int, C.POINTER(C.c_int32),
                                     C.POINTER(C.c_int64)]
        L.orc_opc.restype = C.c_double
        L.orc_opc.argtypes = [C.c_void_p]
        L.orc_export_level.argtypes = [C.c_void_p, C.c_int] + [C.c_void_p] * 7
        L.orc_export_coarse_factor.argtypes = [C.c_void_p, _f64p]
        L.orc_export_coarse_inverse.argtypes = [C.c_void_p, _f64p]
        L.orc_vcycle.argtypes = [C.c_void_p, _f64p, _f64p]
        L.orc_vcycle_f32.argtypes = [C.c_void_p, _f64p, _f64p]
        L.orc_pcg_mixed.argtypes = [C.c_void_p, _f64p, _f64p, C.c_double, C.c_int32,
                                    C.POINTER(C.c_int32), C.POINTER(C.c_double)]
        L.orc_pcg.argtypes = [C.c_void_p, _f64p, _f64p, C.c_double, C.c_int32,
                              C.POINTER(C.c_int32), C.POINTER(C.c_double)]
        L.orc_row_blocks.argtypes = [C.c_int32, C.c_int32, _i32p]
        L.orc_export_part.argtypes = [C.c_void_p, C.c_int, _i32p]
        L.orc_pairwise_step.argtypes = [C.c_int32, _i32p, _i32p, _f64p, _f64p, C.c_void_p, _i32p,
                                        _i32p, _f64p, C.POINTER(C.c_int32),
                                        C.POINTER(C.POINTER(C.c_double)),
                                        C.POINTER(C.POINTER(C.c_int32)),
                                        C.POINTER(C.POINTER(C.c_int32)),
                                        C.POINTER(C.POINTER(C.c_double)),
                                        C.POINTER(C.c_int64)]
        L.orc_free_ptr.argtypes = [C.c_void_p]
        L.orc_nhrc.argtypes = [C.c_void_p]
        L.orc_vcycle_single.argtypes = [C.c_void_p, _f64p, _f64p]
        L.orc_rates.argtypes = [C.c_void_p, _f64p]
        L.orc_component.restype = C.c_void_p
        L.orc_component.argtypes = [C.c_void_p, C.c_int]
    return L


def _csr_args(A):
    return (int(A.n), np.ascontiguousarray(A.row_ptr, np.int32),
            np.ascontiguousarray(A.col, np.int32), np.ascontiguousarray(A.val, np.float64))


def validate(A) -> int:
    return lib().orc_validate(*_csr_args(A))


def spmv(A, x):
    y = np.empty(A.n)
    lib().orc_spmv(*_csr_args(A), np.ascontiguousarray(x, np.float64), y)
    return y


def l1_dinv(A):
    d = np.empty(A.n)
    lib().orc_l1_dinv(*_csr_args(A), d)
    return d


def edge_weights(A, w):
    out = np.empty(A.nnz)
    st = lib().orc_edge_weights(*_csr_args(A), np.ascontiguousarray(w, np.float64), out)
    assert st == OK
    return out


def match_greedy(A, w):
    mate = np.empty(A.n, np.int32)
    st = lib().orc_match_greedy(*_csr_args(A), np.ascontiguousarray(w, np.float64), mate)
    assert st == OK
    return mate


def match_suitor(A, w, order):
    mate = np.empty(A.n, np.int32)
    st = lib().orc_match_suitor(*_csr_args(A), np.ascontiguousarray(w, np.float64),
                                np.ascontiguousarray(order, np.int32), mate)
    assert st == OK
    return mate


def cholesky(D):
    D = np.ascontiguousarray(D, np.float64)
    L = np.empty_like(D)
    st = lib().orc_cholesky(D.shape[0], D, L)
    return st, L


def chol_solve(L, r):
    x = np.empty(L.shape[0])
    lib().orc_chol_solve(L.shape[0], np.ascontiguousarray(L), np.ascontiguousarray(r, np.float64), x)
    return x


def row_blocks(n, n_parts):
    """Row block of each of n rows split into n_parts consecutive blocks (Sec. 4.1)."""
    part = np.empty(n, np.int32)
    assert lib().orc_row_blocks(int(n), int(n_parts), part) == OK
    return part


def pairwise_step(A, w, part=None):
    """One pairwise coarsening step: dict with mate, agg, pval, nc, wc and the coarse CSR.
    part: row block of each row (decoupled aggregation), or None."""
    L = lib()
    n = A.n
    part = None if part is None else np.ascontiguousarray(part, np.int32)
    pp = None if part is None else part.ctypes.data_as(C.c_void_p)
    mate = np.empty(n, np.int32)
    agg = np.empty(n, np.int32)
    pval = np.empty(n)
    nc = C.c_int32()
    wc = C.POINTER(C.c_double)()
    crp = C.POINTER(C.c_int32)()
    cci = C.POINTER(C.c_int32)()
    cv = C.POINTER(C.c_double)()
    cnnz = C.c_int64()
    st = L.orc_pairwise_step(*_csr_args(A), np.ascontiguousarray(w, np.float64), pp, mate, agg, pval,
                             C.byref(nc), C.byref(wc), C.byref(crp), C.byref(cci), C.byref(cv),
                             C.byref(cnnz))
    assert st == OK, st
    m, z = nc.value, cnnz.value
    out = dict(mate=mate, agg=agg, pval=pval, nc=m,
               wc=np.ctypeslib.as_array(wc, (m,)).copy(),
               row_ptr=np.ctypeslib.as_array(crp, (m + 1,)).copy(),
               col=np.ctypeslib.as_array(cci, (max(z, 1),))[:z].copy(),
               val=np.ctypeslib.as_array(cv, (max(z, 1),))[:z].copy())
    for p in (wc, crp, cci, cv):
        L.orc_free_ptr(C.cast(p, C.c_void_p))
    return out


class Hierarchy:
    """Oracle AMG hierarchy: ``Hierarchy(A, AMGParams(...), w=None)``."""

    def __init__(self, A, params: AMGParams | None = None, w=None, timing=False):
        """timing=True: the OpenMP timing build (CPU baseline), not the parity oracle."""
        self.params = params or AMGParams()
        L = self._L = lib_timing() if timing else lib()
        st = C.c_int()
        self._w = None if w is None else np.ascontiguousarray(w, np.float64)
        wp = None if self._w is None else self._w.ctypes.data_as(C.c_void_p)
        cp = self.params.c()
        self.h = L.orc_setup(*_csr_args(A), C.byref(cp), wp, C.byref(st))
        self.status = st.value
        self.n = A.n
        if not self.h:
            raise OracleError(self.status)

    def __del__(self):
        if getattr(self, "h", None) and not getattr(self, "_view", False):
            self._L.orc_free(self.h)
            self.h = None

    @property
    def nhrc(self) -> int:
        """Hierarchies in the bootstrap composite (1 without bootstrap)."""
        return self._L.orc_nhrc(self.h)

    def rates(self):
        """Estimated convergence rates: [j-1] = composite of the first j hierarchies."""
        out = np.empty(16)
        k = self._L.orc_rates(self.h, out)
        return out[:k].copy()

    def component(self, j):
        """Hierarchy j (0-based) of the composite as a non-owning view."""
        v = object.__new__(Hierarchy)
        v._L, v.params, v.n, v.status, v._w = self._L, self.params, self.n, OK, None
        v.h = self._L.orc_component(self.h, int(j))
        assert v.h, "no component %d" % j
        v._view, v._owner = True, self
        return v

    @property
    def nlevels(self) -> int:
        return self._L.orc_nlevels(self.h)

    @property
    def coarse_dense(self) -> bool:
        return bool(self._L.orc_coarse_dense(self.h))

    def level_size(self, k):
        n, z = C.c_int32(), C.c_int64()
        assert self._L.orc_level_size(self.h, k, C.byref(n), C.byref(z)) == OK
        return n.value, z.value

    def sizes(self):
        return [self.level_size(k) for k in range(self.nlevels)]

    def opc(self) -> float:
        return self._L.orc_opc(self.h)

    def level(self, k):
        n, z = self.level_size(k)
        rp = np.empty(n + 1, np.int32)
        ci = np.empty(max(z, 1), np.int32)
        v = np.empty(max(z, 1))
        w = np.empty(n)
        dinv = np.empty(n)
        agg = np.full(n, -1, np.int32)
        pval = np.zeros(n)
        args = [a.ctypes.data_as(C.c_void_p) for a in (rp, ci, v, w, agg, pval, dinv)]
        assert self._L.orc_export_level(self.h, k, *args) == OK
        return dict(n=n, nnz=z, row_ptr=rp, col=ci[:z], val=v[:z], w=w, dinv=dinv,
                    agg=agg if k < self.nlevels - 1 else None,
                    pval=pval if k < self.nlevels - 1 else None)

    def part(self, k):
        """Row block of each row of level k (decoupled aggregation)."""
        n, _ = self.level_size(k)
        out = np.empty(n, np.int32)
        assert self._L.orc_export_part(self.h, k, out) == OK
        return out

    def coarse_factor(self):
        n, _ = self.level_size(self.nlevels - 1)
        Lf = np.empty((n, n))
        assert self._L.orc_export_coarse_factor(self.h, Lf) == OK
        return Lf

    def coarse_inverse(self):
        n, _ = self.level_size(self.nlevels - 1)
        Ai = np.empty((n, n))
        assert self._L.orc_export_coarse_inverse(self.h, Ai) == OK
        return Ai

    def vcycle(self, r, single=False):
        """z = B r: the preconditioner (the bootstrap composite when there is
        one); single=True applies this hierarchy's own V-cycle only."""
        z = np.empty(self.n)
        f = self._L.orc_vcycle_single if single else self._L.orc_vcycle
        assert f(self.h, np.ascontiguousarray(r, np.float64), z) == OK
        return z

    def vcycle_f32(self, r):
        """Mixed-precision form of the V-cycle (binary32 inside, binary64 in/out)."""
        z = np.empty(self.n)
        assert self._L.orc_vcycle_f32(self.h, np.ascontiguousarray(r, np.float64), z) == OK
        return z

    def pcg(self, b, x0=None, rtol=1e-6, maxit=1000, mixed=False):
        """Returns (x, iterations, recurrence relative residual, status)."""
        x = np.zeros(self.n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
        it, rel = C.c_int32(), C.c_double()
        f = self._L.orc_pcg_mixed if mixed else self._L.orc_pcg
        st = f(self.h, np.ascontiguousarray(b, np.float64), x, float(rtol), int(maxit),
               C.byref(it), C.byref(rel))
        return x, it.value, rel.value, st


class OracleError(RuntimeError):
    def __init__(self, status):
        super().__init__("oracle status %d" % status)
        self.status = status
