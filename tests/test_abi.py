"""The C ABI boundary, checked without a GPU: the header compiles as C,
every function it declares is exported by libamg355.so with the binding's
signature, and the ctypes structures match the C layout."""
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "amg355.h")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(amg_[a-z_]+)\s*\(", src)))


def test_header_compiles_as_c(tmp_path):
    c = tmp_path / "t.c"
    c.write_text('#include "amg355.h"\nint main(void){amg_params p; return amg_params_default(&p);}\n')
    subprocess.check_call(["gcc", "-std=c99", "-Wall", "-Werror", "-fsyntax-only",
                           "-I", os.path.dirname(HEADER), str(c)])


def test_library_exports_every_declared_symbol():
    import paper_2303_02352_amd as amd
    L = amd.load()
    decl = _declared_functions()
    assert decl, "no declarations found"
    for name in decl:
        assert hasattr(L, name), name
    assert set(decl) == set(amd.EXPORTS), (set(decl) ^ set(amd.EXPORTS))


def test_struct_layouts_match_c(tmp_path):
    import ctypes as C
    import paper_2303_02352_amd as amd
    prog = tmp_path / "layout.c"
    prog.write_text(r'''
#include <stdio.h>
#include <stddef.h>
#include "amg355.h"
int main(void) {
  printf("%zu %zu %zu %zu\n", sizeof(amg_csr), offsetof(amg_csr, nnz), offsetof(amg_csr, val), offsetof(amg_csr, on_device));
  printf("%zu %zu %zu\n", sizeof(amg_params), offsetof(amg_params, smooth_vector), offsetof(amg_params, stream));
  printf("%zu %zu %zu %zu\n", sizeof(amg_info_t), offsetof(amg_info_t, nnz), offsetof(amg_info_t, opc), offsetof(amg_info_t, device_bytes));
  printf("%zu %zu %zu %zu %zu\n", sizeof(amg_batch_info_t), offsetof(amg_batch_info_t, nnz), offsetof(amg_batch_info_t, cols_per_lane_corr), offsetof(amg_batch_info_t, tile_rows), offsetof(amg_batch_info_t, spmm_cols));
  return 0;
}
''')
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.dirname(HEADER), str(prog), "-o", str(exe)])
    out = subprocess.check_output([str(exe)]).decode().split("\n")
    a = list(map(int, out[0].split()))
    assert a == [C.sizeof(amd.amg_csr), amd.amg_csr.nnz.offset, amd.amg_csr.val.offset,
                 amd.amg_csr.on_device.offset]
    b = list(map(int, out[1].split()))
    assert b == [C.sizeof(amd.amg_params), amd.amg_params.smooth_vector.offset,
                 amd.amg_params.stream.offset]
    c = list(map(int, out[2].split()))
    assert c == [C.sizeof(amd.amg_info_t), amd.amg_info_t.nnz.offset, amd.amg_info_t.opc.offset,
                 amd.amg_info_t.device_bytes.offset]
    d = list(map(int, out[3].split()))
    assert d == [C.sizeof(amd.amg_batch_info_t), amd.amg_batch_info_t.nnz.offset,
                 amd.amg_batch_info_t.cols_per_lane_corr.offset, amd.amg_batch_info_t.tile_rows.offset,
                 amd.amg_batch_info_t.spmm_cols.offset]


def test_defaults_and_strings_without_gpu():
    import paper_2303_02352_amd as amd
    p = amd.default_params()
    assert (p.aggr_steps, p.max_levels, p.coarse_max, p.pre_sweeps, p.post_sweeps) == (2, 40, 100, 4, 4)
    assert p.coarse_solver == amd.AMG_COARSE_CHOLESKY and p.precision == amd.AMG_PREC_DOUBLE
    L = amd.load()
    assert L.amg_strerror(amd.AMG_ERR_NOT_SPD)
    assert L.amg_setup(None, None, None) == amd.AMG_ERR_INVALID
    assert b"NULL" in L.amg_last_error()


def test_binding_has_no_compute_fallback():
    src = open(os.path.join(ROOT, "paper_2303_02352_amd", "__init__.py")).read()
    assert "import oracle" not in src and "from oracle" not in src
    for f in os.listdir(os.path.join(ROOT, "paper_2303_02352_amd", "csrc")):
        assert "oracle" not in open(os.path.join(ROOT, "paper_2303_02352_amd", "csrc", f)).read().lower()


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU; --gpus N > 1 exits with a message before
    touching a device."""
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and "--gpus 1" in r.stderr
