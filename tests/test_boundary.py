"""The C-ABI boundary on the CPU: librp.so loads, exports every entry point
include/rp.h declares, and the ctypes structs match the C layouts.  No GPU
call is made here."""
import ctypes
import os
import re
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rp.h")
PKG = os.path.join(ROOT, "paper_2510_08536_amd")


@pytest.fixture(scope="module")
def lib_path():
    path = os.path.join(PKG, "librp.so")
    if not os.path.exists(path):
        import importlib.util
        spec = importlib.util.spec_from_file_location("_rp_build", os.path.join(PKG, "_build.py"))
        mod = importlib.util.module_from_spec(spec)
        spec.loader.exec_module(mod)
        mod.build()
    return path


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|void|const char\*)\s+(rp_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_boundary():
    names = _declared_functions()
    for required in ("rp_plan_create", "rp_update_values", "rp_solve", "rp_value_grad", "rp_plan_destroy"):
        assert required in names


def test_library_exports_every_declared_symbol(lib_path):
    lib = ctypes.CDLL(lib_path)
    missing = [n for n in _declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol(lib_path):
    import paper_2510_08536_amd.rp as rp
    assert sorted(rp.EXPORTED) == _declared_functions()


def test_struct_layouts_match_header(lib_path):
    import paper_2510_08536_amd.rp as rp
    src = r"""
#include <stddef.h>
#include <stdio.h>
#include "rp.h"
#define F(T, m) printf(#T "." #m " %zu\n", offsetof(T, m))
int main(void) {
  printf("rp_rank_desc %zu\n", sizeof(rp_rank_desc));
  printf("rp_solve_opts %zu\n", sizeof(rp_solve_opts));
  printf("rp_solve_info %zu\n", sizeof(rp_solve_info));
  printf("rp_spmv_format %zu\n", sizeof(rp_spmv_format));
  F(rp_rank_desc, n_cells); F(rp_rank_desc, n_faces); F(rp_rank_desc, owner); F(rp_rank_desc, neighbour);
  F(rp_rank_desc, n_iface); F(rp_rank_desc, iface_cell); F(rp_rank_desc, iface_nbr_rank);
  F(rp_rank_desc, iface_nbr_cell);
  F(rp_solve_opts, tol); F(rp_solve_opts, inner_tol); F(rp_solve_opts, update_delta); F(rp_solve_opts, max_iter);
  F(rp_solve_opts, precision);
  F(rp_solve_opts, max_outer); F(rp_solve_opts, check_every); F(rp_solve_opts, x0_zero);
  F(rp_solve_opts, max_restarts); F(rp_solve_opts, method); F(rp_solve_opts, transpose); F(rp_solve_opts, graph);
  F(rp_solve_opts, precond); F(rp_solve_opts, block_size); F(rp_solve_opts, fused_loop);
  printf("rp_device_ptrs %zu\n", sizeof(rp_device_ptrs));
  F(rp_device_ptrs, row_ptr); F(rp_device_ptrs, col); F(rp_device_ptrs, perm); F(rp_device_ptrs, nl_row_ptr);
  F(rp_device_ptrs, nl_col); F(rp_device_ptrs, val64); F(rp_device_ptrs, val32); F(rp_device_ptrs, dinv64);
  F(rp_device_ptrs, dinv32); F(rp_device_ptrs, recv);
  F(rp_solve_info, status); F(rp_solve_info, iters); F(rp_solve_info, outer_iters); F(rp_solve_info, restarts);
  F(rp_solve_info, rel_res);
  F(rp_spmv_format, enabled); F(rp_spmv_format, reserved); F(rp_spmv_format, n_groups);
  F(rp_spmv_format, coded_groups); F(rp_spmv_format, coded_rows); F(rp_spmv_format, coded_nnz);
  F(rp_spmv_format, bytes64); F(rp_spmv_format, bytes32);
  return 0;
}
"""
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "layout.c")
        exe = os.path.join(d, "layout")
        open(c, "w").write(src)
        subprocess.check_call(["gcc", "-std=c11", "-I", os.path.dirname(HEADER), "-o", exe, c])
        out = subprocess.check_output([exe], text=True).split("\n")
    got = dict(line.rsplit(" ", 1) for line in out if line)
    for name, cls in (("rp_rank_desc", rp.rp_rank_desc), ("rp_solve_opts", rp.rp_solve_opts),
                      ("rp_solve_info", rp.rp_solve_info), ("rp_spmv_format", rp.rp_spmv_format),
                      ("rp_device_ptrs", rp.rp_device_ptrs)):
        assert int(got[name]) == ctypes.sizeof(cls), name
        for field, _ in cls._fields_:
            assert int(got[f"{name}.{field}"]) == getattr(cls, field).offset, (name, field)


def test_opts_defaults(lib_path):
    import paper_2510_08536_amd.rp as rp
    o = rp.default_opts()
    assert o.tol == 1e-8 and o.inner_tol == 1e-4 and o.precision == rp.RP_FP64 and o.check_every > 0
    assert o.update_delta == 0.1 and o.max_outer > 0 and o.method == rp.RP_CG and o.transpose == 0 and o.graph == 0
    assert o.precond == rp.RP_PRECOND_JACOBI and o.block_size == 4 and o.fused_loop == 0


def test_missing_library_fails_loudly():
    """The package refuses to import without librp.so: there is no fallback."""
    with tempfile.TemporaryDirectory() as d:
        pkg = os.path.join(d, "paper_2510_08536_amd")
        os.mkdir(pkg)
        for f in ("__init__.py", "rp.py", "autograd.py"):
            open(os.path.join(pkg, f), "w").write(open(os.path.join(PKG, f)).read())
        p = subprocess.run([sys.executable, "-c", "import paper_2510_08536_amd"], cwd=d,
                           capture_output=True, text=True)
    assert p.returncode != 0 and "ImportError" in p.stderr and "not built" in p.stderr


def test_product_does_not_touch_the_oracle():
    for dirpath, _, files in os.walk(PKG):
        if "_build" in dirpath:
            continue
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".hpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "liboracle" not in text and "oracle.c" not in text, f


def _desc(rp, n_cells, n_faces=0, n_iface=0, arr=None):
    d = rp.rp_rank_desc()
    d.n_cells, d.n_faces, d.n_iface = n_cells, n_faces, n_iface
    if arr is not None:
        p = arr.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        d.owner = d.neighbour = d.iface_cell = d.iface_nbr_rank = d.iface_nbr_cell = p
    return d


@pytest.mark.parametrize("case", ["null_out", "no_ranks", "alpha0", "share_past_end", "first_negative",
                                  "ncells_negative", "ncells_mismatch", "faces_negative", "owner_null",
                                  "iface_null", "share_null"])
def test_plan_create_rejects_bad_arguments_on_host(lib_path, case):
    """Argument errors are caught by host-side checks before any HIP call."""
    import numpy as np
    import paper_2510_08536_amd.rp as rp
    arr = np.zeros(4, np.int32)
    nca = (ctypes.c_int32 * 2)(3, 3)
    descs = (rp.rp_rank_desc * 2)(_desc(rp, 3, 1, 1, arr), _desc(rp, 3, 1, 1, arr))
    out = ctypes.c_void_p()
    args = dict(n=2, nca=nca, first=0, alpha=2, share=descs, out=ctypes.byref(out))
    if case == "null_out":
        args["out"] = None
    elif case == "no_ranks":
        args["n"] = 0
    elif case == "alpha0":
        args["alpha"] = 0
    elif case == "share_past_end":
        args["first"] = 1
    elif case == "first_negative":
        args["first"] = -1
    elif case == "ncells_negative":
        nca[1] = -1
    elif case == "ncells_mismatch":
        descs[1].n_cells = 4
    elif case == "faces_negative":
        descs[0].n_faces = -2
    elif case == "owner_null":
        descs[0].owner = None
    elif case == "iface_null":
        descs[1].iface_nbr_cell = None
    elif case == "share_null":
        args["share"] = None
    rc = rp.rp_plan_create(args["n"], nca, args["first"], args["alpha"], args["share"], args["out"])
    assert rc == rp.RP_ERR_ARG, (case, rc, rp.rp_last_error())
    assert rp.rp_last_error()


def test_plan_create_rejects_overflow_on_host(lib_path):
    """A share whose slots reach 2^31 is refused before anything is allocated."""
    import numpy as np
    import paper_2510_08536_amd.rp as rp
    arr = np.zeros(4, np.int32)
    big = 700_000_000          # 3 ranks x (n + 2 * faces) > 2^31 slots
    nca = (ctypes.c_int32 * 3)(big, big, big)
    descs = (rp.rp_rank_desc * 3)(*[_desc(rp, big, big // 2, 0, arr) for _ in range(3)])
    out = ctypes.c_void_p()
    rc = rp.rp_plan_create(3, nca, 0, 3, descs, ctypes.byref(out))
    assert rc == rp.RP_ERR_OVERFLOW and out.value is None


def test_binding_constants_match_the_header(lib_path):
    """Every numeric RP_* constant the binding defines has the header's value."""
    import paper_2510_08536_amd.rp as rp
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    defs = dict(re.findall(r"^#define\s+(RP_\w+)\s+(-?[0-9][0-9.eE+-]*)\s*$", text, flags=re.M))
    assert "RP_LOOP_TWO_MAX_ROWS" in defs and "RP_PRECOND_AMG" in defs
    shared = [k for k in defs if hasattr(rp, k)]
    assert len(shared) >= 20, shared
    wrong = {k: (defs[k], getattr(rp, k)) for k in shared if float(defs[k]) != float(getattr(rp, k))}
    assert not wrong, wrong
