"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

The oracle (gcc) and the library's host code (hipcc, sanitizers on the host
pass only; the GPU code is built as usual) are rebuilt with
-fsanitize=address,undefined and no recovery, loaded into a fresh Python
process with the matching ASan runtime preloaded, and driven through the
paths that run on the host: the oracle's merge, update, solvers, block
inverses and gradients on small meshes; the library's argument checks of
rp_plan_create, the host reverse Cuthill-McKee ordering and the option
defaults.  Any sanitizer report ends that process with a non-zero status."""
import glob
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TESTS = os.path.dirname(os.path.abspath(__file__))
SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1:halt_on_error=1",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def _run(code, preload):
    env = dict(os.environ, LD_PRELOAD=preload, **SAN_ENV)
    env.pop("PYTHONMALLOC", None)
    env["PYTHONMALLOC"] = "malloc"
    return subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=900)


ORACLE_DRIVER = r"""
import sys
sys.path[:0] = [{root!r}, {tests!r}]
import oracle.oracle as om
om.LIB = {lib!r}
om._lib = None
import test_oracle_pins as pins
for c in range(len(pins.SMALL_CASES)):
    pins.test_p1_global_assembly_identity(c)
    pins.test_p2_brute_force_dense(c, True)
    pins.test_p11_block_inverse_against_lapack(c, 3)
    pins.test_p11_apply_is_the_block_diagonal_solve(c, 4)
for c in range(1, len(pins.SMALL_CASES)):
    pins.test_p7_dense_lu(c)
    pins.test_p9_bicgstab_dense_lu(c)
    pins.test_p11_block_pcg_dense_lu(c, 2)
pins.test_p3_single_rank_is_plain_ldu_to_csr()
pins.test_p3_one_cell_per_rank_all_interfaces()
pins.test_p11_rejects_indefinite_block()
pins.test_p8_slot_gradient_dense()
pins.test_p7_stopping_rule_and_zero_rhs()
print("SANITIZED_OK")
"""


def test_oracle_under_asan_ubsan():
    asan = subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()
    if not os.path.exists(asan):
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    with tempfile.TemporaryDirectory() as d:
        lib = os.path.join(d, "liboracle_san.so")
        subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-ffp-contract=off", "-fno-omit-frame-pointer",
                               "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fPIC", "-shared",
                               "-o", lib, os.path.join(ROOT, "oracle", "oracle.c"), "-lm"])
        p = _run(ORACLE_DRIVER.format(root=ROOT, tests=TESTS, lib=lib), asan)
    assert p.returncode == 0 and "SANITIZED_OK" in p.stdout, p.stderr[-3000:]
    assert "runtime error" not in p.stderr and "AddressSanitizer" not in p.stderr, p.stderr[-3000:]


LIB_DRIVER = r"""
import ctypes as C, sys
import numpy as np
lib = C.CDLL({lib!r})
lib.rp_last_error.restype = C.c_char_p
# option defaults
class Opts(C.Structure):
    _fields_ = [("tol", C.c_double), ("inner_tol", C.c_double), ("update_delta", C.c_double),
                ("i", C.c_int32 * 11)]
o = Opts()
lib.rp_solve_opts_default(C.byref(o))
assert o.tol == 1e-8
# reverse Cuthill-McKee on the host: a ring, a grid, a disconnected pattern, an empty one
def csr(n, pairs):
    rows = [[] for _ in range(n)]
    for a, b in pairs:
        rows[a].append(b); rows[b].append(a)
    rp = np.zeros(n + 1, np.int32); col = []
    for i, r in enumerate(rows):
        col += sorted(r); rp[i + 1] = len(col)
    return rp, np.array(col if col else [0], np.int32)
cases = [(8, [(i, (i + 1) % 8) for i in range(8)]),
         (20, [(i, i + 1) for i in range(19) if (i + 1) % 5] + [(i, i + 5) for i in range(15)]),
         (9, [(0, 1), (1, 2), (4, 5), (7, 8)]),
         (3, [])]
for n, pairs in cases:
    rp, col = csr(n, pairs)
    perm = np.zeros(max(n, 1), np.int32)
    rc = lib.rp_rcm_order(n, rp.ctypes.data_as(C.c_void_p), col.ctypes.data_as(C.c_void_p),
                          perm.ctypes.data_as(C.c_void_p))
    assert rc == 0 and sorted(perm[:n].tolist()) == list(range(n)), (rc, perm)
bad = np.array([0, 2, 1], np.int32)
assert lib.rp_rcm_order(2, bad.ctypes.data_as(C.c_void_p), None, None) == -1
# rp_plan_create: argument errors found before any GPU call
class Desc(C.Structure):
    _fields_ = [("n_cells", C.c_int32), ("n_faces", C.c_int32), ("owner", C.c_void_p), ("neighbour", C.c_void_p),
                ("n_iface", C.c_int32), ("iface_cell", C.c_void_p), ("iface_nbr_rank", C.c_void_p),
                ("iface_nbr_cell", C.c_void_p)]
arr = np.zeros(4, np.int32)
p_ = arr.ctypes.data_as(C.c_void_p)
nca = (C.c_int32 * 2)(3, 3)
out = C.c_void_p()
for first, alpha, ncell, nf in ((0, 0, 3, 1), (1, 2, 3, 1), (0, 2, 4, 1), (0, 2, 3, -1)):
    descs = (Desc * 2)(Desc(ncell, nf, p_, p_, 1, p_, p_, p_), Desc(3, 1, p_, p_, 1, p_, p_, p_))
    rc = lib.rp_plan_create(2, nca, first, alpha, descs, C.byref(out))
    assert rc == -1 and lib.rp_last_error(), rc
assert lib.rp_plan_create(2, nca, 0, 2, None, None) == -1
print("SANITIZED_OK")
"""


def test_library_host_code_under_asan_ubsan():
    rt = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
    if not rt:
        pytest.skip("clang's AddressSanitizer runtime is not installed")
    import importlib.util
    spec = importlib.util.spec_from_file_location("_rp_build", os.path.join(ROOT, "paper_2510_08536_amd", "_build.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
    with tempfile.TemporaryDirectory() as d:
        lib = b.build_variant(d, extra_flags=san, link_flags=["-shared-libasan", "-Xarch_host", "-fsanitize=address",
                                                              "-Xarch_host", "-fsanitize=undefined"])
        syms = subprocess.check_output(["nm", "-D", lib], text=True)
        assert "__asan_" in syms and "__ubsan_" in syms, "the variant is not instrumented"
        p = _run(LIB_DRIVER.format(lib=lib), rt[0])
    assert p.returncode == 0 and "SANITIZED_OK" in p.stdout, p.stderr[-3000:]
    assert "runtime error" not in p.stderr and "AddressSanitizer" not in p.stderr, p.stderr[-3000:]
