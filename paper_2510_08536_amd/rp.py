"""Thin ctypes binding of librp.so (argument marshalling only).

The functions named rp_* mirror the C entry points of include/rp.h one to
one; `Plan` wraps them for torch tensors.  Every step of the path runs in the
HIP library: if librp.so is missing this module raises at import, and there
is no fallback.  torch provides device memory and the current stream.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librp.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() (hipcc for gfx950)")

# torch ships its own HIP runtime.  Loading it first makes librp bind to that
# same runtime (the dependency is matched by soname), so torch's allocations,
# streams and librp's kernels share one runtime in the process.
import torch  # noqa: E402,F401

_lib = C.CDLL(LIB_PATH)

# ---- status codes / enums (include/rp.h) ----------------------------------
RP_OK = 0
RP_NOT_CONVERGED = 1
RP_ERR_ARG = -1
RP_ERR_MESH = -2
RP_ERR_OVERFLOW = -3
RP_ERR_HIP = -4
RP_ERR_UNSUPPORTED = -5
RP_ERR_BREAKDOWN = -6
RP_ERR_VALUE = -7
RP_FP64, RP_MIXED, RP_FP32, RP_MIXED_RR = 0, 1, 2, 3
RP_CG, RP_BICGSTAB = 0, 1
RP_KERNEL_SPMV64, RP_KERNEL_SPMV32, RP_KERNEL_SCATTER = 0, 1, 2

STATUS_NAMES = {0: "RP_OK", 1: "RP_NOT_CONVERGED", -1: "RP_ERR_ARG", -2: "RP_ERR_MESH",
                -3: "RP_ERR_OVERFLOW", -4: "RP_ERR_HIP", -5: "RP_ERR_UNSUPPORTED",
                -6: "RP_ERR_BREAKDOWN", -7: "RP_ERR_VALUE"}

EXPORTED = ["rp_plan_create", "rp_plan_destroy", "rp_plan_sizes", "rp_plan_get_csr", "rp_plan_get_values",
            "rp_plan_spmv_windows", "rp_plan_set_spmv_windows", "rp_plan_spmv_format", "rp_plan_set_spmv_format",
            "rp_update_values", "rp_update_values_slots", "rp_spmv", "rp_solve", "rp_solve_opts_default",
            "rp_value_grad", "rp_sync", "rp_last_error", "rp_plan_set_timing", "rp_plan_kernel_stats",
            "rp_plan_set_solve_order", "rp_plan_solve_order", "rp_rcm_order", "rp_plan_device_ptrs",
            "rp_plan_set_vec_grid", "rp_update_values_noalloc", "rp_plan_block_jacobi", "rp_plan_export_recv",
            "rp_recv_attach", "rp_recv_write", "rp_recv_detach", "rp_plan_amg_setup", "rp_plan_amg_levels",
            "rp_plan_amg_level", "rp_plan_amg_coarse_inverse", "rp_plan_amg_apply"]
RP_PRECOND_JACOBI, RP_PRECOND_BLOCK_JACOBI, RP_PRECOND_AMG = 0, 1, 2
RP_BJ_MAX_BLOCK = 8
RP_AMG_OMEGA = 0.8
RP_AMG_COARSE_MAX = 64
RP_AMG_TAIL_ROWS = 1024
RP_LOOP_AUTO, RP_LOOP_COOPERATIVE, RP_LOOP_THREE = 0, 1, 2
RP_LOOP_TWO_MAX_ROWS = 262144
RP_NOALLOC_MAX_RANKS = 4096


class rp_rank_desc(C.Structure):
    _fields_ = [("n_cells", C.c_int32), ("n_faces", C.c_int32),
                ("owner", C.POINTER(C.c_int32)), ("neighbour", C.POINTER(C.c_int32)),
                ("n_iface", C.c_int32),
                ("iface_cell", C.POINTER(C.c_int32)), ("iface_nbr_rank", C.POINTER(C.c_int32)),
                ("iface_nbr_cell", C.POINTER(C.c_int32))]


class rp_solve_opts(C.Structure):
    _fields_ = [("tol", C.c_double), ("inner_tol", C.c_double), ("update_delta", C.c_double), ("max_iter", C.c_int32),
                ("precision", C.c_int32), ("max_outer", C.c_int32), ("check_every", C.c_int32),
                ("x0_zero", C.c_int32), ("max_restarts", C.c_int32), ("method", C.c_int32),
                ("transpose", C.c_int32), ("graph", C.c_int32), ("precond", C.c_int32), ("block_size", C.c_int32),
                ("fused_loop", C.c_int32)]


class rp_solve_info(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters", C.c_int32), ("outer_iters", C.c_int32),
                ("restarts", C.c_int32), ("rel_res", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class rp_device_ptrs(C.Structure):
    _fields_ = [("row_ptr", C.c_void_p), ("col", C.c_void_p), ("perm", C.c_void_p), ("nl_row_ptr", C.c_void_p),
                ("nl_col", C.c_void_p), ("val64", C.c_void_p), ("val32", C.c_void_p), ("dinv64", C.c_void_p),
                ("dinv32", C.c_void_p), ("recv", C.c_void_p)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class rp_ipc_handle(C.Structure):
    _fields_ = [("bytes", C.c_char * 64)]


class rp_spmv_format(C.Structure):
    _fields_ = [("enabled", C.c_int32), ("reserved", C.c_int32), ("n_groups", C.c_int64),
                ("coded_groups", C.c_int64), ("coded_rows", C.c_int64), ("coded_nnz", C.c_int64),
                ("bytes64", C.c_int64), ("bytes32", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


_P = C.c_void_p
_PP = C.POINTER(C.c_void_p)
_i32p = C.POINTER(C.c_int32)
_i64p = C.POINTER(C.c_int64)
_dblp = C.POINTER(C.c_double)

_sig = {
    "rp_plan_create": (C.c_int, [C.c_int32, _i32p, C.c_int32, C.c_int32, C.POINTER(rp_rank_desc), _PP]),
    "rp_plan_destroy": (None, [_P]),
    "rp_plan_sizes": (C.c_int, [_P, _i64p, _i64p, _i64p, _i64p, _i64p]),
    "rp_plan_get_csr": (C.c_int, [_P, _P, _P, _P, _P, _P]),
    "rp_plan_get_values": (C.c_int, [_P, _P, _P, _P, _P]),
    "rp_plan_spmv_windows": (C.c_int, [_P, _i32p, _i32p, _i32p]),
    "rp_plan_set_spmv_windows": (C.c_int, [_P, C.c_int32]),
    "rp_plan_spmv_format": (C.c_int, [_P, C.POINTER(rp_spmv_format)]),
    "rp_plan_set_spmv_format": (C.c_int, [_P, C.c_int32]),
    "rp_update_values": (C.c_int, [_P, _PP, _PP, _PP, _PP, _P]),
    "rp_update_values_slots": (C.c_int, [_P, _P, _P]),
    "rp_update_values_noalloc": (C.c_int, [_P, _PP, _PP, _PP, _PP, _P]),
    "rp_spmv": (C.c_int, [_P, C.c_int32, _P, _P, _P]),
    "rp_solve": (C.c_int, [_P, _P, _P, C.POINTER(rp_solve_opts), C.POINTER(rp_solve_info), _P]),
    "rp_solve_opts_default": (None, [C.POINTER(rp_solve_opts)]),
    "rp_value_grad": (C.c_int, [_P, _P, _P, _P, _P]),
    "rp_sync": (C.c_int, [_P]),
    "rp_last_error": (C.c_char_p, []),
    "rp_plan_set_timing": (C.c_int, [_P, C.c_int32]),
    "rp_plan_kernel_stats": (C.c_int, [_P, C.c_int32, _i64p, _dblp]),
    "rp_plan_set_solve_order": (C.c_int, [_P, C.c_int32]),
    "rp_plan_solve_order": (C.c_int, [_P, _i32p, _P]),
    "rp_rcm_order": (C.c_int, [C.c_int32, _P, _P, _P]),
    "rp_plan_device_ptrs": (C.c_int, [_P, C.POINTER(rp_device_ptrs)]),
    "rp_plan_set_vec_grid": (C.c_int, [_P, C.c_int32]),
    "rp_plan_block_jacobi": (C.c_int, [_P, C.c_int32, _i64p, _P, _P, _P]),
    "rp_plan_export_recv": (C.c_int, [_P, C.POINTER(rp_ipc_handle), _i64p]),
    "rp_recv_attach": (C.c_int, [C.POINTER(rp_ipc_handle), C.POINTER(C.c_void_p)]),
    "rp_recv_write": (C.c_int, [_P, C.c_int64, _P, C.c_int32, _P, C.c_int32, _P, _P, C.c_int32, _P]),
    "rp_recv_detach": (C.c_int, [_P]),
    "rp_plan_amg_setup": (C.c_int, [_P, _P]),
    "rp_plan_amg_levels": (C.c_int, [_P, _i32p]),
    "rp_plan_amg_level": (C.c_int, [_P, C.c_int32, _i64p, _i64p, _P, _P, _P, _P, _P, _P, _P]),
    "rp_plan_amg_coarse_inverse": (C.c_int, [_P, _P]),
    "rp_plan_amg_apply": (C.c_int, [_P, _P, _P, _P]),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args
    globals()[_name] = _f


class RpError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = rp_last_error().decode(errors="replace")
        super().__init__(f"{where}: {STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def _check(code: int, where: str, ok=(RP_OK,)):
    if code not in ok:
        raise RpError(code, where)
    return code


def library_path() -> str:
    return LIB_PATH


# ---------------------------------------------------------------------------
# torch-facing wrapper
# ---------------------------------------------------------------------------
def _torch():
    import torch
    return torch


def _stream_handle(stream=None):
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _ptr(t):
    """Device or host address of a torch tensor or numpy array."""
    if isinstance(t, np.ndarray):
        return C.c_void_p(t.ctypes.data)
    return C.c_void_p(t.data_ptr())


def rcm_order(row_ptr, col) -> np.ndarray:
    """Reverse Cuthill-McKee order of a structurally symmetric CSR pattern
    (host arrays, no device work): perm[k] = the row placed at position k."""
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
    col = np.ascontiguousarray(col, dtype=np.int32)
    n = row_ptr.size - 1
    perm = np.zeros(max(n, 1), np.int32)
    _check(rp_rcm_order(n, _ptr(row_ptr), _ptr(col) if col.size else None, _ptr(perm)), "rp_rcm_order")
    return perm[:n]


def _set_opts(o: rp_solve_opts, **kw) -> rp_solve_opts:
    for k, v in kw.items():
        if k == "precision" and isinstance(v, str):
            v = {"fp64": RP_FP64, "mixed": RP_MIXED, "mixed_rr": RP_MIXED_RR}[v]
        if k == "method" and isinstance(v, str):
            v = {"cg": RP_CG, "bicgstab": RP_BICGSTAB}[v]
        if k == "precond" and isinstance(v, str):
            v = {"jacobi": RP_PRECOND_JACOBI, "block_jacobi": RP_PRECOND_BLOCK_JACOBI, "amg": RP_PRECOND_AMG}[v]
        setattr(o, k, v)
    return o


def default_opts(**kw) -> rp_solve_opts:
    """The library's default options with the named fields changed
    (precision "fp64" / "mixed" / "mixed_rr", method "cg" / "bicgstab")."""
    o = rp_solve_opts()
    rp_solve_opts_default(C.byref(o))
    return _set_opts(o, **kw)


class Plan:
    """One GPU part: the fused pattern of CPU ranks first..first+alpha-1.

    ranks[s] is a mapping with int32 arrays owner, neighbour, iface_cell,
    iface_nbr_rank, iface_nbr_cell (and n_cells) of rank first+s.
    """

    def __init__(self, n_cells_all, first: int, alpha: int, ranks):
        n_cells_all = np.ascontiguousarray(n_cells_all, dtype=np.int32)
        keep = []
        descs = (rp_rank_desc * alpha)()
        for s in range(alpha):
            r = ranks[s]
            arrs = {k: np.ascontiguousarray(r[k], dtype=np.int32)
                    for k in ("owner", "neighbour", "iface_cell", "iface_nbr_rank", "iface_nbr_cell")}
            keep.append(arrs)
            d = descs[s]
            if "n_cells" in r:
                d.n_cells = int(r["n_cells"])
            else:  # a share outside the rank list is reported by rp_plan_create
                d.n_cells = int(n_cells_all[first + s]) if 0 <= first + s < len(n_cells_all) else 0
            d.n_faces = arrs["owner"].shape[0]
            d.n_iface = arrs["iface_cell"].shape[0]
            for k, a in arrs.items():
                setattr(d, k, a.ctypes.data_as(_i32p))
        h = C.c_void_p()
        _check(rp_plan_create(len(n_cells_all), n_cells_all.ctypes.data_as(_i32p), first, alpha, descs,
                              C.byref(h)), "rp_plan_create")
        self._h = h
        self.first, self.alpha = first, alpha
        self.version = 0
        nr, nnz, nnl, ns = C.c_int64(), C.c_int64(), C.c_int64(), C.c_int64()
        so = np.zeros(alpha + 1, np.int64)
        _check(rp_plan_sizes(h, C.byref(nr), C.byref(nnz), C.byref(nnl), C.byref(ns),
                             so.ctypes.data_as(_i64p)), "rp_plan_sizes")
        self.n_rows, self.nnz, self.nnz_nonlocal, self.n_slots = nr.value, nnz.value, nnl.value, ns.value
        self.slot_off = so

    # -- lifetime ---------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            rp_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    # -- pattern / values out ---------------------------------------------
    def spmv_windows(self):
        """(mode, offsets) of the LDS x-window layout found for this pattern."""
        mode, en = C.c_int32(), C.c_int32()
        off = (C.c_int32 * 2)()
        _check(rp_plan_spmv_windows(self._h, C.byref(mode), off, C.byref(en)), "rp_plan_spmv_windows")
        return mode.value, [off[k] for k in range(max(mode.value, 0))]

    def spmv_windows_enabled(self) -> bool:
        en = C.c_int32()
        _check(rp_plan_spmv_windows(self._h, None, None, C.byref(en)), "rp_plan_spmv_windows")
        return bool(en.value)

    def set_spmv_windows(self, enable: bool):
        _check(rp_plan_set_spmv_windows(self._h, int(bool(enable))), "rp_plan_set_spmv_windows")

    def spmv_format(self) -> dict:
        """Column-index form of the SpMV: coded groups, rows, entries and the
        algorithmic bytes of one FP64 / FP32 y = A x in the form in use."""
        f = rp_spmv_format()
        _check(rp_plan_spmv_format(self._h, C.byref(f)), "rp_plan_spmv_format")
        return f.as_dict()

    def set_spmv_format(self, coded: bool):
        _check(rp_plan_set_spmv_format(self._h, int(bool(coded))), "rp_plan_set_spmv_format")

    def set_solve_order(self, mode):
        """0 / "fused": CG and the mixed solvers run on the fused rows;
        1 / "rcm": on the plan's reverse Cuthill-McKee renumbering (built on
        first use).  b and x stay in fused order either way."""
        if isinstance(mode, str):
            mode = {"fused": 0, "rcm": 1}[mode]
        _check(rp_plan_set_solve_order(self._h, int(mode)), "rp_plan_set_solve_order")

    def solve_order(self):
        """(mode, perm): perm[k] = fused row at solve-order position k (None if no order was built)."""
        mode = C.c_int32()
        _check(rp_plan_solve_order(self._h, C.byref(mode), None), "rp_plan_solve_order")
        perm = np.zeros(max(self.n_rows, 1), np.int32)
        rc = rp_plan_solve_order(self._h, None, _ptr(perm))
        return mode.value, (perm[:self.n_rows] if rc == RP_OK else None)

    def get_csr(self):
        row_ptr = np.zeros(self.n_rows + 1, np.int32)
        col = np.zeros(max(self.nnz, 1), np.int32)
        perm = np.zeros(max(self.n_slots, 1), np.int32)
        nl_row_ptr = np.zeros(self.n_rows + 1, np.int32)
        nl_col = np.zeros(max(self.nnz_nonlocal, 1), np.int64)
        _check(rp_plan_get_csr(self._h, _ptr(row_ptr), _ptr(col), _ptr(perm), _ptr(nl_row_ptr), _ptr(nl_col)),
               "rp_plan_get_csr")
        return dict(row_ptr=row_ptr, col=col[:self.nnz], perm=perm[:self.n_slots], nl_row_ptr=nl_row_ptr,
                    nl_col=nl_col[:self.nnz_nonlocal])

    def device_ptrs(self) -> dict:
        """Device addresses of the pattern and value arrays (rp_plan_device_ptrs)."""
        d = rp_device_ptrs()
        _check(rp_plan_device_ptrs(self._h, C.byref(d)), "rp_plan_device_ptrs")
        return d.as_dict()

    def block_jacobi(self, block_size: int):
        """(start, minv64, minv32) of the block-Jacobi preconditioner for the
        current values (built on the GPU; rp_plan_block_jacobi)."""
        nb = C.c_int64()
        _check(rp_plan_block_jacobi(self._h, int(block_size), C.byref(nb), None, None, None), "rp_plan_block_jacobi")
        P = block_size * (block_size + 1) // 2
        start = np.zeros(nb.value + 1, np.int32)
        m64 = np.zeros(max(nb.value * P, 1), np.float64)
        m32 = np.zeros(max(nb.value * P, 1), np.float32)
        _check(rp_plan_block_jacobi(self._h, int(block_size), C.byref(nb), _ptr(start), _ptr(m64), _ptr(m32)),
               "rp_plan_block_jacobi")
        return start, m64[:nb.value * P], m32[:nb.value * P]

    # -- multigrid ---------------------------------------------------------------
    def amg_setup(self, stream=None):
        """Build the multigrid hierarchy from the current values."""
        _check(rp_plan_amg_setup(self._h, _stream_handle(stream)), "rp_plan_amg_setup")

    def amg_levels(self) -> int:
        n = C.c_int32()
        _check(rp_plan_amg_levels(self._h, C.byref(n)), "rp_plan_amg_levels")
        return n.value

    def amg_level(self, level: int) -> dict:
        """Host copies of level `level`: n, row_ptr, col, val, dinv and (all
        but the coarsest) agg, mem_ptr, mem."""
        n, nnz = C.c_int64(), C.c_int64()
        _check(rp_plan_amg_level(self._h, int(level), C.byref(n), C.byref(nnz), *([None] * 7)), "rp_plan_amg_level")
        n, nnz = n.value, nnz.value
        last = level == self.amg_levels() - 1
        nc = 0
        if not last:
            m = C.c_int64()
            _check(rp_plan_amg_level(self._h, int(level) + 1, C.byref(m), None, *([None] * 7)), "rp_plan_amg_level")
            nc = m.value
        d = dict(n=n, row_ptr=np.zeros(n + 1, np.int32), col=np.zeros(max(nnz, 1), np.int32),
                 val=np.zeros(max(nnz, 1)), dinv=np.zeros(max(n, 1)))
        agg, mem_ptr, mem = np.zeros(max(n, 1), np.int32), np.zeros(nc + 1, np.int32), np.zeros(max(n, 1), np.int32)
        _check(rp_plan_amg_level(self._h, int(level), None, None, _ptr(d["row_ptr"]), _ptr(d["col"]), _ptr(d["val"]),
                                 _ptr(d["dinv"]), _ptr(agg), _ptr(mem_ptr), _ptr(mem)), "rp_plan_amg_level")
        d["col"], d["val"], d["dinv"] = d["col"][:nnz], d["val"][:nnz], d["dinv"][:n]
        if not last:
            d.update(agg=agg[:n], mem_ptr=mem_ptr, mem=mem[:n])
        return d

    def amg_coarse_inverse(self) -> np.ndarray:
        nL = self.amg_level(self.amg_levels() - 1)["n"]
        out = np.zeros(max(nL * nL, 1))
        _check(rp_plan_amg_coarse_inverse(self._h, _ptr(out)), "rp_plan_amg_coarse_inverse")
        return out[:nL * nL].reshape(nL, nL)

    def amg_apply(self, r, z=None, stream=None):
        """z = one V-cycle of the multigrid on r (float64 CUDA tensors)."""
        torch = _torch()
        if z is None:
            z = torch.empty_like(r)
        _check(rp_plan_amg_apply(self._h, _ptr(r), _ptr(z), _stream_handle(stream)), "rp_plan_amg_apply")
        return z

    def set_vec_grid(self, blocks: int):
        """Fix the solvers' elementwise-kernel grid (0 = default sizing)."""
        _check(rp_plan_set_vec_grid(self._h, int(blocks)), "rp_plan_set_vec_grid")

    def get_values(self):
        v64 = np.zeros(max(self.n_slots, 1), np.float64)
        v32 = np.zeros(max(self.n_slots, 1), np.float32)
        d64 = np.zeros(max(self.n_rows, 1), np.float64)
        d32 = np.zeros(max(self.n_rows, 1), np.float32)
        _check(rp_plan_get_values(self._h, _ptr(v64), _ptr(v32), _ptr(d64), _ptr(d32)), "rp_plan_get_values")
        return v64[:self.n_slots], v32[:self.n_slots], d64[:self.n_rows], d32[:self.n_rows]

    # -- update -------------------------------------------------------------
    def update(self, diag, upper, iface, lower=None, stream=None):
        """Per-rank value arrays (torch tensors on the GPU or the host, or numpy
        arrays), float64, in each rank's LDU order."""
        A = self.alpha

        def norm(lst):
            if lst is None:
                return None
            assert len(lst) == A, "one array per rank of the share"
            return [np.ascontiguousarray(a, dtype=np.float64) if isinstance(a, np.ndarray) else a for a in lst]

        diag, upper, iface, lower = norm(diag), norm(upper), norm(iface), norm(lower)
        arrs = [diag, upper, iface] + ([lower] if lower is not None else [])
        host = any(isinstance(a, np.ndarray) or not a.is_cuda for lst in arrs for a in lst)

        def table(lst):
            t = (C.c_void_p * A)()
            for i, a in enumerate(lst):
                t[i] = _ptr(a).value
            return t

        td, tu, ti = table(diag), table(upper), table(iface)
        tl = table(lower) if lower is not None else None
        _check(rp_update_values(self._h, C.cast(td, _PP), C.cast(tu, _PP), C.cast(tl, _PP) if tl else None,
                                C.cast(ti, _PP), _stream_handle(stream)), "rp_update_values")
        if host:
            # host arrays may be released by the caller on return
            self.sync()
        self.version += 1

    def update_noalloc(self, diag, upper, iface, lower=None, stream=None):
        """rp_update_values_noalloc: per-rank float64 CUDA tensors; the library
        allocates nothing for the call (its pointer table lives in a fixed
        device array shared by all calls on the GPU)."""
        A = self.alpha

        def table(lst):
            assert len(lst) == A, "one array per rank of the share"
            t = (C.c_void_p * A)()
            for i, a in enumerate(lst):
                t[i] = _ptr(a).value
            return t

        td, tu, ti = table(diag), table(upper), table(iface)
        tl = table(lower) if lower is not None else None
        _check(rp_update_values_noalloc(self._h, C.cast(td, _PP), C.cast(tu, _PP),
                                        C.cast(tl, _PP) if tl else None, C.cast(ti, _PP), _stream_handle(stream)),
               "rp_update_values_noalloc")
        self.version += 1

    def export_recv(self) -> bytes:
        """IPC handle (64 bytes) of the plan's receive buffer, for rank
        processes that write their values straight into it (RecvWriter)."""
        h = rp_ipc_handle()
        _check(rp_plan_export_recv(self._h, C.byref(h), None), "rp_plan_export_recv")
        return C.string_at(C.addressof(h), 64)

    def update_from_recv(self, stream=None):
        """Reorder the plan's own receive buffer (filled by rank processes)."""
        _check(rp_update_values_slots(self._h, C.c_void_p(self.device_ptrs()["recv"]), _stream_handle(stream)),
               "rp_update_values_slots")
        self.version += 1

    def update_slots(self, slots, stream=None):
        """slots: float64 CUDA tensor of n_slots values in receive-buffer order."""
        assert slots.is_cuda and slots.dtype == _torch().float64 and slots.is_contiguous()
        assert slots.numel() == self.n_slots
        _check(rp_update_values_slots(self._h, _ptr(slots), _stream_handle(stream)), "rp_update_values_slots")
        self.version += 1

    def sync(self):
        _check(rp_sync(self._h), "rp_sync")

    # -- kernels --------------------------------------------------------------
    def spmv(self, x, y=None, stream=None):
        torch = _torch()
        prec = RP_FP64 if x.dtype == torch.float64 else RP_FP32
        if y is None:
            y = torch.empty_like(x)
        _check(rp_spmv(self._h, prec, _ptr(x), _ptr(y), _stream_handle(stream)), "rp_spmv")
        return y

    def solve(self, b, x=None, opts=None, stream=None, check=True, **kw):
        """Solve A x = b (b, x float64 CUDA tensors).  Returns (x, info dict).
        opts is read, never changed; keyword arguments set fields of a copy."""
        torch = _torch()
        if opts is None:
            o = default_opts(**kw)
        else:
            o = rp_solve_opts()
            C.memmove(C.byref(o), C.byref(opts), C.sizeof(rp_solve_opts))
            _set_opts(o, **kw)
        if x is None:
            x = torch.zeros_like(b)
            o.x0_zero = 1
        info = rp_solve_info()
        rc = rp_solve(self._h, _ptr(b), _ptr(x), C.byref(o), C.byref(info), _stream_handle(stream))
        if check:
            _check(rc, "rp_solve")
        d = info.as_dict()
        d["status_name"] = STATUS_NAMES.get(rc, rc)
        return x, d

    def value_grad(self, lam, x, g=None, stream=None):
        torch = _torch()
        if g is None:
            g = torch.empty(self.n_slots, dtype=torch.float64, device=x.device)
        _check(rp_value_grad(self._h, _ptr(lam), _ptr(x), _ptr(g), _stream_handle(stream)), "rp_value_grad")
        return g

    # -- timing ---------------------------------------------------------------
    def set_timing(self, enable):
        """False / 0: off; True / 1: HIP events around every launch of the
        timed kernels; n > 1: around every n-th launch."""
        if isinstance(enable, bool):
            enable = int(enable)
        _check(rp_plan_set_timing(self._h, int(enable)), "rp_plan_set_timing")

    def kernel_stats(self, kernel: int):
        n, ms = C.c_int64(), C.c_double()
        _check(rp_plan_kernel_stats(self._h, kernel, C.byref(n), C.byref(ms)), "rp_plan_kernel_stats")
        return n.value, ms.value


class RecvWriter:
    """Rank-process side of the receive buffer: maps the owner's buffer from
    its IPC handle and writes one rank's slot block at a time into it."""

    def __init__(self, handle: bytes):
        h = rp_ipc_handle()
        C.memmove(C.addressof(h), handle, 64)
        ptr = C.c_void_p()
        _check(rp_recv_attach(C.byref(h), C.byref(ptr)), "rp_recv_attach")
        self._ptr = ptr

    def write(self, slot_offset: int, diag, upper, iface, lower=None, stream=None):
        """Host (numpy) or device (torch) float64 arrays of one rank, LDU order."""
        arrs = [diag, upper, iface] + ([lower] if lower is not None else [])
        arrs = [np.ascontiguousarray(a, dtype=np.float64) if isinstance(a, np.ndarray) else a for a in arrs]
        d, u, i = arrs[:3]
        lo = arrs[3] if lower is not None else None
        _check(rp_recv_write(self._ptr, int(slot_offset), _ptr(d), len(d), _ptr(u), len(u),
                             _ptr(lo) if lo is not None else None, _ptr(i), len(i), _stream_handle(stream)),
               "rp_recv_write")

    def close(self):
        if getattr(self, "_ptr", None) is not None:
            rp_recv_detach(self._ptr)
            self._ptr = None
