"""ctypes access to the serial FP64 oracle in oracle.c (test infrastructure only).

Paper sections cited per function; the C source carries the definitions.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "oracle.c")
LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_I32 = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_I64 = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
_F64 = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
_F32 = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"oracle {what} failed with status {code}")
        self.code = code


def build() -> str:
    """Compile the oracle: plain gcc, no FMA contraction, no fast-math."""
    tmp = LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
                           "-fPIC", "-shared", "-o", tmp, SRC, "-lm"])
    os.replace(tmp, LIB)
    return LIB


def loaded_library():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        lib = C.CDLL(LIB)
        lib.or_merge_sizes.argtypes = [C.c_int, _I32, _I32, _I32, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        lib.or_merge.argtypes = [C.c_int, _I32, C.c_int, C.c_int, _I32, _I32, _I32, _I32, _I32, _I32, _I32,
                                 _I32, _I32, _I32, _I64, _I32, _I64, _I32, _I64, _I32, _I64]
        lib.or_update.argtypes = [C.c_int64, C.c_int64, _I32, _I32, _F64, _F64, _F32, _F64, _F32]
        lib.or_spmv.argtypes = [C.c_int64, _I32, _I32, _F64, _F64, _F64]
        lib.or_true_relres.argtypes = [C.c_int64, _I32, _I32, _F64, _F64, _F64]
        lib.or_true_relres.restype = C.c_double
        lib.or_pcg.argtypes = [C.c_int64, _I32, _I32, _F64, _F64, _F64, C.c_double, C.c_int64, C.c_int,
                               _I64, _F64]
        lib.or_bicgstab.argtypes = lib.or_pcg.argtypes
        lib.or_value_grad.argtypes = [C.c_int64, _I32, _I64, C.c_int64, C.c_int64, _F64, _F64, _F64]
        lib.or_face_grad.argtypes = [C.c_int64, _I64, _I64, _F64, _F64, _F64]
        lib.or_block_starts.argtypes = [C.c_int, _I32, C.c_int, C.c_void_p]
        lib.or_block_starts.restype = C.c_int64
        lib.or_block_jacobi_inverse.argtypes = [_I32, _I32, _F64, C.c_int64, _I32, C.c_int, _F64]
        lib.or_block_jacobi_apply.argtypes = [C.c_int64, _I32, C.c_int, _F64, _F64, _F64]
        lib.or_pcg_block_jacobi.argtypes = [C.c_int64, _I32, _I32, _F64, C.c_int, _I32, C.c_int, _F64, _F64,
                                            C.c_double, C.c_int64, C.c_int, _I64, _F64]
        lib.or_amg_build.argtypes = [C.c_int64, _I32, _I32, _F64, C.c_double, C.c_int64, C.POINTER(C.c_int)]
        lib.or_amg_build.restype = C.c_void_p
        lib.or_amg_free.argtypes = [C.c_void_p]
        lib.or_amg_refresh.argtypes = [C.c_void_p, _F64]
        lib.or_amg_levels.argtypes = [C.c_void_p]
        lib.or_amg_level_sizes.argtypes = [C.c_void_p, C.c_int, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        lib.or_amg_level_get.argtypes = [C.c_void_p, C.c_int] + [C.c_void_p] * 7
        lib.or_amg_coarse_inverse.argtypes = [C.c_void_p, _F64]
        lib.or_amg_vcycle.argtypes = [C.c_void_p, _F64, _F64]
        lib.or_pcg_amg.argtypes = [C.c_void_p, _F64, _F64, C.c_double, C.c_int64, C.c_int, _I64, _F64]
        _lib = lib
    return _lib


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _cat(ranks, key):
    parts = [np.asarray(r[key], dtype=np.int32) for r in ranks]
    return np.ascontiguousarray(np.concatenate(parts) if parts else np.zeros(0, np.int32), dtype=np.int32)


@dataclass
class Merged:
    """The three structures of the repartitioning (Sec. 3): pattern, update
    pattern (slot_off) and permutation P (perm), plus slot coordinates."""
    first: int
    alpha: int
    lo: int                 # global id of the first fused row
    n_rows: int
    n_slots: int
    nnz_local: int
    nnz_nonlocal: int
    row_ptr: np.ndarray
    col: np.ndarray
    nl_row_ptr: np.ndarray
    nl_col: np.ndarray
    perm: np.ndarray
    slot_off: np.ndarray
    slot_row: np.ndarray
    slot_col: np.ndarray
    diag_slot: np.ndarray


def merge(n_cells_all, first: int, alpha: int, ranks: list) -> Merged:
    """Fuse the LDU patterns of CPU ranks first..first+alpha-1 (Sec. 3, steps
    1-3, the localisation rule and the three resulting structures).  ranks[s]
    holds owner/neighbour/iface_cell/iface_nbr_rank/iface_nbr_cell of rank
    first+s."""
    lib = loaded_library()
    n_cells_all = _i32(n_cells_all)
    if alpha < 1 or first < 0 or first + alpha > len(n_cells_all) or len(ranks) != alpha:
        raise OracleError(-1, "merge (share outside the rank range)")
    nc_share = _i32([n_cells_all[first + s] for s in range(alpha)])
    nf = _i32([len(r["owner"]) for r in ranks])
    ni = _i32([len(r["iface_cell"]) for r in ranks])
    n_rows, n_slots = C.c_int64(), C.c_int64()
    lib.or_merge_sizes(alpha, nc_share, nf, ni, C.byref(n_rows), C.byref(n_slots))
    nr, ns = n_rows.value, n_slots.value
    row_ptr = np.zeros(nr + 1, np.int32)
    col = np.zeros(max(ns, 1), np.int32)
    nl_row_ptr = np.zeros(nr + 1, np.int32)
    nl_col = np.zeros(max(ns, 1), np.int64)
    perm = np.zeros(max(ns, 1), np.int32)
    slot_off = np.zeros(alpha + 1, np.int64)
    slot_row = np.zeros(max(ns, 1), np.int32)
    slot_col = np.zeros(max(ns, 1), np.int64)
    diag_slot = np.zeros(max(nr, 1), np.int32)
    counts = np.zeros(2, np.int64)
    st = lib.or_merge(len(n_cells_all), n_cells_all, first, alpha, nf,
                      _cat(ranks, "owner"), _cat(ranks, "neighbour"), ni,
                      _cat(ranks, "iface_cell"), _cat(ranks, "iface_nbr_rank"), _cat(ranks, "iface_nbr_cell"),
                      row_ptr, col, nl_row_ptr, nl_col, perm, slot_off, slot_row, slot_col, diag_slot, counts)
    if st != 0:
        raise OracleError(st, "merge")
    nnz, nnz_nl = int(counts[0]), int(counts[1])
    lo = int(np.sum(n_cells_all[:first], dtype=np.int64))
    return Merged(first, alpha, lo, nr, ns, nnz, nnz_nl, row_ptr, col[:nnz].copy(), nl_row_ptr,
                  nl_col[:nnz_nl].copy(), perm[:ns].copy(), slot_off, slot_row[:ns].copy(),
                  slot_col[:ns].copy(), diag_slot[:nr].copy())


def receive_buffer(values: list) -> np.ndarray:
    """The contiguous buffer of the update procedure (Sec. 3): ranks in order,
    each as [diag | upper | lower | interface]; lower = upper when absent."""
    parts = []
    for v in values:
        up = np.asarray(v["upper"], dtype=np.float64)
        lo = up if v.get("lower") is None else np.asarray(v["lower"], dtype=np.float64)
        parts += [np.asarray(v["diag"], dtype=np.float64), up, lo, np.asarray(v["iface"], dtype=np.float64)]
    return np.ascontiguousarray(np.concatenate(parts))


def update(m: Merged, buf: np.ndarray):
    """Reorder the buffer by P (Sec. 3, update procedure) and derive the FP32
    copy and the Jacobi inverse diagonal.  Returns (val64, val32, dinv64, dinv32);
    val arrays hold the local block then the non-local block."""
    lib = loaded_library()
    buf = np.ascontiguousarray(buf, dtype=np.float64)
    assert buf.shape[0] == m.n_slots
    val64 = np.zeros(max(m.n_slots, 1), np.float64)
    val32 = np.zeros(max(m.n_slots, 1), np.float32)
    dinv64 = np.zeros(max(m.n_rows, 1), np.float64)
    dinv32 = np.zeros(max(m.n_rows, 1), np.float32)
    lib.or_update(m.n_rows, m.n_slots, m.perm if m.n_slots else np.zeros(1, np.int32),
                  m.diag_slot if m.n_rows else np.zeros(1, np.int32),
                  buf if m.n_slots else np.zeros(1), val64, val32, dinv64, dinv32)
    return val64[:m.n_slots], val32[:m.n_slots], dinv64[:m.n_rows], dinv32[:m.n_rows]


def spmv(m: Merged, val64: np.ndarray, x: np.ndarray) -> np.ndarray:
    lib = loaded_library()
    y = np.zeros(max(m.n_rows, 1))
    lib.or_spmv(m.n_rows, m.row_ptr, _i32(m.col if m.nnz_local else np.zeros(1)),
                np.ascontiguousarray(val64[:max(m.nnz_local, 1)], dtype=np.float64) if m.nnz_local else np.zeros(1),
                np.ascontiguousarray(x, dtype=np.float64) if m.n_rows else np.zeros(1), y)
    return y[:m.n_rows]


def true_relres(m: Merged, val64, b, x) -> float:
    lib = loaded_library()
    return float(lib.or_true_relres(m.n_rows, m.row_ptr, _i32(m.col),
                                    np.ascontiguousarray(val64[:m.nnz_local], dtype=np.float64),
                                    np.ascontiguousarray(b, dtype=np.float64),
                                    np.ascontiguousarray(x, dtype=np.float64)))


def pcg(m: Merged, val64, b, x0=None, tol=1e-8, max_iter=100000, max_restarts=5):
    """Jacobi-preconditioned CG (the CG of Sec. 4, M = diag(A)).  Returns
    (x, status, iterations, restarts, true relative residual)."""
    lib = loaded_library()
    if m.nnz_nonlocal:
        raise OracleError(-5, "pcg (non-local block present)")
    x = np.zeros(m.n_rows) if x0 is None else np.array(x0, dtype=np.float64)
    out = np.zeros(2, np.int64)
    res = np.zeros(1)
    st = lib.or_pcg(m.n_rows, m.row_ptr, _i32(m.col), np.ascontiguousarray(val64[:m.nnz_local], dtype=np.float64),
                    np.ascontiguousarray(b, dtype=np.float64), x, float(tol), int(max_iter), int(max_restarts),
                    out, res)
    return x, int(st), int(out[0]), int(out[1]), float(res[0])


def bicgstab_csr(row_ptr, col, val, b, x0=None, tol=1e-8, max_iter=100000, max_restarts=5):
    """Jacobi right-preconditioned BiCGStab on a CSR matrix (the momentum
    solver of Sec. 4; van der Vorst 1992, Saad Alg. 7.7).  Returns (x, status,
    iterations, restarts, true relative residual)."""
    lib = loaded_library()
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
    n = row_ptr.shape[0] - 1
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    out = np.zeros(2, np.int64)
    res = np.zeros(1)
    st = lib.or_bicgstab(n, row_ptr, _i32(col), np.ascontiguousarray(val, dtype=np.float64),
                         np.ascontiguousarray(b, dtype=np.float64), x, float(tol), int(max_iter), int(max_restarts),
                         out, res)
    return x, int(st), int(out[0]), int(out[1]), float(res[0])


def bicgstab(m: Merged, val64, b, x0=None, tol=1e-8, max_iter=100000, max_restarts=5):
    """BiCGStab (as bicgstab_csr) on the fused local block."""
    if m.nnz_nonlocal:
        raise OracleError(-5, "bicgstab (non-local block present)")
    return bicgstab_csr(m.row_ptr, m.col[:m.nnz_local], val64[:m.nnz_local], b, x0, tol, max_iter, max_restarts)


def value_grad(m: Merged, lam, x) -> np.ndarray:
    """dL/dv_k = -lambda_row(k) x_col(k) for every receive-buffer slot."""
    lib = loaded_library()
    g = np.zeros(max(m.n_slots, 1))
    lib.or_value_grad(m.n_slots, m.slot_row, m.slot_col, m.lo, m.n_rows,
                      np.ascontiguousarray(lam, dtype=np.float64), np.ascontiguousarray(x, dtype=np.float64), g)
    return g[:m.n_slots]


def face_grad(row_a, row_b, lam, x) -> np.ndarray:
    """dL/dc_f for face coefficients (interior: -(l_a-l_b)(x_a-x_b); wall: -l_a x_a)."""
    lib = loaded_library()
    row_a = np.ascontiguousarray(row_a, dtype=np.int64)
    row_b = np.ascontiguousarray(row_b, dtype=np.int64)
    g = np.zeros(max(row_a.shape[0], 1))
    lib.or_face_grad(row_a.shape[0], row_a, row_b, np.ascontiguousarray(lam, dtype=np.float64),
                     np.ascontiguousarray(x, dtype=np.float64), g)
    return g[:row_a.shape[0]]


def block_starts(n_cells_share, bs: int) -> np.ndarray:
    """First fused row of every block-Jacobi block: each share rank's rows cut
    into runs of bs (the last run of a rank may be shorter); last entry n_rows."""
    lib = loaded_library()
    nc = _i32(n_cells_share)
    nb = lib.or_block_starts(len(nc), nc, int(bs), None)
    start = np.zeros(nb + 1, np.int32)
    lib.or_block_starts(len(nc), nc, int(bs), start.ctypes.data_as(C.c_void_p))
    return start


def block_jacobi_inverse(m: Merged, val64, start, bs: int) -> np.ndarray:
    """Packed upper triangles of the Gauss-Jordan inverses of the diagonal
    blocks (the block-Jacobi preconditioner, Sec. 5 outlook)."""
    lib = loaded_library()
    start = _i32(start)
    nb = start.shape[0] - 1
    minv = np.zeros(max(nb, 1) * (bs * (bs + 1) // 2))
    st = lib.or_block_jacobi_inverse(m.row_ptr, _i32(m.col if m.nnz_local else np.zeros(1)),
                                     np.ascontiguousarray(val64[:max(m.nnz_local, 1)], dtype=np.float64),
                                     nb, start, int(bs), minv)
    if st != 0:
        raise OracleError(st, "block_jacobi_inverse")
    return minv[:nb * (bs * (bs + 1) // 2)]


def block_jacobi_apply(start, bs: int, minv, r) -> np.ndarray:
    """z = M^-1 r with the packed block inverses."""
    lib = loaded_library()
    start = _i32(start)
    r = np.ascontiguousarray(r, dtype=np.float64)
    z = np.zeros(max(r.shape[0], 1))
    lib.or_block_jacobi_apply(start.shape[0] - 1, start, int(bs),
                              np.ascontiguousarray(minv, dtype=np.float64) if len(minv) else np.zeros(1),
                              r if r.shape[0] else np.zeros(1), z)
    return z[:r.shape[0]]


def pcg_block_jacobi(m: Merged, val64, b, n_cells_share, bs: int, x0=None, tol=1e-8, max_iter=100000,
                     max_restarts=5):
    """PCG (as pcg) with the block-Jacobi preconditioner of block size bs.
    Returns (x, status, iterations, restarts, true relative residual)."""
    lib = loaded_library()
    if m.nnz_nonlocal:
        raise OracleError(-5, "pcg_block_jacobi (non-local block present)")
    x = np.zeros(m.n_rows) if x0 is None else np.array(x0, dtype=np.float64)
    out = np.zeros(2, np.int64)
    res = np.zeros(1)
    nc = _i32(n_cells_share)
    st = lib.or_pcg_block_jacobi(m.n_rows, m.row_ptr, _i32(m.col),
                                 np.ascontiguousarray(val64[:m.nnz_local], dtype=np.float64), len(nc), nc, int(bs),
                                 np.ascontiguousarray(b, dtype=np.float64), x, float(tol), int(max_iter),
                                 int(max_restarts), out, res)
    return x, int(st), int(out[0]), int(out[1]), float(res[0])


class AmgHierarchy:
    """Aggregation multigrid hierarchy of the fused local block (the
    multigrid preconditioner of the Sec. 5 outlook; the C source states the
    aggregation, the Galerkin products and the V-cycle).  build() takes the
    aggregates from the values given; refresh() keeps them and recomputes
    every coarse value for new level-0 values on the same pattern."""

    def __init__(self, m: Merged, val64, omega: float = 0.8, coarse_max: int = 64):
        lib = loaded_library()
        if m.nnz_nonlocal:
            raise OracleError(-5, "AmgHierarchy (non-local block present)")
        self._lib = lib
        self.n = m.n_rows
        self.omega = float(omega)
        st = C.c_int(0)
        col = _i32(m.col[:m.nnz_local]) if m.nnz_local else np.zeros(1, np.int32)
        val = np.ascontiguousarray(val64[:max(m.nnz_local, 1)], dtype=np.float64)
        self._h = lib.or_amg_build(m.n_rows, m.row_ptr, col, val, self.omega, int(coarse_max), C.byref(st))
        if not self._h:
            raise OracleError(st.value, "amg_build")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.or_amg_free(h)
            self._h = None

    def refresh(self, val64):
        st = self._lib.or_amg_refresh(self._h, np.ascontiguousarray(val64, dtype=np.float64))
        if st != 0:
            raise OracleError(st, "amg_refresh")

    @property
    def n_levels(self) -> int:
        return self._lib.or_amg_levels(self._h)

    def level(self, l: int) -> dict:
        """Level l: n, row_ptr, col, val, dinv, and (all but the coarsest)
        agg, mem_ptr, mem."""
        n, nnz = C.c_int64(), C.c_int64()
        self._lib.or_amg_level_sizes(self._h, l, C.byref(n), C.byref(nnz))
        n, nnz = n.value, nnz.value
        d = dict(n=n, row_ptr=np.zeros(n + 1, np.int32), col=np.zeros(max(nnz, 1), np.int32),
                 val=np.zeros(max(nnz, 1)), dinv=np.zeros(max(n, 1)))
        last = l == self.n_levels - 1
        nc = 0 if last else self.level_size(l + 1)
        agg = np.zeros(max(n, 1), np.int32)
        mem_ptr = np.zeros(nc + 1, np.int32)
        mem = np.zeros(max(n, 1), np.int32)
        P = C.c_void_p
        self._lib.or_amg_level_get(self._h, l, d["row_ptr"].ctypes.data_as(P), d["col"].ctypes.data_as(P),
                                   d["val"].ctypes.data_as(P), d["dinv"].ctypes.data_as(P),
                                   agg.ctypes.data_as(P), mem_ptr.ctypes.data_as(P), mem.ctypes.data_as(P))
        d["col"], d["val"], d["dinv"] = d["col"][:nnz], d["val"][:nnz], d["dinv"][:n]
        if not last:
            d.update(agg=agg[:n], mem_ptr=mem_ptr, mem=mem[:n])
        return d

    def level_size(self, l: int) -> int:
        n, nnz = C.c_int64(), C.c_int64()
        self._lib.or_amg_level_sizes(self._h, l, C.byref(n), C.byref(nnz))
        return n.value

    def coarse_inverse(self) -> np.ndarray:
        nL = self.level_size(self.n_levels - 1)
        out = np.zeros(max(nL * nL, 1))
        self._lib.or_amg_coarse_inverse(self._h, out)
        return out[:nL * nL].reshape(nL, nL)

    def vcycle(self, r) -> np.ndarray:
        r = np.ascontiguousarray(r, dtype=np.float64)
        y = np.zeros(max(self.n, 1))
        self._lib.or_amg_vcycle(self._h, r if r.shape[0] else np.zeros(1), y)
        return y[:self.n]

    def pcg(self, b, x0=None, tol=1e-8, max_iter=100000, max_restarts=5):
        """PCG (as pcg) with z = V-cycle(r) on the hierarchy's level-0
        matrix.  Returns (x, status, iterations, restarts, true rel. res.)."""
        x = np.zeros(self.n) if x0 is None else np.array(x0, dtype=np.float64)
        out = np.zeros(2, np.int64)
        res = np.zeros(1)
        st = self._lib.or_pcg_amg(self._h, np.ascontiguousarray(b, dtype=np.float64), x, float(tol),
                                  int(max_iter), int(max_restarts), out, res)
        return x, int(st), int(out[0]), int(out[1]), float(res[0])
