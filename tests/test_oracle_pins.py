"""Pins of the serial oracle against facts that do not come from the oracle.

Each test names what fixes the result: the undecomposed global assembly, a
brute-force dense build, a hand-derived example, closed-form solutions of the
1D and 3D Poisson problems, dense LU, finite differences for the adjoint, and
(P9) the termination properties of BiCGStab on non-symmetric systems.
"""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import synth
from helpers import (share_ranks, share_values, merged_row_of_natural, oracle_system,
                     random_ldu_values)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

SMALL_CASES = [
    dict(shape=(8, 1, 1), decomp=("blocks", 4, 1, 1), walls=(True, False, False)),
    dict(shape=(4, 4, 4), decomp=("blocks", 2, 2, 2), kappa=(1e-2, 1.0)),
    dict(shape=(5, 4, 3), decomp=("rcb", 3), kappa=(1e-3, 1.0), scramble=True),
    dict(shape=(6, 5, 7), decomp=("rcb", 5), kappa=(1e-3, 1.0), scramble=True, stretch=100.0),
    dict(shape=(6, 6, 4), decomp=("blocks", 3, 2, 1), kappa=(1e-2, 1.0)),
]


def _small(i, seed=100):
    kw = dict(SMALL_CASES[i])
    return synth.small(kw.pop("shape"), kw.pop("decomp"), kappa=kw.pop("kappa", None), seed=seed + i, **kw)


def _csr_rows(m, val):
    for i in range(m.n_rows):
        p0, p1 = m.row_ptr[i], m.row_ptr[i + 1]
        yield i, m.col[p0:p1], val[p0:p1]


def _bits(a):
    return np.asarray(a, dtype=np.float64).view(np.uint64)


# --------------------------------------------------------------------------
# P1: merged matrix == global assembly of the undecomposed mesh, renumbered
# --------------------------------------------------------------------------
@pytest.mark.parametrize("case", range(len(SMALL_CASES)))
def test_p1_global_assembly_identity(case):
    w = _small(case)
    m, buf, val64, *_ = oracle_system(w)
    c = w.coefficients()
    pi = merged_row_of_natural(w)
    # assemble the global matrix face by face, diagonal summed in face order
    entries = {}
    diag = [0.0] * w.n_cells
    for f in range(w.mesh.n_faces):
        a, b, cf = int(w.mesh.face_a[f]), int(w.mesh.face_b[f]), float(c[f])
        if b >= 0:
            entries[(pi[a], pi[b])] = -cf
            entries[(pi[b], pi[a])] = -cf
            diag[b] += cf
        diag[a] += cf
    for a in range(w.n_cells):
        entries[(pi[a], pi[a])] = diag[a]
    assert m.nnz_nonlocal == 0 and m.nnz_local == len(entries)
    for i, cols, vals in _csr_rows(m, val64):
        want = sorted((j, v) for (r, j), v in entries.items() if r == i) if m.n_rows < 50 else None
        if want is None:
            break
        assert list(cols) == [j for j, _ in want]
        assert (_bits(vals) == _bits([v for _, v in want])).all()
    # full comparison through a COO of the global assembly
    keys = np.array(list(entries.keys()), dtype=np.int64)
    vals = np.array(list(entries.values()))
    o = np.lexsort((keys[:, 1], keys[:, 0]))
    rows_ref, cols_ref, vals_ref = keys[o, 0], keys[o, 1], vals[o]
    rows_or = np.repeat(np.arange(m.n_rows), np.diff(m.row_ptr))
    assert (rows_or == rows_ref).all() and (m.col == cols_ref).all()
    assert (_bits(val64[:m.nnz_local]) == _bits(vals_ref)).all()


# --------------------------------------------------------------------------
# P2: brute-force dense build from the per-rank LDU arrays (non-symmetric values)
# --------------------------------------------------------------------------
def _dense_from_ldu(w, values, first, alpha):
    off = np.concatenate([[0], np.cumsum(w.part.n_cells)])
    lo = off[first]
    n_glob = int(off[-1])
    n_rows = int(off[first + alpha] - lo)
    D = np.zeros((n_rows, n_glob))
    for s in range(alpha):
        r = first + s
        d, v = w.part.rank(r), values[r]
        row0 = off[r] - lo
        for c in range(d["n_cells"]):
            D[row0 + c, off[r] + c] = v["diag"][c]
        for f, (o, b) in enumerate(zip(d["owner"], d["neighbour"])):
            D[row0 + o, off[r] + b] = v["upper"][f]
            D[row0 + b, off[r] + o] = v["lower"][f]
        for e, (c, q, dd) in enumerate(zip(d["iface_cell"], d["iface_nbr_rank"], d["iface_nbr_cell"])):
            D[row0 + c, off[q] + dd] = v["iface"][e]
    return D, lo


@pytest.mark.parametrize("case", range(len(SMALL_CASES)))
@pytest.mark.parametrize("sub", [False, True])
def test_p2_brute_force_dense(case, sub):
    w = _small(case)
    rng = np.random.default_rng(case)
    values = random_ldu_values(w, rng)
    first, alpha = (1, max(1, w.n_ranks - 2)) if (sub and w.n_ranks > 2) else (0, w.n_ranks)
    m = oracle.merge(w.part.n_cells, first, alpha, share_ranks(w, first, alpha))
    buf = oracle.receive_buffer(values[first:first + alpha])
    val64, *_ = oracle.update(m, buf)
    D, lo = _dense_from_ldu(w, values, first, alpha)
    got = np.zeros_like(D)
    for i in range(m.n_rows):
        for p in range(m.row_ptr[i], m.row_ptr[i + 1]):
            got[i, lo + m.col[p]] = val64[p]
        for p in range(m.nl_row_ptr[i], m.nl_row_ptr[i + 1]):
            got[i, m.nl_col[p]] = val64[m.nnz_local + p]
    assert (got.view(np.uint64) == D.view(np.uint64)).all()
    # each row: local columns ascending, non-local columns ascending
    for i in range(m.n_rows):
        assert (np.diff(m.col[m.row_ptr[i]:m.row_ptr[i + 1]]) > 0).all()
        assert (np.diff(m.nl_col[m.nl_row_ptr[i]:m.nl_row_ptr[i + 1]]) > 0).all()
    # perm is a bijection onto device positions
    assert (np.sort(m.perm) == np.arange(m.n_slots)).all()


# --------------------------------------------------------------------------
# hand-derived alpha = 2 example (Sec. 3)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("which", ["alpha2", "rank1_alone"])
def test_golden_alpha2_chain(which):
    g = json.load(open(os.path.join(GOLDEN, "alpha2_chain.json")))
    exp = g[which]
    first, alpha = exp["first"], exp["alpha"]
    ranks = [{k: np.array(v, dtype=np.int32) for k, v in g["ranks"][r].items()
              if k in ("owner", "neighbour", "iface_cell", "iface_nbr_rank", "iface_nbr_cell")}
             for r in range(first, first + alpha)]
    m = oracle.merge(g["n_cells_all"], first, alpha, ranks)
    buf = oracle.receive_buffer([g["ranks"][r] for r in range(first, first + alpha)])
    val64, *_ = oracle.update(m, buf)
    assert m.row_ptr.tolist() == exp["row_ptr"]
    assert m.col.tolist() == exp["col"]
    assert m.perm.tolist() == exp["perm"]
    assert m.slot_off.tolist() == exp["slot_off"]
    assert m.nl_row_ptr.tolist() == exp["nl_row_ptr"]
    assert m.nl_col.tolist() == exp["nl_col"]
    assert val64.tolist() == exp["val"]


# --------------------------------------------------------------------------
# P3: special cases
# --------------------------------------------------------------------------
def test_p3_single_rank_is_plain_ldu_to_csr():
    w = synth.small((5, 4, 3), ("blocks", 1, 1, 1), kappa=(1e-2, 1.0), seed=21, scramble=True)
    rng = np.random.default_rng(0)
    values = random_ldu_values(w, rng)
    m = oracle.merge(w.part.n_cells, 0, 1, share_ranks(w))
    assert m.n_slots == m.nnz_local and m.nnz_nonlocal == 0
    assert w.part.if_cell.shape[0] == 0
    val64, *_ = oracle.update(m, oracle.receive_buffer(values))
    d, v = w.part.rank(0), values[0]
    n = d["n_cells"]
    rows = np.concatenate([np.arange(n), d["owner"], d["neighbour"]])
    cols = np.concatenate([np.arange(n), d["neighbour"], d["owner"]])
    data = np.concatenate([v["diag"], v["upper"], v["lower"]])
    ref = sp.coo_matrix((data, (rows, cols)), shape=(n, n)).tocsr()
    ref.sort_indices()
    assert (ref.indptr == m.row_ptr).all() and (ref.indices == m.col).all()
    assert (ref.data.view(np.uint64) == val64.view(np.uint64)).all()


def test_p3_one_cell_per_rank_all_interfaces():
    n = 6
    w = synth.small((n, 1, 1), ("blocks", n, 1, 1), seed=2, walls=(True, False, False))
    assert w.part.owner.shape[0] == 0
    m, buf, val64, *_ = oracle_system(w)
    assert m.nnz_local == n + 2 * (n - 1)
    dense = np.zeros((n, n))
    for i, cols, vals in _csr_rows(m, val64):
        dense[i, cols] = vals
    ref = 2 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    assert (dense == ref).all()


def test_p3_nonlocal_iff_strict_subset():
    w = synth.small((6, 6, 6), ("blocks", 2, 2, 2), seed=4)
    full = oracle.merge(w.part.n_cells, 0, 8, share_ranks(w))
    assert full.nnz_nonlocal == 0
    sub = oracle.merge(w.part.n_cells, 2, 4, share_ranks(w, 2, 4))
    # non-local entries = interface couplings of ranks 2..5 to ranks outside 2..5
    expect = sum(int(np.sum((w.part.rank(r)["iface_nbr_rank"] < 2) | (w.part.rank(r)["iface_nbr_rank"] >= 6)))
                 for r in range(2, 6))
    assert sub.nnz_nonlocal == expect > 0
    lo = int(w.part.cell_ptr[2]); hi = int(w.part.cell_ptr[6])
    assert ((sub.nl_col < lo) | (sub.nl_col >= hi)).all()


def _chain_ranks():
    g = json.load(open(os.path.join(GOLDEN, "alpha2_chain.json")))
    return [{k: np.array(v, dtype=np.int32) for k, v in r.items()
             if k in ("owner", "neighbour", "iface_cell", "iface_nbr_rank", "iface_nbr_cell")}
            for r in g["ranks"]]


@pytest.mark.parametrize("mutation,code", [
    ("self_face", -2), ("owner_range", -2), ("duplicate", -2), ("unpaired", -2),
    ("iface_rank_range", -2), ("iface_self_rank", -2), ("bad_alpha", -1)])
def test_p3_rejects_bad_addressing(mutation, code):
    ranks = _chain_ranks()
    nca, first, alpha = [2, 2], 0, 2
    if mutation == "self_face":
        ranks[0]["neighbour"] = np.array([0], np.int32)
    elif mutation == "owner_range":
        ranks[1]["owner"] = np.array([2], np.int32)
    elif mutation == "duplicate":
        ranks[0]["owner"] = np.array([0, 1], np.int32)
        ranks[0]["neighbour"] = np.array([1, 0], np.int32)
    elif mutation == "unpaired":
        ranks[1]["iface_cell"] = np.array([1], np.int32)
    elif mutation == "iface_rank_range":
        ranks[0]["iface_nbr_rank"] = np.array([5], np.int32)
    elif mutation == "iface_self_rank":
        ranks[0]["iface_nbr_rank"] = np.array([0], np.int32)
    elif mutation == "bad_alpha":
        alpha = 3
        ranks.append(ranks[0])
    with pytest.raises(oracle.OracleError) as e:
        oracle.merge(nca, first, alpha, ranks)
    assert e.value.code == code


# --------------------------------------------------------------------------
# P4: symmetry and positive definiteness
# --------------------------------------------------------------------------
@pytest.mark.parametrize("case", range(len(SMALL_CASES)))
def test_p4_symmetric_positive_definite(case):
    w = _small(case)
    m, buf, val64, val32, d64, d32 = oracle_system(w)
    A = sp.csr_matrix((val64, m.col, m.row_ptr), shape=(m.n_rows, m.n_rows))
    At = A.T.tocsr()
    At.sort_indices()
    assert (At.indptr == A.indptr).all() and (At.indices == A.indices).all()
    assert (At.data.view(np.uint64) == A.data.view(np.uint64)).all()
    dense = A.toarray()
    assert (np.diag(dense) > 0).all()
    np.linalg.cholesky(dense)      # raises unless SPD
    # Jacobi inverse: one IEEE division per row, FP32 copies are RNE casts
    assert (d64 == 1.0 / np.diag(dense)).all()
    assert (d32 == d64.astype(np.float32)).all() and (val32 == val64.astype(np.float32)).all()


# --------------------------------------------------------------------------
# P5: closed-form 3D solutions
# --------------------------------------------------------------------------
def test_p5_sine_eigenvector_one_iteration():
    N = 12
    w = synth.small((N, N, N), ("blocks", 2, 1, 3), seed=1)
    m, buf, val64, *_ = oracle_system(w)
    h = 1.0 / (N + 1)
    p, q, s = 2, 3, 5
    nat = np.arange(w.n_cells)
    i, j, k = nat % N + 1, (nat // N) % N + 1, nat // (N * N) + 1
    v_nat = np.sin(np.pi * p * i * h) * np.sin(np.pi * q * j * h) * np.sin(np.pi * s * k * h)
    lam = 6 - 2 * np.cos(np.pi * p * h) - 2 * np.cos(np.pi * q * h) - 2 * np.cos(np.pi * s * h)
    v = w.merged(v_nat)
    x, st, it, rs, rr = oracle.pcg(m, val64, v, tol=1e-10)
    assert st == 0 and it == 1
    assert np.max(np.abs(x - v / lam)) < 1e-13


def test_p5_manufactured_solution_second_order():
    errs = []
    for N in (7, 15, 31):
        w = synth.small((N, N, N), ("blocks", 1, 1, 2), seed=1)
        m, buf, val64, *_ = oracle_system(w)
        h = 1.0 / (N + 1)
        nat = np.arange(w.n_cells)
        xs = [(nat % N + 1) * h, ((nat // N) % N + 1) * h, (nat // (N * N) + 1) * h]
        u = np.sin(np.pi * xs[0]) * np.sin(np.pi * xs[1]) * np.sin(np.pi * xs[2])
        b = w.merged(h * h * 3 * np.pi ** 2 * u)
        x, st, it, rs, rr = oracle.pcg(m, val64, b, tol=1e-12)
        assert st == 0
        errs.append(np.max(np.abs(x - w.merged(u))))
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(1.8 < r < 2.2 for r in rates), (errs, rates)


def test_p5_two_eigenvalues_two_iterations():
    """Pairs of cells coupled by -rho*sqrt(a*b) make every 2x2 block of
    M^-1 A (M = diag A) have eigenvalues 1 +- rho, so Jacobi-PCG must finish in
    two iterations; plain CG on A, whose spectrum is spread, cannot."""
    m_pairs, rho = 40, 0.5
    rng = np.random.default_rng(12)
    a, b = rng.uniform(1, 100, m_pairs), rng.uniform(1, 100, m_pairs)
    n = 2 * m_pairs
    ranks = [dict(owner=np.arange(0, n, 2, dtype=np.int32), neighbour=np.arange(1, n, 2, dtype=np.int32),
                  iface_cell=np.zeros(0, np.int32), iface_nbr_rank=np.zeros(0, np.int32),
                  iface_nbr_cell=np.zeros(0, np.int32))]
    diag = np.empty(n)
    diag[0::2], diag[1::2] = a, b
    off = -rho * np.sqrt(a * b)
    m = oracle.merge([n], 0, 1, ranks)
    val64, *_ = oracle.update(m, oracle.receive_buffer([dict(diag=diag, upper=off, iface=np.zeros(0))]))
    rhs = rng.uniform(-1, 1, n)
    x, st, it, rs, rr = oracle.pcg(m, val64, rhs, tol=1e-10)
    assert st == 0 and it == 2 and rs == 0
    A = sp.csr_matrix((val64, m.col, m.row_ptr), shape=(n, n)).toarray()
    assert np.linalg.norm(A @ x - rhs) <= 1e-12 * np.linalg.norm(rhs)


# --------------------------------------------------------------------------
# P6: closed-form inverse of tridiag(-1, 2, -1)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n_ranks", [1, 3, 5])
def test_p6_tridiagonal_inverse(n_ranks):
    N = 30
    w = synth.small((N, 1, 1), ("blocks", n_ranks, 1, 1), seed=3, walls=(True, False, False))
    m, buf, val64, *_ = oracle_system(w)
    idx = np.arange(1, N + 1)
    Ainv = np.minimum.outer(idx, idx) * (N + 1 - np.maximum.outer(idx, idx)) / (N + 1)
    rng = np.random.default_rng(6)
    b = rng.uniform(-1, 1, N)
    x, st, it, rs, rr = oracle.pcg(m, val64, b, tol=1e-13)
    assert st == 0 and it <= N
    assert np.max(np.abs(x - Ainv @ b)) < 1e-10 * np.max(np.abs(Ainv @ b))


# --------------------------------------------------------------------------
# P7: dense LU on small irregular systems
# --------------------------------------------------------------------------
@pytest.mark.parametrize("case", range(1, len(SMALL_CASES)))
def test_p7_dense_lu(case):
    w = _small(case, seed=300)
    m, buf, val64, *_ = oracle_system(w)
    A = sp.csr_matrix((val64, m.col, m.row_ptr), shape=(m.n_rows, m.n_rows)).toarray()
    b = w.rhs()
    xl = np.linalg.solve(A, b)
    x, st, it, rs, rr = oracle.pcg(m, val64, b, tol=1e-12)
    assert st == 0 and rr <= 1e-12
    assert np.linalg.norm(x - xl) <= 1e-8 * np.linalg.norm(xl)
    # the oracle's own residual agrees with numpy's
    assert abs(oracle.true_relres(m, val64, b, x) - np.linalg.norm(b - A @ x) / np.linalg.norm(b)) < 1e-14


def test_p7_stopping_rule_and_zero_rhs():
    w = _small(3, seed=301)
    m, buf, val64, *_ = oracle_system(w)
    b = w.rhs()
    for tol in (1e-4, 1e-8):
        x, st, it, rs, rr = oracle.pcg(m, val64, b, tol=tol)
        assert st == 0 and rr <= tol
        # one iteration fewer does not reach the tolerance
        x1, st1, it1, _, rr1 = oracle.pcg(m, val64, b, tol=tol, max_iter=it - 1)
        assert st1 == 1 and it1 == it - 1
    x, st, it, rs, rr = oracle.pcg(m, val64, np.zeros(m.n_rows), x0=np.ones(m.n_rows))
    assert st == 0 and it == 0 and (x == 0).all()


# --------------------------------------------------------------------------
# P9: BiCGStab on non-symmetric (momentum-type) systems
# --------------------------------------------------------------------------
def _momentum_system(case, seed, **kw):
    w = _small(case, seed=seed)
    v = w.momentum_values(**kw)
    m = oracle.merge(w.part.n_cells, 0, w.n_ranks, share_ranks(w))
    val64, *_ = oracle.update(m, oracle.receive_buffer(share_values(w, values=v)))
    A = sp.csr_matrix((val64, m.col, m.row_ptr), shape=(m.n_rows, m.n_rows)).toarray()
    return w, m, val64, A


@pytest.mark.parametrize("case", range(1, len(SMALL_CASES)))
def test_p9_bicgstab_dense_lu(case):
    """Non-symmetric convection-diffusion systems, blocked and scrambled RCB
    numberings: BiCGStab against a dense LU solve."""
    w, m, val64, A = _momentum_system(case, 900, pe=6.0)
    assert np.abs(A - A.T).max() > 1e-3          # genuinely non-symmetric
    b = w.rhs()
    xl = np.linalg.solve(A, b)
    x, st, it, rs, rr = oracle.bicgstab(m, val64, b, tol=1e-12)
    assert st == 0 and rr <= 1e-12
    assert np.linalg.norm(b - A @ x) <= 1e-12 * np.linalg.norm(b) * (1 + 1e-9)
    assert np.linalg.norm(x - xl) <= 1e-8 * np.linalg.norm(xl)


def test_p9_bicgstab_diagonal_one_iteration():
    """M = diag(A) makes A M^-1 = I for a diagonal A: one iteration, x = b / d."""
    n = 37
    rng = np.random.default_rng(91)
    d = rng.uniform(0.5, 50.0, n)
    ranks = [dict(owner=np.zeros(0, np.int32), neighbour=np.zeros(0, np.int32), iface_cell=np.zeros(0, np.int32),
                  iface_nbr_rank=np.zeros(0, np.int32), iface_nbr_cell=np.zeros(0, np.int32))]
    m = oracle.merge([n], 0, 1, ranks)
    val64, *_ = oracle.update(m, oracle.receive_buffer([dict(diag=d, upper=np.zeros(0), iface=np.zeros(0))]))
    b = rng.uniform(-1, 1, n)
    x, st, it, rs, rr = oracle.bicgstab(m, val64, b, tol=1e-8)
    assert st == 0 and it == 1 and rs == 0
    assert np.max(np.abs(x - b / d) / np.abs(b / d)) < 1e-14


def test_p9_bicgstab_two_eigenvalues_two_iterations():
    """Non-symmetric 2x2 blocks [[a, u], [w, e]] with u w = rho^2 a e give
    A M^-1 the eigenvalues 1 +- rho only: the BiCG polynomial of degree two
    annihilates the residual, so BiCGStab ends within two iterations."""
    m_pairs, rho = 40, 0.5
    rng = np.random.default_rng(92)
    a, e = rng.uniform(1, 100, m_pairs), rng.uniform(1, 100, m_pairs)
    s = rng.uniform(0.2, 5.0, m_pairs)                 # u / w: the blocks are not symmetric
    u = -rho * np.sqrt(a * e * s)
    wv = -rho * np.sqrt(a * e / s)
    n = 2 * m_pairs
    ranks = [dict(owner=np.arange(0, n, 2, dtype=np.int32), neighbour=np.arange(1, n, 2, dtype=np.int32),
                  iface_cell=np.zeros(0, np.int32), iface_nbr_rank=np.zeros(0, np.int32),
                  iface_nbr_cell=np.zeros(0, np.int32))]
    diag = np.empty(n)
    diag[0::2], diag[1::2] = a, e
    m = oracle.merge([n], 0, 1, ranks)
    val64, *_ = oracle.update(m, oracle.receive_buffer([dict(diag=diag, upper=u, lower=wv, iface=np.zeros(0))]))
    rhs = rng.uniform(-1, 1, n)
    x, st, it, rs, rr = oracle.bicgstab(m, val64, rhs, tol=1e-10)
    assert st == 0 and it <= 2 and rs == 0
    A = sp.csr_matrix((val64, m.col, m.row_ptr), shape=(n, n)).toarray()
    assert np.abs(A - A.T).max() > 1.0
    assert np.linalg.norm(A @ x - rhs) <= 1e-10 * np.linalg.norm(rhs)


def test_p9_bicgstab_stopping_rule_and_zero_rhs():
    w, m, val64, A = _momentum_system(3, 901)
    b = w.rhs()
    for tol in (1e-4, 1e-8):
        x, st, it, rs, rr = oracle.bicgstab(m, val64, b, tol=tol)
        assert st == 0 and rr <= tol and it >= 2
        x1, st1, it1, _, rr1 = oracle.bicgstab(m, val64, b, tol=tol, max_iter=it - 1)
        assert st1 == 1 and it1 == it - 1 and rr1 > tol
    x, st, it, rs, rr = oracle.bicgstab(m, val64, np.zeros(m.n_rows), x0=np.ones(m.n_rows))
    assert st == 0 and it == 0 and (x == 0).all()


def test_p9_bicgstab_symmetric_agrees_with_cg():
    """On the symmetric pressure matrix both Krylov methods reach the same x."""
    w = _small(4, seed=902)
    m, buf, val64, *_ = oracle_system(w)
    b = w.rhs()
    xc, *_ = oracle.pcg(m, val64, b, tol=1e-12)
    xb, st, it, rs, rr = oracle.bicgstab(m, val64, b, tol=1e-12)
    assert st == 0 and np.linalg.norm(xb - xc) <= 1e-9 * np.linalg.norm(xc)


# --------------------------------------------------------------------------
# P8: adjoint
# --------------------------------------------------------------------------
def _loss_and_state(w, c, xt, tol=1e-13):
    import oracle as o
    vals = synth.ldu_values(w.mesh, w.part, c)
    m = o.merge(w.part.n_cells, 0, w.n_ranks, share_ranks(w))
    val64, *_ = o.update(m, o.receive_buffer(share_values(w, values=vals)))
    x, st, it, rs, rr = o.pcg(m, val64, w.rhs(), tol=tol)
    assert st == 0
    return 0.5 * np.sum((x - xt) ** 2), x, m, val64


def test_p8_adjoint_face_gradient_finite_difference():
    w = synth.build("c4fd")
    xt = w.target()
    c0 = w.coefficients()
    L0, x, m, val64 = _loss_and_state(w, c0, xt)
    lam, st, *_ = oracle.pcg(m, val64, x - xt, tol=1e-13)
    assert st == 0
    pi = merged_row_of_natural(w)
    fb = w.mesh.face_b
    row_b = np.where(fb >= 0, pi[np.maximum(fb, 0)], -1)
    g = oracle.face_grad(pi[w.mesh.face_a], row_b, lam, x)
    rng = np.random.default_rng(44)
    faces = np.concatenate([rng.choice(w.mesh.n_interior, 48, replace=False),
                            rng.choice(np.arange(w.mesh.n_interior, w.mesh.n_faces), 16, replace=False)])
    h = 1e-6
    for f in faces:
        cp, cm = c0.copy(), c0.copy()
        cp[f] += h
        cm[f] -= h
        fd = (_loss_and_state(w, cp, xt)[0] - _loss_and_state(w, cm, xt)[0]) / (2 * h)
        assert abs(fd - g[f]) <= 1e-5 * max(1.0, abs(g[f])), (f, fd, g[f])
    # dL/db = lambda, through a random direction
    db = rng.uniform(-1, 1, m.n_rows)
    b = w.rhs()
    xp, *_ = oracle.pcg(m, val64, b + h * db, tol=1e-13)
    xm, *_ = oracle.pcg(m, val64, b - h * db, tol=1e-13)
    fd = (0.5 * np.sum((xp - xt) ** 2) - 0.5 * np.sum((xm - xt) ** 2)) / (2 * h)
    assert abs(fd - lam @ db) <= 1e-6 * max(1.0, abs(lam @ db))


def test_p8_slot_gradient_dense():
    """Per-slot gradient on a non-symmetric perturbation, with dense solves."""
    w = _small(4, seed=500)
    m, buf, val64, *_ = oracle_system(w)
    n = m.n_rows

    def dense(bf):
        v, *_ = oracle.update(m, bf)
        return sp.csr_matrix((v, m.col, m.row_ptr), shape=(n, n)).toarray()

    b = w.rhs()
    xt = w.target()
    A = dense(buf)
    x = np.linalg.solve(A, b)
    lam = np.linalg.solve(A.T, x - xt)
    g = oracle.value_grad(m, lam, x)
    h = 1e-6
    rng = np.random.default_rng(5)
    for k in rng.choice(m.n_slots, 40, replace=False):
        bp, bm = buf.copy(), buf.copy()
        bp[k] += h
        bm[k] -= h
        Lp = 0.5 * np.sum((np.linalg.solve(dense(bp), b) - xt) ** 2)
        Lm = 0.5 * np.sum((np.linalg.solve(dense(bm), b) - xt) ** 2)
        fd = (Lp - Lm) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k])), (k, fd, g[k])


def test_p8_reciprocity_identity():
    w = _small(2, seed=600)
    m, buf, val64, *_ = oracle_system(w)
    rng = np.random.default_rng(7)
    g, db = rng.uniform(-1, 1, m.n_rows), rng.uniform(-1, 1, m.n_rows)
    lam, *_ = oracle.pcg(m, val64, g, tol=1e-13)
    dx, *_ = oracle.pcg(m, val64, db, tol=1e-13)
    assert abs(lam @ db - g @ dx) <= 1e-10 * max(1.0, abs(lam @ db))


# --------------------------------------------------------------------------
# P11: block-Jacobi preconditioner (blocks of consecutive rows inside a rank)
# --------------------------------------------------------------------------
BJ_SIZES = [1, 2, 3, 4, 8]


def _dense_share(w):
    """The whole-share matrix built straight from the per-rank LDU arrays
    (P2's brute force, independent of the oracle's merge)."""
    vals = [dict(v, lower=v.get("lower", v["upper"])) for v in share_values(w)]
    D, lo = _dense_from_ldu(w, vals, 0, w.n_ranks)
    return D


def _unpack(minv, b, bs, m):
    """Block b of the packed store as a full m x m matrix: entry (i, j),
    i <= j, at i*bs - i*(i-1)/2 + (j-i), mirrored below the diagonal."""
    P = bs * (bs + 1) // 2
    out = np.zeros((m, m))
    for i in range(m):
        for j in range(i, m):
            out[i, j] = out[j, i] = minv[b * P + i * bs - i * (i - 1) // 2 + (j - i)]
    return out


def test_p11_block_starts_hand_derived():
    # ranks of 5, 3, 0 and 4 rows, blocks of 2: no block crosses a rank
    assert oracle.block_starts([5, 3, 0, 4], 2).tolist() == [0, 2, 4, 5, 7, 8, 10, 12]
    assert oracle.block_starts([5, 3, 0, 4], 8).tolist() == [0, 5, 8, 12]
    assert oracle.block_starts([5, 3, 0, 4], 1).tolist() == list(range(13))


@pytest.mark.parametrize("case", range(len(SMALL_CASES)))
@pytest.mark.parametrize("bs", BJ_SIZES)
def test_p11_block_inverse_against_lapack(case, bs):
    w = _small(case, seed=1100)
    m, buf, val64, *_ = oracle_system(w)
    D = _dense_share(w)
    start = oracle.block_starts(w.part.n_cells, bs)
    minv = oracle.block_jacobi_inverse(m, val64, start, bs)
    for b in range(len(start) - 1):
        s0, s1 = start[b], start[b + 1]
        assert 1 <= s1 - s0 <= bs
        Binv = np.linalg.inv(D[s0:s1, s0:s1])
        got = _unpack(minv, b, bs, s1 - s0)
        assert np.abs(got - Binv).max() <= 1e-12 * np.abs(Binv).max(), (b, got, Binv)


@pytest.mark.parametrize("case", range(len(SMALL_CASES)))
def test_p11_block_size_one_is_jacobi(case):
    w = _small(case, seed=1200)
    m, buf, val64, val32, d64, d32 = oracle_system(w)
    start = oracle.block_starts(w.part.n_cells, 1)
    minv = oracle.block_jacobi_inverse(m, val64, start, 1)
    assert np.array_equal(_bits(minv), _bits(d64))          # 1 / diag, one IEEE division
    b = w.rhs()
    x1, st1, it1, *_ = oracle.pcg_block_jacobi(m, val64, b, w.part.n_cells, 1, tol=1e-10)
    x0, st0, it0, *_ = oracle.pcg(m, val64, b, tol=1e-10)
    assert st1 == st0 == 0 and abs(it1 - it0) <= 1
    assert np.linalg.norm(x1 - x0) <= 1e-8 * np.linalg.norm(x0)


@pytest.mark.parametrize("case", range(len(SMALL_CASES)))
@pytest.mark.parametrize("bs", [2, 4, 8])
def test_p11_apply_is_the_block_diagonal_solve(case, bs):
    w = _small(case, seed=1300)
    m, buf, val64, *_ = oracle_system(w)
    D = _dense_share(w)
    start = oracle.block_starts(w.part.n_cells, bs)
    minv = oracle.block_jacobi_inverse(m, val64, start, bs)
    r = np.random.default_rng(case).uniform(-1, 1, m.n_rows)
    z = oracle.block_jacobi_apply(start, bs, minv, r)
    want = np.concatenate([np.linalg.solve(D[s0:s1, s0:s1], r[s0:s1]) for s0, s1 in zip(start[:-1], start[1:])])
    assert np.abs(z - want).max() <= 1e-12 * max(1.0, np.abs(want).max())


def test_p11_one_block_is_the_exact_inverse():
    """A single rank of 8 cells with blocks of 8: M = A, so PCG's first step
    already solves the system."""
    w = synth.small((2, 2, 2), ("blocks", 1, 1, 1), kappa=(1e-2, 1.0), seed=7)
    m, buf, val64, *_ = oracle_system(w)
    b = w.rhs()
    x, st, it, rs, rr = oracle.pcg_block_jacobi(m, val64, b, w.part.n_cells, 8, tol=1e-13)
    A = _dense_share(w)
    assert st == 0 and it == 1
    assert np.linalg.norm(x - np.linalg.solve(A, b)) <= 1e-13 * np.linalg.norm(x)


@pytest.mark.parametrize("case", range(1, len(SMALL_CASES)))
@pytest.mark.parametrize("bs", [2, 4, 8])
def test_p11_block_pcg_dense_lu(case, bs):
    w = _small(case, seed=1400)
    m, buf, val64, *_ = oracle_system(w)
    A = _dense_share(w)
    b = w.rhs()
    xl = np.linalg.solve(A, b)
    x, st, it, rs, rr = oracle.pcg_block_jacobi(m, val64, b, w.part.n_cells, bs, tol=1e-12)
    assert st == 0 and rr <= 1e-12
    assert np.linalg.norm(x - xl) <= 1e-8 * np.linalg.norm(xl)


def test_p11_rejects_indefinite_block():
    """diag 1, coupling -2 inside one block: the second pivot is -3."""
    ranks = [dict(owner=np.array([0], np.int32), neighbour=np.array([1], np.int32),
                  iface_cell=np.zeros(0, np.int32), iface_nbr_rank=np.zeros(0, np.int32),
                  iface_nbr_cell=np.zeros(0, np.int32))]
    m = oracle.merge([2], 0, 1, ranks)
    v64, *_ = oracle.update(m, oracle.receive_buffer([dict(diag=[1.0, 1.0], upper=[-2.0], iface=[])]))
    with pytest.raises(oracle.OracleError):
        oracle.block_jacobi_inverse(m, v64, oracle.block_starts([2], 2), 2)
    x, st, *_ = oracle.pcg_block_jacobi(m, v64, np.ones(2), [2], 2)
    assert st == -6
