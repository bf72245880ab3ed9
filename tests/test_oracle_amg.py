"""P12: pins of the oracle's aggregation multigrid preconditioner (the
multigrid option of the Sec. 5 outlook) against facts that do not come from
the oracle: hand-derived aggregates and coarse matrices of small chains, the
Galerkin product P^T A P formed densely, the V-cycle operator written as the
textbook two-grid product of dense matrices, the exact inverse when no
coarsening happens, symmetry and positive definiteness of M^-1, and dense LU
for the preconditioned solve."""
import numpy as np
import pytest

import oracle
import synth
from helpers import oracle_system

OMEGA = 0.8


def _chain(couplings):
    """1D chain, one rank: coupling c_f > 0 between cells f and f + 1
    (entry -c_f), diagonal 1 + the couplings of the cell."""
    n = len(couplings) + 1
    ranks = [dict(owner=np.arange(n - 1, dtype=np.int32), neighbour=np.arange(1, n, dtype=np.int32),
                  iface_cell=np.zeros(0, np.int32), iface_nbr_rank=np.zeros(0, np.int32),
                  iface_nbr_cell=np.zeros(0, np.int32))]
    c = np.asarray(couplings, dtype=np.float64)
    diag = np.ones(n)
    diag[:-1] += c
    diag[1:] += c
    m = oracle.merge([n], 0, 1, ranks)
    v64, *_ = oracle.update(m, oracle.receive_buffer([dict(diag=diag, upper=-c, iface=[])]))
    return m, v64


def _dense(lv):
    n = lv["n"]
    A = np.zeros((n, n))
    for i in range(n):
        for p in range(lv["row_ptr"][i], lv["row_ptr"][i + 1]):
            A[i, lv["col"][p]] = lv["val"][p]
    return A


def _prolongation(agg, nc):
    P = np.zeros((len(agg), nc))
    P[np.arange(len(agg)), agg] = 1.0
    return P


MESHES = {
    "cube8_const": lambda: synth.small((8, 8, 8), ("blocks", 2, 1, 1), seed=40),
    "ragged_rcb": lambda: synth.small((9, 7, 6), ("rcb", 3), kappa=(1e-3, 1.0), seed=41, scramble=True),
    "slab_stretched": lambda: synth.small((10, 8, 9), ("blocks", 1, 1, 3), kappa=(1e-2, 1.0), seed=42,
                                          stretch=50.0),
    "box27": lambda: synth.small((8, 7, 6), ("blocks", 2, 1, 1), kappa=(1e-2, 1.0), seed=43, stencil=27),
}


def _hier(name, **kw):
    w = MESHES[name]()
    m, buf, v64, *_ = oracle_system(w)
    return w, m, v64, oracle.AmgHierarchy(m, v64, omega=OMEGA, **kw)


# --------------------------------------------------------------------------
# hand-derived aggregates and coarse matrices
# --------------------------------------------------------------------------
def test_p12_chain4_pair_and_joiners():
    """couplings 1, 3, 2: rows 1 and 2 pick each other (3 is the strongest
    coupling of both), rows 0 and 3 find no unmatched neighbour in the next
    round and join that pair: one aggregate, the 1x1 coarse matrix is the
    sum of all entries = the sum of the added 1s = 4."""
    m, v = _chain([1.0, 3.0, 2.0])
    h = oracle.AmgHierarchy(m, v, omega=OMEGA, coarse_max=1)
    assert h.n_levels == 2
    l0 = h.level(0)
    assert list(l0["agg"]) == [0, 0, 0, 0]
    assert list(l0["mem_ptr"]) == [0, 4] and list(l0["mem"]) == [0, 1, 2, 3]
    l1 = h.level(1)
    assert l1["n"] == 1 and list(l1["val"]) == [4.0]
    assert h.coarse_inverse()[0, 0] == 0.25


def test_p12_chain6_two_pairs():
    """couplings 1, 5, 1, 5, 1: pairs (1, 2) and (3, 4) in round one; rows 0
    and 5 join them.  Coarse matrix by hand: [[4, -1], [-1, 4]] (within an
    aggregate the diagonals 2 + 7 + 7 and twice the couplings -1 and -5);
    the next level matches the two coarse rows (-1 < 0) into one row of
    value 4 + 4 - 2 = 6."""
    m, v = _chain([1.0, 5.0, 1.0, 5.0, 1.0])
    h = oracle.AmgHierarchy(m, v, omega=OMEGA, coarse_max=1)
    assert [h.level_size(l) for l in range(h.n_levels)] == [6, 2, 1]
    assert list(h.level(0)["agg"]) == [0, 0, 0, 1, 1, 1]
    l1 = h.level(1)
    assert list(l1["row_ptr"]) == [0, 2, 4] and list(l1["col"]) == [0, 1, 0, 1]
    assert list(l1["val"]) == [4.0, -1.0, -1.0, 4.0]
    assert list(l1["dinv"]) == [0.25, 0.25]
    assert list(h.level(2)["val"]) == [6.0]


def test_p12_positive_couplings_never_match():
    """A row whose only off-diagonal entry is positive stays alone; with no
    aggregate formed at all, coarsening stalls and the build reports it."""
    ranks = [dict(owner=np.array([0], np.int32), neighbour=np.array([1], np.int32),
                  iface_cell=np.zeros(0, np.int32), iface_nbr_rank=np.zeros(0, np.int32),
                  iface_nbr_cell=np.zeros(0, np.int32))]
    m = oracle.merge([2], 0, 1, ranks)
    v, *_ = oracle.update(m, oracle.receive_buffer([dict(diag=[3.0, 3.0], upper=[1.0], iface=[])]))
    with pytest.raises(oracle.OracleError) as e:
        oracle.AmgHierarchy(m, v, coarse_max=1)
    assert e.value.code == -5


# --------------------------------------------------------------------------
# the Galerkin product and the aggregates on real meshes
# --------------------------------------------------------------------------
@pytest.mark.parametrize("name", sorted(MESHES))
def test_p12_galerkin_is_dense_ptap(name):
    w, m, v, h = _hier(name, coarse_max=8)
    assert h.n_levels >= 3
    for l in range(h.n_levels - 1):
        f, c = h.level(l), h.level(l + 1)
        nc = c["n"]
        agg = f["agg"]
        assert agg.min() == 0 and agg.max() == nc - 1
        # members: the rows of each aggregate, ascending
        for I in range(nc):
            assert list(f["mem"][f["mem_ptr"][I]:f["mem_ptr"][I + 1]]) == list(np.flatnonzero(agg == I))
        P = _prolongation(agg, nc)
        A = _dense(f)
        Ac = P.T @ A @ P
        S = (P.T @ (A != 0).astype(float) @ P) != 0      # structural pattern
        got = _dense(c)
        assert np.array_equal(np.argwhere(S), _pattern(c))
        assert np.allclose(got, Ac, rtol=1e-13, atol=1e-13 * np.abs(Ac).max())
        assert np.array_equal(c["dinv"], 1.0 / np.diag(got))
        # every aggregate of two or more rows is connected through negative couplings
        for I in range(nc):
            rows = np.flatnonzero(agg == I)
            if len(rows) > 1:
                sub = (A[np.ix_(rows, rows)] < 0)
                seen, stack = {0}, [0]
                while stack:
                    a = stack.pop()
                    for b in np.flatnonzero(sub[a]):
                        if b not in seen:
                            seen.add(b)
                            stack.append(b)
                assert len(seen) == len(rows)
    assert h.level_size(h.n_levels - 1) <= 8


def _pattern(lv):
    rows = np.repeat(np.arange(lv["n"]), np.diff(lv["row_ptr"]))
    return np.stack([rows, lv["col"]], axis=1)


# --------------------------------------------------------------------------
# the V-cycle operator
# --------------------------------------------------------------------------
def _vcycle_dense(h):
    """M^-1 from the levels' matrices and aggregates by the textbook
    products: coarsest A^-1 (numpy); odd level P V P^T; even level
    S + (I - S A)(S + P V P^T (I - A S)), S = omega D^-1."""
    L = h.n_levels
    V = np.linalg.inv(_dense(h.level(L - 1)))
    for l in range(L - 2, -1, -1):
        lv = h.level(l)
        P = _prolongation(lv["agg"], V.shape[0])
        C = P @ V @ P.T
        if l % 2 == 1:
            V = C
        else:
            A = _dense(lv)
            S = np.diag(OMEGA / np.diag(A))
            I = np.eye(lv["n"])
            V = S + (I - S @ A) @ (S + C @ (I - A @ S))
    return V


def _probe(h):
    n = h.n
    return np.stack([h.vcycle(e) for e in np.eye(n)], axis=1)


@pytest.mark.parametrize("name,coarse_max", [("cube8_const", 256), ("ragged_rcb", 256), ("box27", 100),
                                             ("slab_stretched", 40)])
def test_p12_vcycle_is_the_multigrid_product(name, coarse_max):
    w, m, v, h = _hier(name, coarse_max=coarse_max)
    assert h.n_levels >= 2
    M = _probe(h)
    Md = _vcycle_dense(h)
    assert np.allclose(M, Md, rtol=1e-10, atol=1e-12 * np.abs(Md).max())
    # symmetric positive definite
    assert np.abs(M - M.T).max() <= 1e-12 * np.abs(M).max()
    assert np.linalg.eigvalsh(0.5 * (M + M.T)).min() > 0


def test_p12_hierarchies_of_two_and_three_levels():
    """The product test above covers an odd (unsmoothed) level only when the
    hierarchy has three or more levels: make sure the cases do."""
    sizes = {name: _hier(name, coarse_max=cm)[3].n_levels
             for name, cm in (("cube8_const", 256), ("box27", 100), ("slab_stretched", 40))}
    assert sizes["cube8_const"] == 2 and sizes["box27"] >= 3 and sizes["slab_stretched"] >= 4


def test_p12_no_coarsening_is_the_exact_inverse():
    w = synth.small((6, 5, 4), ("blocks", 2, 1, 1), kappa=(1e-2, 1.0), seed=44)
    m, buf, v, *_ = oracle_system(w)
    h = oracle.AmgHierarchy(m, v, omega=OMEGA, coarse_max=256)
    assert h.n_levels == 1
    A = _dense(h.level(0))
    r = np.random.default_rng(0).uniform(-1, 1, m.n_rows)
    assert np.allclose(h.vcycle(r), np.linalg.solve(A, r), rtol=1e-11, atol=1e-13)
    x, st, it, rs, rr = h.pcg(w.rhs(), tol=1e-8)
    assert st == 0 and it == 1 and rr <= 1e-8


@pytest.mark.parametrize("name", sorted(MESHES))
def test_p12_amg_pcg_dense_lu(name):
    w, m, v, h = _hier(name, coarse_max=32)
    A = _dense(h.level(0))
    b = w.rhs()
    x_lu = np.linalg.solve(A, b)
    x, st, it, rs, rr = h.pcg(b, tol=1e-10)
    _, _, it_j, _, _ = oracle.pcg(m, v, b, tol=1e-10)
    assert st == 0 and rs == 0 and rr <= 1e-10
    assert np.linalg.norm(x - x_lu) <= 1e-7 * np.linalg.norm(x_lu)
    assert it < it_j


def test_p12_refresh_keeps_aggregates_and_recomputes_values():
    w = synth.small((9, 7, 6), ("rcb", 3), kappa=(1e-3, 1.0), seed=41, scramble=True, timesteps=3)
    m, buf, v0, *_ = oracle_system(w, t=0)
    _, _, v1, *_ = oracle_system(w, t=1)
    h = oracle.AmgHierarchy(m, v0, omega=OMEGA, coarse_max=8)
    aggs = [h.level(l)["agg"].copy() for l in range(h.n_levels - 1)]
    h.refresh(v1)
    A = _dense(h.level(0))
    assert np.array_equal(h.level(0)["val"], v1[:m.nnz_local])
    for l in range(h.n_levels - 1):
        f, c = h.level(l), h.level(l + 1)
        assert np.array_equal(f["agg"], aggs[l])
        P = _prolongation(f["agg"], c["n"])
        Ac = P.T @ _dense(f) @ P
        assert np.allclose(_dense(c), Ac, rtol=1e-13, atol=1e-13 * np.abs(Ac).max())
    assert np.allclose(h.coarse_inverse(), np.linalg.inv(_dense(h.level(h.n_levels - 1))), rtol=1e-9,
                       atol=1e-12)
    x, st, it, rs, rr = h.pcg(w.rhs(), tol=1e-9)
    assert st == 0 and rr <= 1e-9
    assert np.linalg.norm(x - np.linalg.solve(A, w.rhs())) <= 1e-6 * np.linalg.norm(x)
