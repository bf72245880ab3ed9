"""The solve-order renumbering on the host (rp_rcm_order: no device work).

The order is an implementation choice, not part of the method, so there is
no oracle value for it; these tests fix what makes it correct and useful:
a permutation, deterministic, each connected component contiguous, a path
recovered exactly, and on scrambled meshes a bandwidth close to scipy's
reverse Cuthill-McKee and far below the scrambled one."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.csgraph as csgraph

import synth


@pytest.fixture(scope="module")
def rp():
    import paper_2510_08536_amd as pkg
    return pkg


def _grid(dims, seed=None):
    """Structurally symmetric 7-point pattern of a box, optionally scrambled."""
    nx, ny, nz = dims
    n = nx * ny * nz
    idx = np.arange(n).reshape(nz, ny, nx)
    rows, cols = [np.arange(n)], [np.arange(n)]
    for ax in range(3):
        a = np.take(idx, np.arange(idx.shape[ax] - 1), axis=ax).ravel()
        b = np.take(idx, np.arange(1, idx.shape[ax]), axis=ax).ravel()
        rows += [a, b]
        cols += [b, a]
    A = sp.csr_matrix((np.ones(sum(r.size for r in rows)), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n))
    if seed is not None:
        P = np.random.default_rng(seed).permutation(n)
        A = A[P][:, P].tocsr()
    A.sort_indices()
    return A


def _bandwidth(A, perm=None):
    if perm is not None:
        A = A[perm][:, perm]
    c = A.tocoo()
    return int(np.abs(c.row - c.col).max()) if c.nnz else 0


@pytest.mark.parametrize("dims,seed", [((12, 10, 8), 1), ((30, 20, 1), 2), ((7, 7, 7), 3), ((64, 1, 1), 4)])
def test_permutation_and_bandwidth(rp, dims, seed):
    A = _grid(dims, seed)
    perm = rp.rcm_order(A.indptr, A.indices)
    assert np.array_equal(np.sort(perm), np.arange(A.shape[0]))
    ref = csgraph.reverse_cuthill_mckee(A, symmetric_mode=True)
    bw, bw_ref, bw_in = _bandwidth(A, perm), _bandwidth(A, ref), _bandwidth(A)
    assert bw <= max(2, 1.5 * bw_ref), (bw, bw_ref)
    assert bw < bw_in / 4, (bw, bw_in)


def test_path_is_recovered(rp):
    """A scrambled path: RCM starts at one end and walks it, bandwidth 1."""
    n = 50
    A = _grid((n, 1, 1), seed=7)
    perm = rp.rcm_order(A.indptr, A.indices)
    assert _bandwidth(A, perm) == 1


def test_deterministic_and_components_contiguous(rp):
    """Two disjoint grids, an isolated row and a self-loop-only row: every
    component occupies one contiguous stretch of the order."""
    A1, A2 = _grid((5, 4, 3), seed=11), _grid((6, 1, 1), seed=12)
    iso = sp.csr_matrix(([1.0], ([0], [0])), shape=(1, 1))
    empty = sp.csr_matrix((1, 1))
    A = sp.block_diag([A1, iso, A2, empty]).tocsr()
    A.sort_indices()
    perm = rp.rcm_order(A.indptr, A.indices)
    assert np.array_equal(perm, rp.rcm_order(A.indptr, A.indices))
    n1, n2 = A1.shape[0], A2.shape[0]
    comp = np.concatenate([np.zeros(n1), [1], np.full(n2, 2), [3]])[perm]
    changes = np.count_nonzero(np.diff(comp))
    assert changes == 3, comp


def test_fused_share_of_a_scrambled_workload(rp):
    """The fused local block of a scrambled RCB workload, as the plan builds
    it (the oracle's merge): the order cuts its bandwidth by an order of
    magnitude."""
    import oracle
    from helpers import share_ranks
    w = synth.small((16, 14, 12), ("rcb", 6), seed=5, scramble=True)
    m = oracle.merge(w.part.n_cells, 0, w.n_ranks, share_ranks(w, 0, w.n_ranks))
    A = sp.csr_matrix((np.ones(m.nnz_local), np.asarray(m.col), np.asarray(m.row_ptr)),
                      shape=(m.n_rows, m.n_rows))
    perm = rp.rcm_order(A.indptr, A.indices)
    assert np.array_equal(np.sort(perm), np.arange(m.n_rows))
    assert _bandwidth(A, perm) * 10 < _bandwidth(A)


def test_empty_and_bad_patterns(rp):
    import paper_2510_08536_amd.rp as low
    assert rp.rcm_order(np.zeros(1, np.int32), np.zeros(0, np.int32)).size == 0
    with pytest.raises(low.RpError):
        rp.rcm_order(np.array([0, 1, 2], np.int32), np.array([0, 2], np.int32))   # column out of range
    with pytest.raises(low.RpError):
        rp.rcm_order(np.array([0, 2, 1], np.int32), np.array([0, 1], np.int32))   # row_ptr decreases
    with pytest.raises(low.RpError):
        rp.rcm_order(np.array([1, 2], np.int32), np.array([0, 0], np.int32))      # row_ptr[0] != 0
