"""The seeded input generator: sizes, pairing and reproducibility."""
import numpy as np
import pytest

import synth


def _expected_counts(nx, ny, nz):
    n = nx * ny * nz
    interior = (nx - 1) * ny * nz + nx * (ny - 1) * nz + nx * ny * (nz - 1)
    return n, interior, n + 2 * interior


@pytest.mark.parametrize("name", ["c1", "c4fd"])
def test_recipe_sizes(name):
    w = synth.build(name)
    n, interior, nnz = _expected_counts(*w.recipe.shape)
    p = w.part
    assert w.n_cells == n
    assert p.owner.shape[0] + p.if_cell.shape[0] // 2 == interior
    assert n + 2 * p.owner.shape[0] + p.if_cell.shape[0] == nnz


def test_c1_constant_coefficients():
    w = synth.build("c1")
    v = w.values()
    assert (v.diag == 6.0).all() and (v.upper == -1.0).all() and (v.iface == -1.0).all()
    # 4 z-slabs of 32x32x8: 3 planes of 32x32 interface faces, two sides each
    assert w.part.if_cell.shape[0] == 2 * 3 * 32 * 32
    assert w.n_ranks == 4 and (w.part.n_cells == 8192).all()


def test_interface_pairs_are_mutual():
    w = synth.small((7, 5, 4), ("rcb", 6), kappa=(1e-2, 1.0), seed=11, scramble=True)
    p = w.part
    seen = {}
    for r in range(p.n_ranks):
        d = p.rank(r)
        for c, q, e in zip(d["iface_cell"], d["iface_nbr_rank"], d["iface_nbr_cell"]):
            seen[(r, int(c), int(q), int(e))] = True
    for (r, c, q, e) in seen:
        assert (q, e, r, c) in seen
    # per rank interface order: nbr rank ascending, both sides of a patch in the same face order
    for r in range(p.n_ranks):
        i0, i1 = p.if_ptr[r], p.if_ptr[r + 1]
        keys = list(zip(p.if_nbr_rank[i0:i1], p.if_gid[i0:i1]))
        assert keys == sorted(keys)


def test_faces_upper_triangular_sorted():
    w = synth.small((6, 6, 6), ("blocks", 2, 1, 3), seed=3, scramble=True)
    p = w.part
    for r in range(p.n_ranks):
        d = p.rank(r)
        o, b = d["owner"].astype(np.int64), d["neighbour"].astype(np.int64)
        assert (o < b).all()
        key = o * 10**6 + b
        assert (np.diff(key) > 0).all()


def test_local_order_by_global_id():
    w = synth.small((5, 4, 3), ("rcb", 3), seed=5, scramble=True)
    p = w.part
    for r in range(p.n_ranks):
        cells = p.rank_cells[p.cell_ptr[r]:p.cell_ptr[r + 1]]
        assert (np.diff(p.gid[cells]) > 0).all()
        assert (p.cell_rank[cells] == r).all()


def test_rcb_parts_nonempty_and_reproducible():
    a = synth.small((10, 9, 8), ("rcb", 13), seed=7)
    b = synth.small((10, 9, 8), ("rcb", 13), seed=7)
    assert a.n_ranks == 13 and (a.part.n_cells > 0).all()
    assert (a.part.cell_rank == b.part.cell_rank).all()
    assert (a.kappa0 == b.kappa0).all() and (a.b_nat == b.b_nat).all()


def test_timestep_perturbation_bounds():
    w = synth.small((6, 6, 6), ("blocks", 1, 1, 2), kappa=(1e-2, 1.0), seed=9, timesteps=3)
    for t in range(3):
        ratio = w.kappa(t) / w.kappa0
        assert (ratio >= 0.95).all() and (ratio <= 1.05).all()
    assert not np.array_equal(w.kappa(0), w.kappa(1))


def test_stretched_spacing():
    dz = synth.stretched_dz(160, 100.0)
    assert dz[0] == 1.0 and abs(dz[-1] - 0.01) < 1e-15
    assert (np.diff(dz) < 0).all()
