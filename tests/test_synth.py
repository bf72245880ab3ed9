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


# --------------------------------------------------------------------------
# non-symmetric momentum-type values
# --------------------------------------------------------------------------
MOMENTUM_CASES = [((7, 6, 5), ("blocks", 2, 3, 1), dict(kappa=(1e-2, 1.0))),
                  ((6, 5, 7), ("rcb", 5), dict(kappa=(1e-3, 1.0), scramble=True, stretch=100.0))]


def _global_momentum(w, pe, sigma):
    """The operator assembled straight from the undecomposed face arrays:
    A(a,b) = -(c + max(-F,0)), A(b,a) = -(c + max(F,0)); diag as the sum of
    c + max(F_out, 0) over faces (walls c) plus sigma (natural numbering)."""
    mesh = w.mesh
    c = w.coefficients()
    cm = float(np.median(c))
    F = synth.stream_fluxes(mesh)
    F = F * (pe * cm / np.abs(F).max())
    n, ni = mesh.n_cells, mesh.n_interior
    A = np.zeros((n, n))
    d = np.zeros(n)
    for f in range(mesh.n_faces):
        a, b = mesh.face_a[f], mesh.face_b[f]
        if f < ni:
            A[a, b] = -(c[f] + max(-F[f], 0.0))
            A[b, a] = -(c[f] + max(F[f], 0.0))
            d[a] += c[f] + max(F[f], 0.0)
            d[b] += c[f] + max(-F[f], 0.0)
        else:
            d[a] += c[f]
    A[np.arange(n), np.arange(n)] = d + sigma * cm
    return A, F


@pytest.mark.parametrize("case", range(len(MOMENTUM_CASES)))
def test_momentum_values_match_global_assembly(case):
    """Per-rank upper / lower / interface values place every entry of the
    global operator at its (row, column), bit for bit: checks the orientation
    of each rank's faces and interfaces against the mesh."""
    shape, decomp, kw = MOMENTUM_CASES[case]
    w = synth.small(shape, decomp, seed=40 + case, **kw)
    pe, sigma = 5.0, 0.5
    A, F = _global_momentum(w, pe, sigma)
    v = w.momentum_values(pe=pe, sigma=sigma)
    p = w.part
    nat = p.rank_cells
    got = np.zeros_like(A)
    for r in range(w.n_ranks):
        d = p.rank(r)
        vr = v.rank(p, r)
        base = p.cell_ptr[r]
        cells = nat[base:base + d["n_cells"]]
        got[cells, cells] = vr["diag"]
        got[cells[d["owner"]], cells[d["neighbour"]]] = vr["upper"]
        got[cells[d["neighbour"]], cells[d["owner"]]] = vr["lower"]
        nb = nat[p.cell_ptr[d["iface_nbr_rank"]] + d["iface_nbr_cell"]]
        got[cells[d["iface_cell"]], nb] = vr["iface"]
    assert np.array_equal(got.view(np.uint64), A.view(np.uint64))
    assert np.abs(A - A.T).max() > 0.1 * np.abs(F).max()


@pytest.mark.parametrize("case", range(len(MOMENTUM_CASES)))
def test_momentum_m_matrix_and_divergence_free(case):
    shape, decomp, kw = MOMENTUM_CASES[case]
    w = synth.small(shape, decomp, seed=50 + case, **kw)
    mesh = w.mesh
    F = synth.stream_fluxes(mesh)
    ni = mesh.n_interior
    div = np.zeros(mesh.n_cells)
    np.add.at(div, mesh.face_a[:ni], F[:ni])
    np.add.at(div, mesh.face_b[:ni], -F[:ni])
    assert np.abs(div).max() <= 1e-14 * np.abs(F).max() and np.abs(F).max() > 0
    assert (F[ni:] == 0).all()
    v = w.momentum_values(pe=8.0, sigma=1.0)
    assert (v.upper < 0).all() and (v.lower < 0).all() and (v.iface < 0).all() and (v.diag > 0).all()
    A, _ = _global_momentum(w, 8.0, 1.0)
    sigma = np.median(w.coefficients())
    # row sums: sigma + wall coefficients + net outflow (0): every row dominant
    assert (A.sum(axis=1) >= sigma * (1 - 1e-9)).all()


def test_momentum_without_flux_is_pressure_plus_sigma():
    w = synth.small((6, 5, 4), ("blocks", 2, 1, 2), seed=60, kappa=(1e-2, 1.0))
    v0, vp = w.momentum_values(pe=0.0, sigma=0.0), w.values()
    assert np.array_equal(v0.upper, vp.upper) and np.array_equal(v0.lower, vp.upper)
    assert np.array_equal(v0.iface, vp.iface) and np.array_equal(v0.diag, vp.diag)
