"""Structured finite-volume meshes, their rank decompositions and LDU coefficients.

This module produces *inputs* for the repartitioning path: a 7-point
finite-volume mesh, a split of its cells over CPU ranks, and for every rank the
matrix in LDU form (diag over cells, upper/lower over owner<neighbour internal
faces) plus the processor-interface couplings to cells on other ranks.  It does
no merging, value scattering or solving; both the oracle and the GPU path
consume what it emits.

Global face enumeration (fixed, used for coefficient draws and for the order in
which a cell's diagonal is accumulated):
  1. interior x faces, 2. interior y faces, 3. interior z faces, each listed in
     the natural order of the cell on the minus side;
  4. wall faces, grouped x-, x+, y-, y+, z-, z+, each in natural cell order.
Natural cell id of (i, j, k) is i + nx*(j + ny*k).

Face coefficient: c_f = kappa_f * area_f / dist_f with dx = dy = 1 and a
per-layer dz.  A wall face acts as a ghost value 0 one cell width away.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


# ----------------------------------------------------------------------------
# mesh
# ----------------------------------------------------------------------------
@dataclass
class Mesh:
    nx: int
    ny: int
    nz: int
    dz: np.ndarray                  # float64[nz] cell widths along z
    walls: tuple                    # (x, y, z) booleans: emit wall faces on that axis
    face_a: np.ndarray = field(repr=False)     # int64[nf] natural id, minus side
    face_b: np.ndarray = field(repr=False)     # int64[nf] natural id, plus side, -1 = wall
    geom: np.ndarray = field(repr=False)       # float64[nf] area/dist
    n_interior: int = 0

    @property
    def n_cells(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def n_faces(self) -> int:
        return int(self.face_a.shape[0])

    def centres(self) -> np.ndarray:
        """float64[N, 3] cell centres in natural order."""
        n = self.n_cells
        nat = np.arange(n, dtype=np.int64)
        i = nat % self.nx
        j = (nat // self.nx) % self.ny
        k = nat // (self.nx * self.ny)
        zc = np.cumsum(self.dz) - 0.5 * self.dz
        return np.stack([i + 0.5, j + 0.5, zc[k]], axis=1)


def stretched_dz(nz: int, ratio: float) -> np.ndarray:
    """dz_k = ratio**(-k/(nz-1)), k = 0..nz-1: widths fall from 1 to 1/ratio."""
    if nz == 1:
        return np.ones(1)
    k = np.arange(nz, dtype=np.float64)
    return ratio ** (-k / (nz - 1))


def structured_mesh(nx: int, ny: int, nz: int, dz=None, walls=(True, True, True)) -> Mesh:
    dz = np.ones(nz) if dz is None else np.asarray(dz, dtype=np.float64)
    assert dz.shape == (nz,)
    idx = np.arange(nx * ny * nz, dtype=np.int64).reshape(nz, ny, nx)
    kk = np.broadcast_to(np.arange(nz)[:, None, None], (nz, ny, nx))

    a_parts, b_parts, g_parts = [], [], []
    # interior x and y faces: area dz_k, centre distance 1
    a_parts.append(idx[:, :, :-1].ravel()); b_parts.append(idx[:, :, 1:].ravel())
    g_parts.append(dz[kk[:, :, :-1].ravel()])
    a_parts.append(idx[:, :-1, :].ravel()); b_parts.append(idx[:, 1:, :].ravel())
    g_parts.append(dz[kk[:, :-1, :].ravel()])
    # interior z faces: area 1, centre distance (dz_k + dz_{k+1}) / 2
    a_parts.append(idx[:-1, :, :].ravel()); b_parts.append(idx[1:, :, :].ravel())
    zg = 2.0 / (dz[:-1] + dz[1:])
    g_parts.append(np.repeat(zg, nx * ny))
    n_interior = int(sum(p.shape[0] for p in a_parts))

    # walls: ghost at one cell width normal to the wall
    wx, wy, wz = walls
    if wx:
        for sl in (idx[:, :, 0], idx[:, :, -1]):
            c = sl.ravel(); a_parts.append(c); g_parts.append(dz[c // (nx * ny)])
    if wy:
        for sl in (idx[:, 0, :], idx[:, -1, :]):
            c = sl.ravel(); a_parts.append(c); g_parts.append(dz[c // (nx * ny)])
    if wz:
        for kz, sl in ((0, idx[0]), (nz - 1, idx[-1])):
            c = sl.ravel(); a_parts.append(c); g_parts.append(np.full(c.shape[0], 1.0 / dz[kz]))
    n_wall = int(sum(p.shape[0] for p in a_parts)) - n_interior
    b_parts.append(np.full(n_wall, -1, dtype=np.int64))

    return Mesh(nx, ny, nz, dz, tuple(walls),
                np.ascontiguousarray(np.concatenate(a_parts)),
                np.ascontiguousarray(np.concatenate(b_parts)),
                np.ascontiguousarray(np.concatenate(g_parts)),
                n_interior)


def box27_mesh(nx: int, ny: int, nz: int) -> Mesh:
    """Unit cells coupled to all 26 neighbours (faces, edges and corners of
    the cell), so every interior row holds 27 entries: rows with far more
    couplings than a 7-point stencil, as polyhedral finite-volume cells have.
    Interior "faces" are the neighbour pairs, listed per offset (13 offsets
    with a positive first non-zero component in z, y, x order) in the natural
    order of the minus-side cell; geometric weight 1 / |offset|^2.  Walls as
    structured_mesh on all six sides."""
    idx = np.arange(nx * ny * nz, dtype=np.int64).reshape(nz, ny, nx)
    offs = [(dz_, dy_, dx_) for dz_ in (-1, 0, 1) for dy_ in (-1, 0, 1) for dx_ in (-1, 0, 1)
            if (dz_, dy_, dx_) > (0, 0, 0)]
    a_parts, b_parts, g_parts = [], [], []
    for dz_, dy_, dx_ in offs:
        zs = slice(max(0, -dz_), nz - max(0, dz_))
        ys = slice(max(0, -dy_), ny - max(0, dy_))
        xs = slice(max(0, -dx_), nx - max(0, dx_))
        a = idx[zs, ys, xs].ravel()
        a_parts.append(a)
        b_parts.append(a + dx_ + nx * (dy_ + ny * dz_))
        g_parts.append(np.full(a.shape[0], 1.0 / (dx_ * dx_ + dy_ * dy_ + dz_ * dz_)))
    n_interior = int(sum(p.shape[0] for p in a_parts))
    for sl in (idx[:, :, 0], idx[:, :, -1], idx[:, 0, :], idx[:, -1, :], idx[0], idx[-1]):
        c = sl.ravel()
        a_parts.append(c)
        g_parts.append(np.ones(c.shape[0]))
    n_wall = int(sum(p.shape[0] for p in a_parts)) - n_interior
    b_parts.append(np.full(n_wall, -1, dtype=np.int64))
    return Mesh(nx, ny, nz, np.ones(nz), (True, True, True),
                np.ascontiguousarray(np.concatenate(a_parts)),
                np.ascontiguousarray(np.concatenate(b_parts)),
                np.ascontiguousarray(np.concatenate(g_parts)),
                n_interior)


# ----------------------------------------------------------------------------
# decompositions: natural cell id -> rank
# ----------------------------------------------------------------------------
def decompose_blocks(mesh: Mesh, px: int, py: int, pz: int) -> np.ndarray:
    """Balanced blocks (equal when the counts divide); rank = bx + px*(by + py*bz)."""
    assert px <= mesh.nx and py <= mesh.ny and pz <= mesh.nz
    nat = np.arange(mesh.n_cells, dtype=np.int64)
    i = nat % mesh.nx
    j = (nat // mesh.nx) % mesh.ny
    k = nat // (mesh.nx * mesh.ny)
    bx = (i * px) // mesh.nx
    by = (j * py) // mesh.ny
    bz = (k * pz) // mesh.nz
    return (bx + px * (by + py * bz)).astype(np.int32)


def decompose_rcb(mesh: Mesh, n_parts: int, rng: np.random.Generator,
                  jitter: float = 0.25) -> np.ndarray:
    """Recursive coordinate bisection with random cut planes.

    A set holding p parts is split into floor(p/2) and ceil(p/2) parts along an
    axis drawn uniformly from {x, y, z}; the cut sits at the cell-centre quantile
    (floor(p/2)/p)*(1+U[-jitter, jitter]) of that axis (ties broken by natural
    id), clipped so that every part keeps at least one cell.  Ranks are numbered
    depth first, lower side first.  Draws are taken in that depth-first order.
    """
    cen = mesh.centres()
    rank = np.empty(mesh.n_cells, dtype=np.int32)

    def split(cells: np.ndarray, p: int, first: int):
        if p == 1:
            rank[cells] = first
            return
        axis = int(rng.integers(3))
        u = float(rng.uniform(-jitter, jitter))
        pl = p // 2
        q = (pl / p) * (1.0 + u)
        order = np.lexsort((cells, cen[cells, axis]))
        m = int(round(q * cells.shape[0]))
        m = min(max(m, pl), cells.shape[0] - (p - pl))
        s = cells[order]
        split(np.sort(s[:m]), pl, first)
        split(np.sort(s[m:]), p - pl, first + pl)

    assert mesh.n_cells >= n_parts
    split(np.arange(mesh.n_cells, dtype=np.int64), n_parts, 0)
    return rank


# ----------------------------------------------------------------------------
# partitioned LDU structure
# ----------------------------------------------------------------------------
@dataclass
class Partition:
    """Per-rank LDU addressing, concatenated over ranks (slices via *_ptr).

    rank_cells  natural ids of each rank's cells in local order (sorted by
                global id, the global id being natural or scrambled)
    owner/neighbour  internal faces, owner < neighbour (local ids), sorted by
                (owner, neighbour)
    if_*        processor-interface couplings: this rank's cell, the rank and
                local id of the cell across the face; sorted by (nbr rank,
                global face id) so both sides list a shared patch in one order
    wall_*      wall faces (local cell), kept for gradients w.r.t. wall
                coefficients
    """
    n_ranks: int
    gid: np.ndarray          # int64[N] natural id -> global (possibly scrambled) id
    cell_rank: np.ndarray    # int32[N]
    cell_local: np.ndarray   # int32[N]
    n_cells: np.ndarray      # int64[n_ranks]
    cell_ptr: np.ndarray     # int64[n_ranks+1]
    rank_cells: np.ndarray   # int64[N]
    face_ptr: np.ndarray
    owner: np.ndarray        # int32
    neighbour: np.ndarray    # int32
    face_gid: np.ndarray     # int64
    if_ptr: np.ndarray
    if_cell: np.ndarray      # int32
    if_nbr_rank: np.ndarray  # int32
    if_nbr_cell: np.ndarray  # int32
    if_gid: np.ndarray       # int64
    wall_ptr: np.ndarray
    wall_cell: np.ndarray    # int32
    wall_gid: np.ndarray     # int64

    def rank(self, r: int) -> dict:
        """Contiguous per-rank addressing arrays (int32)."""
        f0, f1 = self.face_ptr[r], self.face_ptr[r + 1]
        i0, i1 = self.if_ptr[r], self.if_ptr[r + 1]
        return dict(
            n_cells=int(self.n_cells[r]),
            owner=self.owner[f0:f1], neighbour=self.neighbour[f0:f1],
            iface_cell=self.if_cell[i0:i1], iface_nbr_rank=self.if_nbr_rank[i0:i1],
            iface_nbr_cell=self.if_nbr_cell[i0:i1])


def partition(mesh: Mesh, cell_rank: np.ndarray, gid: np.ndarray | None = None) -> Partition:
    n = mesh.n_cells
    n_ranks = int(cell_rank.max()) + 1
    gid = np.arange(n, dtype=np.int64) if gid is None else np.asarray(gid, dtype=np.int64)
    cell_rank = cell_rank.astype(np.int32)
    counts = np.bincount(cell_rank, minlength=n_ranks).astype(np.int64)
    assert (counts > 0).all(), "every rank must own at least one cell"
    cell_ptr = np.zeros(n_ranks + 1, dtype=np.int64)
    np.cumsum(counts, out=cell_ptr[1:])
    # local order: by (rank, global id)
    rank_cells = np.lexsort((gid, cell_rank)).astype(np.int64)
    cell_local = np.empty(n, dtype=np.int32)
    cell_local[rank_cells] = (np.arange(n, dtype=np.int64) - cell_ptr[cell_rank[rank_cells]]).astype(np.int32)

    a, b = mesh.face_a, mesh.face_b
    ni = mesh.n_interior
    fa, fb = a[:ni], b[:ni]
    ra, rb = cell_rank[fa], cell_rank[fb]
    la, lb = cell_local[fa], cell_local[fb]

    # internal faces
    inner = np.nonzero(ra == rb)[0]
    own = np.minimum(la[inner], lb[inner]).astype(np.int64)
    nbr = np.maximum(la[inner], lb[inner]).astype(np.int64)
    rr = ra[inner].astype(np.int64)
    m = int(counts.max())
    key = (rr * m + own) * m + nbr
    o = np.argsort(key, kind="stable")
    face_gid = inner[o].astype(np.int64)
    owner = own[o].astype(np.int32)
    neighbour = nbr[o].astype(np.int32)
    face_ptr = np.zeros(n_ranks + 1, dtype=np.int64)
    np.cumsum(np.bincount(rr, minlength=n_ranks), out=face_ptr[1:])
    del key, o, own, nbr, rr

    # interfaces: one entry on each side
    cross = np.nonzero(ra != rb)[0]
    e_rank = np.concatenate([ra[cross], rb[cross]]).astype(np.int64)
    e_cell = np.concatenate([la[cross], lb[cross]])
    e_nrank = np.concatenate([rb[cross], ra[cross]]).astype(np.int64)
    e_ncell = np.concatenate([lb[cross], la[cross]])
    e_gid = np.concatenate([cross, cross]).astype(np.int64)
    o = np.lexsort((e_gid, e_nrank, e_rank))
    if_ptr = np.zeros(n_ranks + 1, dtype=np.int64)
    np.cumsum(np.bincount(e_rank, minlength=n_ranks), out=if_ptr[1:])

    # walls
    wall_gid = np.arange(ni, mesh.n_faces, dtype=np.int64)
    wr = cell_rank[a[ni:]].astype(np.int64)
    wo = np.lexsort((wall_gid, wr))
    wall_ptr = np.zeros(n_ranks + 1, dtype=np.int64)
    np.cumsum(np.bincount(wr, minlength=n_ranks), out=wall_ptr[1:])

    return Partition(
        n_ranks=n_ranks, gid=gid, cell_rank=cell_rank, cell_local=cell_local,
        n_cells=counts, cell_ptr=cell_ptr, rank_cells=rank_cells,
        face_ptr=face_ptr, owner=owner, neighbour=neighbour, face_gid=face_gid,
        if_ptr=if_ptr, if_cell=e_cell[o].astype(np.int32),
        if_nbr_rank=e_nrank[o].astype(np.int32), if_nbr_cell=e_ncell[o].astype(np.int32),
        if_gid=e_gid[o],
        wall_ptr=wall_ptr, wall_cell=cell_local[a[ni:]][wo].astype(np.int32),
        wall_gid=wall_gid[wo])


# ----------------------------------------------------------------------------
# coefficients -> LDU values
# ----------------------------------------------------------------------------
def cell_diagonal(mesh: Mesh, c: np.ndarray) -> np.ndarray:
    """diag of each cell (natural order): sum of its face coefficients, added in
    ascending global face order starting from 0.0."""
    ni = mesh.n_interior
    nf = mesh.n_faces
    cells = np.empty(2 * ni + (nf - ni), dtype=np.int64)
    w = np.empty(cells.shape[0], dtype=np.float64)
    cells[0:2 * ni:2] = mesh.face_a[:ni]
    cells[1:2 * ni:2] = mesh.face_b[:ni]
    w[0:2 * ni:2] = c[:ni]
    w[1:2 * ni:2] = c[:ni]
    cells[2 * ni:] = mesh.face_a[ni:]
    w[2 * ni:] = c[ni:]
    # bincount accumulates sequentially in input order
    return np.bincount(cells, weights=w, minlength=mesh.n_cells)


@dataclass
class LduValues:
    """Per-rank LDU values concatenated over ranks, slices as in Partition.
    lower is None for a symmetric matrix (lower == upper, not stored)."""
    diag: np.ndarray    # float64[N]       by rank, local cell order
    upper: np.ndarray   # float64[faces]   A(owner, neighbour)
    iface: np.ndarray   # float64[ifaces]  A(cell, cell across the interface)
    lower: np.ndarray | None = None   # float64[faces]  A(neighbour, owner)

    def rank(self, part: Partition, r: int) -> dict:
        c0, c1 = part.cell_ptr[r], part.cell_ptr[r + 1]
        f0, f1 = part.face_ptr[r], part.face_ptr[r + 1]
        i0, i1 = part.if_ptr[r], part.if_ptr[r + 1]
        out = dict(diag=self.diag[c0:c1], upper=self.upper[f0:f1], iface=self.iface[i0:i1])
        if self.lower is not None:
            out["lower"] = self.lower[f0:f1]
        return out


def ldu_values(mesh: Mesh, part: Partition, c: np.ndarray) -> LduValues:
    diag_nat = cell_diagonal(mesh, c)
    return LduValues(diag=diag_nat[part.rank_cells],
                     upper=-c[part.face_gid],
                     iface=-c[part.if_gid])


# ----------------------------------------------------------------------------
# non-symmetric convection-diffusion (momentum-type) values
# ----------------------------------------------------------------------------
def stream_fluxes(mesh: Mesh) -> np.ndarray:
    """Face fluxes along +axis (from face_a to face_b) of a rotating flow in
    every x-y plane, from the stream function psi(X, Y) = sin(pi X) sin(pi Y)
    at the cell corners X = i / nx, Y = j / ny: an x face carries
    (psi(top corner) - psi(bottom corner)) dz_k, a y face
    -(psi(right) - psi(left)) dz_k, z faces and walls none.  The four fluxes
    of a cell cancel, so the flow is divergence-free cell by cell."""
    nx, ny, nz = mesh.nx, mesh.ny, mesh.nz
    X = np.arange(nx + 1) / nx
    Y = np.arange(ny + 1) / ny
    psi = np.sin(np.pi * X)[None, :] * np.sin(np.pi * Y)[:, None]      # [ny+1, nx+1]
    dz = mesh.dz
    # x faces between i and i+1 (i < nx-1), in (k, j, i) order
    fx = (psi[1:, 1:nx] - psi[:-1, 1:nx])[None, :, :] * dz[:, None, None]            # [nz, ny, nx-1]
    # y faces between j and j+1 (j < ny-1)
    fy = -(psi[1:ny, 1:] - psi[1:ny, :-1])[None, :, :] * dz[:, None, None]           # [nz, ny-1, nx]
    fz = np.zeros((nz - 1) * ny * nx)
    flux = np.zeros(mesh.n_faces)
    interior = np.concatenate([fx.ravel(), fy.ravel(), fz])
    assert interior.shape[0] == mesh.n_interior
    flux[:mesh.n_interior] = interior
    return flux


def momentum_ldu(mesh: Mesh, part: Partition, c: np.ndarray, flux: np.ndarray, sigma: np.ndarray) -> LduValues:
    """Upwind convection-diffusion matrix with a transient term: for an
    interior face a -> b with diffusion coefficient c_f and flux F_f,
    A(a, b) = -(c_f + max(-F_f, 0)) and A(b, a) = -(c_f + max(F_f, 0)); the
    diagonal of a cell sums c_f + max(F_out, 0) over its faces (walls: c_w)
    in ascending global face order, then adds sigma of the cell.  With a
    divergence-free flux the matrix is a diagonally dominant M-matrix,
    non-symmetric wherever F_f != 0."""
    ni, nf = mesh.n_interior, mesh.n_faces
    a, b = mesh.face_a, mesh.face_b
    F = flux[:ni]
    a_ab = -(c[:ni] + np.maximum(-F, 0.0))      # A(a, b)
    a_ba = -(c[:ni] + np.maximum(F, 0.0))       # A(b, a)
    cells = np.empty(2 * ni + (nf - ni), dtype=np.int64)
    w = np.empty(cells.shape[0], dtype=np.float64)
    cells[0:2 * ni:2] = a[:ni]
    cells[1:2 * ni:2] = b[:ni]
    w[0:2 * ni:2] = c[:ni] + np.maximum(F, 0.0)
    w[1:2 * ni:2] = c[:ni] + np.maximum(-F, 0.0)
    cells[2 * ni:] = a[ni:]
    w[2 * ni:] = c[ni:]
    diag_nat = np.bincount(cells, weights=w, minlength=mesh.n_cells) + sigma

    # internal faces: is the rank-local owner the mesh's minus side?
    f_rank = np.repeat(np.arange(part.n_ranks), np.diff(part.face_ptr))
    own_nat = part.rank_cells[part.cell_ptr[f_rank] + part.owner]
    fwd = own_nat == a[part.face_gid]
    upper = np.where(fwd, a_ab[part.face_gid], a_ba[part.face_gid])
    lower = np.where(fwd, a_ba[part.face_gid], a_ab[part.face_gid])
    # interfaces: the entry of the passing rank's own row
    i_rank = np.repeat(np.arange(part.n_ranks), np.diff(part.if_ptr))
    cell_nat = part.rank_cells[part.cell_ptr[i_rank] + part.if_cell]
    iface = np.where(cell_nat == a[part.if_gid], a_ab[part.if_gid], a_ba[part.if_gid])
    return LduValues(diag=diag_nat[part.rank_cells], upper=upper, iface=iface, lower=lower)
