"""Seeded workload recipes shaped like the paper's pressure systems.

The paper's benchmark is the pressure equation of a lid-driven-cavity case on
uniform cubic grids decomposed over many CPU ranks (Section 4).  Those
matrices are not available, so these recipes build 7-point finite-volume
Poisson-type systems of the same shape: one GPU's share of the ranks, with
processor-interface faces between them.

Random streams: numpy.random.SeedSequence(seed).spawn(5 + T) taken in the
fixed order [coefficients, rhs, target, permutation, rcb, timestep 0..T-1].
kappa is log-uniform: exp(U[ln lo, ln hi]) per global face (walls included).
Timestep t uses kappa_t = kappa_0 * (1 + 0.05 * U[-1, 1]) per face
(non-compounding); b stays fixed across timesteps.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .mesh import (Mesh, Partition, LduValues, structured_mesh, stretched_dz, box27_mesh,
                   decompose_blocks, decompose_rcb, partition, ldu_values, stream_fluxes, momentum_ldu)


@dataclass
class Recipe:
    name: str
    shape: tuple
    decomp: tuple               # ("blocks", px, py, pz) | ("rcb", p)
    kappa: tuple | None         # (lo, hi) log-uniform, None = constant 1
    seed: int
    timesteps: int = 1
    stretch: float | None = None   # z aspect ratio (dz from 1 to 1/stretch)
    scramble: bool = False
    walls: tuple = (True, True, True)
    note: str = ""
    stencil: int = 7               # 7: face neighbours; 27: all 26 neighbours (box27_mesh)


RECIPES = {
    # 32^3, 4 z-slabs: constant coefficients (diag 6, off-diagonal -1)
    "c1": Recipe("c1", (32, 32, 32), ("blocks", 1, 1, 4), None, 1,
                 note="32^3 unit spacing, 4 z-slab ranks, diag 6 / off -1, FP64 PCG"),
    # 128^3, 32 ranks as 4x4x2 blocks of 32x32x64, 20 perturbed timesteps
    "c2": Recipe("c2", (128, 128, 128), ("blocks", 4, 4, 2), (1e-2, 1.0), 2, timesteps=20,
                 note="128^3, 32 ranks, log-uniform [1e-2,1], 20 timesteps of update + FP64 PCG"),
    # 256^3, 64 ranks as 4x4x4 blocks of 64^3
    "c3": Recipe("c3", (256, 256, 256), ("blocks", 4, 4, 4), (1e-3, 1.0), 3, timesteps=8,
                 note="256^3, 64 ranks, log-uniform [1e-3,1], FP64 vs mixed PCG"),
    # adjoint: 96^3, 16 ranks as 2x2x4 blocks of 48x48x24
    "c4": Recipe("c4", (96, 96, 96), ("blocks", 2, 2, 4), (1e-2, 1.0), 4,
                 note="96^3, 16 ranks, adjoint backward"),
    "c4fd": Recipe("c4fd", (16, 16, 16), ("blocks", 2, 2, 2), (1e-2, 1.0), 4,
                   note="16^3, 8 ranks, finite-difference check of the adjoint"),
    # scrambled, stretched, RCB
    "c5": Recipe("c5", (160, 160, 160), ("rcb", 48), (1e-3, 1.0), 5, timesteps=10,
                 stretch=100.0, scramble=True,
                 note="160^3 stretched z (aspect 100), scrambled ids, 48 RCB ranks"),
}


@dataclass
class Workload:
    recipe: Recipe
    mesh: Mesh
    part: Partition
    kappa0: np.ndarray
    b_nat: np.ndarray        # float64[N] natural order
    xt_nat: np.ndarray       # float64[N] natural order (adjoint target)
    step_seqs: list

    @property
    def n_ranks(self) -> int:
        return self.part.n_ranks

    @property
    def n_cells(self) -> int:
        return self.mesh.n_cells

    def kappa(self, t: int | None = None) -> np.ndarray:
        if t is None:
            return self.kappa0
        rng = np.random.default_rng(self.step_seqs[t])
        return self.kappa0 * (1.0 + 0.05 * rng.uniform(-1.0, 1.0, self.kappa0.shape[0]))

    def coefficients(self, t: int | None = None) -> np.ndarray:
        return self.kappa(t) * self.mesh.geom

    def values(self, t: int | None = None) -> LduValues:
        return ldu_values(self.mesh, self.part, self.coefficients(t))

    def momentum_values(self, t: int | None = None, pe: float = 4.0, sigma: float = 1.0) -> LduValues:
        """Non-symmetric momentum-type matrix on the same mesh and ranks:
        diffusion c_f = coefficients(t), the rotating flux of stream_fluxes
        scaled so its largest face flux is pe * median(c), and a transient
        term sigma * median(c) on every diagonal."""
        c = self.coefficients(t)
        cm = float(np.median(c))
        flux = stream_fluxes(self.mesh)
        fmax = float(np.abs(flux).max())
        if fmax > 0.0:
            flux = flux * (pe * cm / fmax)
        return momentum_ldu(self.mesh, self.part, c, flux, np.full(self.mesh.n_cells, sigma * cm))

    def merged(self, v_nat: np.ndarray, first: int = 0, alpha: int | None = None) -> np.ndarray:
        """A natural-order cell field in merged order: the share's ranks in
        order, each in its local cell order."""
        alpha = self.n_ranks - first if alpha is None else alpha
        c0, c1 = self.part.cell_ptr[first], self.part.cell_ptr[first + alpha]
        return np.ascontiguousarray(v_nat[self.part.rank_cells[c0:c1]])

    def rhs(self) -> np.ndarray:
        return self.merged(self.b_nat)

    def target(self) -> np.ndarray:
        return self.merged(self.xt_nat)


def build(recipe: Recipe | str, **overrides) -> Workload:
    if isinstance(recipe, str):
        recipe = RECIPES[recipe]
    if overrides:
        recipe = Recipe(**{**recipe.__dict__, **overrides})
    nx, ny, nz = recipe.shape
    seqs = np.random.SeedSequence(recipe.seed).spawn(5 + max(recipe.timesteps, 1))
    s_coef, s_rhs, s_tgt, s_perm, s_rcb = seqs[:5]
    dz = stretched_dz(nz, recipe.stretch) if recipe.stretch else None
    if recipe.stencil == 27:
        assert dz is None and recipe.walls == (True, True, True)
        mesh = box27_mesh(nx, ny, nz)
    else:
        mesh = structured_mesh(nx, ny, nz, dz=dz, walls=recipe.walls)
    n = mesh.n_cells

    gid = None
    if recipe.scramble:
        gid = np.random.default_rng(s_perm).permutation(n).astype(np.int64)
    kind = recipe.decomp[0]
    if kind == "blocks":
        cell_rank = decompose_blocks(mesh, *recipe.decomp[1:])
    elif kind == "rcb":
        cell_rank = decompose_rcb(mesh, recipe.decomp[1], np.random.default_rng(s_rcb))
    else:
        raise ValueError(kind)
    part = partition(mesh, cell_rank, gid)

    if recipe.kappa is None:
        kappa0 = np.ones(mesh.n_faces)
    else:
        lo, hi = recipe.kappa
        kappa0 = np.exp(np.random.default_rng(s_coef).uniform(np.log(lo), np.log(hi), mesh.n_faces))
    b = np.random.default_rng(s_rhs).uniform(-1.0, 1.0, n)
    xt = np.random.default_rng(s_tgt).uniform(-1.0, 1.0, n)
    return Workload(recipe, mesh, part, kappa0, b, xt, list(seqs[5:]))


def small(shape, decomp, kappa=None, seed=0, **kw) -> Workload:
    """Ad-hoc small workload for tests."""
    return build(Recipe("small", tuple(shape), tuple(decomp), kappa, seed, **kw))
