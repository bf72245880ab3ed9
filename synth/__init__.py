"""Seeded synthetic inputs (meshes, rank decompositions, LDU coefficients).

Shared by the oracle and the GPU path as input only; holds none of the
repartitioning, update or solver arithmetic.
"""
from .mesh import (Mesh, Partition, LduValues, structured_mesh, stretched_dz, box27_mesh,
                   decompose_blocks, decompose_rcb, partition, cell_diagonal, ldu_values, stream_fluxes,
                   momentum_ldu)
from .workloads import RECIPES, Recipe, Workload, build, small

__all__ = [
    "Mesh", "Partition", "LduValues", "structured_mesh", "stretched_dz", "box27_mesh",
    "decompose_blocks", "decompose_rcb", "partition", "cell_diagonal", "ldu_values", "stream_fluxes", "momentum_ldu",
    "RECIPES", "Recipe", "Workload", "build", "small",
]
