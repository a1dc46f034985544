"""Seeded synthetic inputs for the GN/LM PCG path.

This package only draws inputs: lattices, constraint sets, masks, smooth random
fields, noise textures, icosphere meshes, voxel blocks, and the rendered shading image of a
smooth surface (``render``: the exact normal of the continuous surface under the
scene's lighting).  It holds none of the solver's arithmetic (no residual,
Jacobian, difference normal or step), so the oracle and the HIP path can both be
fed from it without sharing any of the method.

Every generator takes an explicit ``seed`` and uses
``numpy.random.default_rng(seed)``; the same call always returns bit-identical
arrays.
"""
from .grids import (arap_warp, poisson_edit, shape_from_shading, optical_flow,
                    laplacian_grid, lp_smooth, intrinsic_image, SFS_LIGHTING)
from .mesh import icosphere, morton_order, arap_mesh, laplacian_mesh, grid_edges
from .volume import arap_volume, lattice_edges

__all__ = ["arap_warp", "poisson_edit", "shape_from_shading", "optical_flow",
           "laplacian_grid", "lp_smooth", "intrinsic_image", "SFS_LIGHTING", "icosphere", "morton_order",
           "arap_mesh", "laplacian_mesh", "grid_edges", "arap_volume", "lattice_edges"]
