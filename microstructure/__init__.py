"""Seeded synthetic microstructures for the periodic cell problem.

This package only describes *inputs*: nodal level-set values (signed distance to
the nearest interface), nodal phase labels and isotropic Lame pairs per phase.
It contains none of the discretisation or solver arithmetic, so both the CPU
oracle and the GPU path can consume the same arrays without sharing any of the
method's code.

Conventions
-----------
* Grid ``n = (n0, n1, n2)`` nodes per axis, periodic, node ``(i, j, k)`` sits at
  ``x = (i, j, k) * h``.  Flat index ``i + n0 * (j + n1 * k)`` (x fastest); the
  numpy arrays returned here are flat vectors in that order.
* Generators work in voxel units (``h = 1``, cell length ``n`` voxels) unless a
  ``length`` is passed explicitly.
* Level set: positive in the matrix (phase 0 for inclusions), negative inside
  inclusions; phases beyond two are carried by the label array, not by the sign.
"""

from .grid import node_coords, periodic_delta, flat_shape
from .materials import lame_from_E_nu, isotropic_bulk_shear
from .shapes import (
    spheres_levelset,
    rsa_spheres,
    laminate_levelset,
    coated_sphere_levelset,
    ellipsoids_levelset,
    rsa_ellipsoids,
)
from .configs import (
    config_single_sphere,
    config_spheres64,
    config_spheres128,
    config_uneven_batch,
    config_ellipsoids,
    mandel_unit_loads,
)

__all__ = [
    "node_coords", "periodic_delta", "flat_shape",
    "lame_from_E_nu", "isotropic_bulk_shear",
    "spheres_levelset", "rsa_spheres", "laminate_levelset",
    "coated_sphere_levelset", "ellipsoids_levelset", "rsa_ellipsoids",
    "config_single_sphere", "config_spheres64", "config_spheres128",
    "config_uneven_batch", "config_ellipsoids", "mandel_unit_loads",
]
