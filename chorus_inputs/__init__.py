"""Seeded synthetic inputs shared by the oracle and the GPU library.

This package only *generates inputs*: 20-node hexahedral meshes (a
cubed-sphere shell and Cartesian boxes, optionally periodic and curved) and
seeded random numbers (noise, initial network parameters, smooth random
velocity fields).  It holds none of the spectral-difference arithmetic:
no solution/flux points, no interpolation, no metrics, no fluxes and no
physical initial state.  Both sides consume exactly these arrays.

Hex20 node ordering (local reference cube [0,1]^3, axes xi, eta, zeta):
  corners 0..7      : (i, j, k) in {0,1}^3, index i + 2j + 4k
  xi-edges  8..11   : (1/2, j, k), index 8 + j + 2k
  eta-edges 12..15  : (i, 1/2, k), index 12 + i + 2k
  zeta-edges 16..19 : (i, j, 1/2), index 16 + i + 2j
Faces: 0 xi=0, 1 xi=1, 2 eta=0, 3 eta=1, 4 zeta=0, 5 zeta=1.
Boundary tags: -1 interior, 1 inner sphere wall, 2 outer sphere wall,
3 far-field state boundary.
"""
from .meshes import (HEX20_LOCAL, Hex20Mesh, cubed_sphere_shell, box_mesh,
                     two_element_mesh, warped_slab_mesh, walled_slab_mesh,
                     shell_params_from_config,
                     uniform_noise, mlp_init, random_velocity, CONFIGS)

__all__ = ["HEX20_LOCAL", "Hex20Mesh", "cubed_sphere_shell", "box_mesh",
           "two_element_mesh", "warped_slab_mesh",
           "walled_slab_mesh", "shell_params_from_config", "uniform_noise",
           "mlp_init", "random_velocity", "CONFIGS"]
