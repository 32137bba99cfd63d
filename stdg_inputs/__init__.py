"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This package holds no arithmetic of the discretisation: it only produces
meshes (vertex coordinates and tetrahedron connectivity), the coordinates at
which nodal values live (the layout of the coefficient vectors), and the
closed-form or seeded velocity/pressure fields that are sampled there.

Layout conventions (they define the meaning of every coefficient vector):

* A tetrahedron's local vertex order is the order of its row in ``tets``; the
  affine map sends local vertex 0 to the reference origin and local vertices
  1, 2, 3 to the unit points on the xi, eta and zeta axes (Sec. 2.3).
* Spatial nodes are the equispaced points (j1, j2, j3)/p with j1+j2+j3 <= p,
  enumerated with j1 fastest, then j2, then j3 (Sec. 2.3, eq. bf_1).
* Time nodes are the Gauss-Legendre points of [0, 1] (Sec. 2.3); the time
  coefficient with index a is the value at the a-th point in ascending order.
* Pressure vectors are laid out [tet][time node][spatial node].
* A curved element is given by the physical positions of its spatial nodes,
  in the same order ([tet][node][3]).
"""

from .mesh import kuhn_mesh, hex_count_for
from .fields import (beltrami_velocity, beltrami_pressure, fourier_modes,
                     fourier_velocity)
from .nodes import (node_reference_points, node_coordinates, time_nodes,
                    n_spatial)
from .curved import curved_mesh, deform

__all__ = ["kuhn_mesh", "hex_count_for", "beltrami_velocity",
           "beltrami_pressure", "fourier_modes", "fourier_velocity",
           "node_reference_points", "node_coordinates", "time_nodes",
           "n_spatial", "curved_mesh", "deform"]
