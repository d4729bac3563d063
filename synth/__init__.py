"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package produces *inputs only*: meridian-plane meshes with tagged
boundary segments, particle initial conditions and analytic initial fields
projected onto mesh cells by plain quadrature.  It contains none of the
method's own arithmetic (no incidence signs, Hodge matrices, SPAI, push,
walk or deposit), so the oracle and the GPU library can both consume it
without sharing any of the scheme they are compared on.

Coordinates are (z, rho) in metres throughout: the meridian plane is the
Cartesian (x, y) := (z, rho) plane, so counter-clockwise triangles in that
plane carry the azimuthal unit vector as their normal.
"""

from .meshes import (  # noqa: F401
    Mesh, BC_PEC, BC_AXIS, BC_EMITTER, BC_OPEN, BC_NAMES,
    canonical_edges, rect_mesh, rippled_mesh, grid_mesh, tiny_mesh,
)
from .fields import tm010_fields, uniform_field_dofs, edge_line_integrals, face_flux_integrals  # noqa: F401
from .particles import (  # noqa: F401
    ELECTRON_CHARGE, ELECTRON_MASS, C_LIGHT, EPS0, MU0,
    disk_beam, annular_beam, gamma_beta_from_kev, random_momenta,
)
