"""Seeded synthetic inputs for the mortar coupling path.

This package generates surface meshes (nodal coordinates and quad4
connectivity) and keyed upstream weights.  It holds none of the mortar
method's arithmetic: no projection, clipping, quadrature or assembly.  Both
the HIP path's tests/bench and the CPU oracle draw their inputs from here.
"""

from .meshes import (  # noqa: F401
    Mesh,
    Interface,
    tensor_grid,
    flat_tied,
    cylinder,
    wavy,
    kite_fan,
    graded_flat,
    interface_config,
    opposing,
    renumbered,
    batched_instances,
    CONFIG_NAMES,
)
from .degenerate import collapsed_slave, perpendicular_master  # noqa: F401
from .weights import keyed_normal, upstream_weights  # noqa: F401
