"""Seeded synthetic inputs for the extruded-prism DG tracer operator.

This package only builds meshes, layer levels, velocity samples, initial
fields and parameters.  It holds none of the discretisation's arithmetic:
both the oracle (``oracle/``) and the HIP library receive the arrays it
produces and compute everything else themselves.
"""

from .prism_mesh import (  # noqa: F401
    Workload,
    square_mesh,
    hilbert_order,
    triangle_neighbours,
    sigma_levels,
    zlevel_levels,
    solid_body_velocity,
    cfl_dt,
    rotating_blob,
    four_field_ocean,
    zlevel_ensemble,
    adjoint_blob,
    small_ensemble,
    tiny,
    ragged,
    natural_prism_count,
)
