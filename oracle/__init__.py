"""FP64 CPU oracle for the extruded-prism DG tracer step.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import this
package: it is used by ``tests/``, by ``__graft_entry__.smoke()`` to check one
small GPU invocation, and by ``bench.py``'s ``cpu_baseline`` leg.  It shares no
code with the HIP library.
"""

from .prism_dg import (  # noqa: F401
    TRI_PTS, TRI_W, GL2_PTS, GL2_W, GL3_PTS, GL3_W,
    PrismMesh,
    reference_basis,
    mass_matrix,
    advective_residual,
    volume_term,
    lateral_flux_term,
    horizontal_flux_term,
    column_system,
    RK3_COEFFS,
    explicit_operator,
    rk_stage,
    vertical_diffusion_matrix,
    vertical_diffusion_matrices,
    implicit_solve,
    step,
    mass,
    boundary_flux,
)
from . import column_dv  # noqa: F401,E402
from . import split_imex  # noqa: F401,E402
from . import horizontal_diffusion  # noqa: F401,E402
