"""MI355X (gfx950) HIP implementation of the extruded-prism DG tracer step.

The compute path is libslimdg.so (``csrc/``, C ABI in ``include/slimdg.h``);
``slimdg`` is its ctypes binding.
"""

from .slimdg import (  # noqa: F401
    SDG_DV_MAX_COMP,
    SDG_DV_VD,
    SDG_DV_VU,
    SDG_FP32,
    SDG_FP32_STATE_FP64_SOLVE,
    SDG_FP64,
    SDG_PROBE_COPY,
    SDG_PROBE_READ,
    SDG_PROBE_WRITE,
    SDG_SCHEME_SPLIT_IMEX,
    SDG_SCHEME_SSPRK3_LIE,
    EXPORTED,
    LIB_PATH,
    Mesh,
    SlimDG,
    SlimDGError,
    Tuning,
    from_workload,
    load_library,
    stream_probe,
)
from .autograd import (  # noqa: F401
    MNorm,
    TracerSteps,
)
