"""MI355X (gfx950) butterfly counting and tip / wing decomposition.

The work runs in libpbng.so (hand-written HIP, C ABI in include/pbng.h);
``binding`` marshals arguments to it.  PyTorch is used only for device
memory.
"""
from .binding import (  # noqa: F401
    COUNT_EDGE,
    COUNT_VERTEX_U,
    COUNT_VERTEX_V,
    SIDE_U,
    SIDE_V,
    BOUND_PLAIN,
    BOUND_LEARNED,
    BOUND_RANDOM,
    BOUND_PAPER,
    F_NO_BATCH,
    F_NO_DENSE_TILE,
    F_NO_DYNAMIC,
    F_HOST_ROUNDS,
    F_SHORT_PROBE,
    Context,
    DeviceGraph,
    PbngError,
    count,
    host_csr,
    make_opts,
    tip,
    tip_batch,
    tip_schedule,
    tip_hinted,
    tip_components,
    wing_components,
    tip_features,
    wing_batch,
    to_numpy_u64,
    wing,
    load,
    LIB_PATH,
)
