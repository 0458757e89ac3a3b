"""MI355X (gfx950) box code for the 2D Laplace volume potential on adaptive quadtrees.

The hot path of the paper's bulk solve (Sec. 4.2, eq. (vbulk)) as hand-written HIP kernels behind
a C ABI (include/volpot.h); this package holds the HIP sources (csrc/), the in-tree build
(build.py) and the ctypes binding (volpot.py).
"""
from .volpot import (  # noqa: F401
    LayerPlan,
    PointPlan,
    StripPlan,
    EXPORTED,
    Plan,
    VolpotError,
    autotune,
    build_tree,
    lib,
    near_relation,
    nodes,
    validate_tree,
    volume_potential,
)
