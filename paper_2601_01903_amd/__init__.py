"""MI355X (gfx950) implementation of the Faithful Shapley Interaction operator
v -> FSI(v) (TT-FSI, arXiv 2601.01903): C ABI in include/fsi.h, HIP kernels in
csrc/, Python binding in fsi.py."""
from .fsi import (  # noqa: F401
    BatchPlan,
    Forest,
    FsiError,
    Plan,
    load,
    num_outputs,
)
