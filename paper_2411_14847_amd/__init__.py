"""MI355X (gfx950) hot path of per-timestep Gaussian-splatting streaming (DASS, arXiv 2411.14847).

The computation lives in libdass.so (hand-written HIP kernels behind the C ABI of
include/dass.h); this package only marshals torch device tensors into those calls.
"""
from ._ffi import DASS_ADJOINT, DASS_FWD, EXPORTS, LIB_PATH, MAX_VIEWS, MissingLibrary  # noqa: F401
from .api import Context, DassError, GaussianBuffers, HashField, RenderOut, camera_struct, geometric_res, n_sh  # noqa: F401
