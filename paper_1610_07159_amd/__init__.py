"""Halfway-domain scene flow on MI355X (gfx950): a C-ABI HIP library
(libsf.so, include/sf.h) and its Python binding."""
from . import sf  # noqa: F401  (raises ImportError if libsf.so is missing)
from .solver import SceneFlowSolver, calib_from_dict  # noqa: F401
