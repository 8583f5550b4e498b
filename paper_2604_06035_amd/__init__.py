"""MI355X (gfx950) multigrid Poisson solver for one level of an oct-based mesh.

The compute path is the HIP library ``libmg.so`` (C ABI in ``include/mg.h``);
``abi`` is its ctypes binding.  Build with ``python -m paper_2604_06035_amd.build``.
"""
from . import abi  # noqa: F401
from .abi import (MG_ERR_ARG, MG_ERR_DIVERGED, MG_ERR_NESTING, MG_ERR_TABLE, MG_NOT_CONVERGED, MG_OK,  # noqa: F401
                  MG_PREC_FP64, MG_PREC_MIXED, MgError, mg_build_level, mg_destroy_level, mg_get_neighbors,
                  mg_hierarchy_info, mg_residual_norm, mg_solve)
