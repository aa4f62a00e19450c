"""MI355X (gfx950) SPH density/force path over hierarchical cells with sorted
cell-pair sweeps (arXiv:1309.3783, Section II).

The compute runs in libsphcell.so (HIP, built by ``build.py``); this package
only marshals arguments (``binding``) and drives batches and request streams
(``pipeline``, ``serve``) and time stepping (``integrate``).
"""
from .binding import (Batch, Context, DensityOut, ForceOut, SphError, Tree, batch_from_sets,  # noqa: F401
                      footprint, lib, params, solve_with_rebuild, workspace_size, SPH_FLAG_PAIR_HASH,
                      SPH_FLAG_NO_BLOCK_SKIP, SPH_FLAG_SORTED_ONLY, SPH_OK, SPH_E_ARG, SPH_E_CAPACITY,
                      SPH_E_REBUILD, SPH_E_NOCONV, SPH_E_STATE, SPH_E_WORKSPACE, kick, drift, cfl_dt)
