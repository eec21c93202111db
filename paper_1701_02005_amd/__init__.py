"""MI355X (gfx950) solver for the coupled Navier-Stokes / Poisson-Nernst-Planck
equations of sheared electrolyte between two sliding charged walls, after
Ostilla-Monico & Lee, arXiv:1701.02005.  The compute path is the HIP library
``libnspnp.so`` (C ABI in include/nspnp.h); this package binds it."""
from .binding import (STATS_NAMES, Config, Ensemble, Mlp, NsPnpError, Solver, grid, load_library,  # noqa: F401
                      poisson_solve_noalloc, workspace_bytes)
from . import configs  # noqa: F401
