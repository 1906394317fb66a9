"""MI355X-native (gfx950) Godunov step for compressible CT-MHD and multifluid dust.

The update of the paper's method (reconstruction of primitives, HLLE/HLLD face fluxes,
Gardiner-Stone constrained-transport EMFs and face-field update, conserved update in
the two-register stage form, IMEX2P with the closed-form implicit drag, CFL
reduction) runs in hand-written HIP kernels behind the C ABI of include/mhd950.h,
for one periodic grid (``Sim``) or a batch of uneven self-periodic meshblocks
(``Batch``);
this package holds the ctypes binding (``binding``) and the seeded synthetic inputs
(``inputs``).  Importing the package loads nothing; the library is opened on first
use and its absence is an error.
"""
from .binding import (Batch, Closure, Domain, MhdError, box_filter, Sim, load_library, make_grid, make_physics, make_scheme,  # noqa: F401
                      mhd_create, mhd_destroy, mhd_diagnostics, mhd_dt_cfl, mhd_get_state,
                      mhd_set_state, mhd_state_len, mhd_step, mhd_strerror, mhd_timing_enable,
                      mhd_timing_name, mhd_timing_read, mhd_workspace_bytes,
                      mhd_batch_create, mhd_batch_destroy, mhd_batch_dt_cfl, mhd_batch_get_shapes,
                      mhd_batch_get_state, mhd_batch_set_shapes, mhd_batch_set_state,
                      mhd_batch_state_len, mhd_batch_step, mhd_batch_tune,
                      mhd_batch_workspace_bytes)
