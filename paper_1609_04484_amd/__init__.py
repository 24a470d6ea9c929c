"""MI355X-native solver for the completed double-layer Stokes system of a
pipe filled with circular pores: HIP kernels behind a C ABI
(``include/stokes_ifmm.h``) and this thin Python binding."""
from ._lib import (FMM, MLP, BlockDiagonal, DeviceGeometry, IFMM, SbieError, SolveResult,  # noqa: F401
                   assemble, gmres, gmres_batched, ifmm_factor_batched, kernel_time,
                   kernel_timing, load, matvec, matvec_batched, matvec_noalloc, set_matvec_shape,
                   set_batched_schedule, set_matvec_symmetric, matvec_plan,
                   validate, velocity, slp_weights, slp_matvec, slp_assemble, gmres_slp,
                   slp_velocity,
                   warmstart_assemble, warmstart_features, warmstart_labels,
                   warmstart_refine)
