"""MI355X-native Chebyshev Filtered Subspace Iteration (ChFSI).

The solver is the C-ABI library libchfsi.so (include/chfsi.h), built from
hand-written gfx950 HIP kernels; ``binding`` exposes its entry points to
Python with torch tensors for device memory and streams.
"""
from .binding import (ChfsiError, ChfsiInfo, ChfsiOpts, chfsi_default_opts, chfsi_degrees,  # noqa
                      chfsi_autotune_filter, chfsi_autotune_reset, chfsi_autotune_set,
                      chfsi_degree_features, chfsi_degrees_sequence, chfsi_degrees_learned, chfsi_mlp_adam,
                      chfsi_mlp_forward, chfsi_mlp_gradient, chfsi_mlp_train,
                      chfsi_eigh_projected, chfsi_filter, chfsi_filter_noalloc, chfsi_filter_noalloc_need_bytes, chfsi_filter_defect, chfsi_filter_defect_split, chfsi_split_schedule, chfsi_lanczos_bounds, chfsi_orthonormalize,
                      chfsi_rayleigh_ritz, chfsi_reduce_standard, chfsi_reduce_workspace_bytes,
                      chfsi_solve, chfsi_solve_batch, chfsi_batch_workspace_bytes,
                      chfsi_status_string, chfsi_step_workspace_bytes,
                      chfsi_workspace_bytes, chfsi_zgemm, colmajor, header_functions, lib)
