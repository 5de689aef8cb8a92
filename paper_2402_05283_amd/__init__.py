"""MI355X-native CPRA hot path: HIP kernels behind a C ABI (libcpra.so).

The Python layer only marshals arguments; see include/cpra.h for the ABI.
"""
from ._lib import (  # noqa: F401
    AMP_F16, AMP_F32, ER, HIO, INSERT_BILINEAR, INSERT_NEAREST, RAAR, REAL_F32, REAL_F64, WRAP_MIRROR,
    WRAP_PLAIN, CpraError, Plan, Tuning, autotune, coupling_table, iterate_batch, load, get_batch_fusion, make_params, set_batch_fusion,
    slice_cells,
    workspace_size,
)
