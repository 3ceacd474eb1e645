"""MI355X (gfx950) CSR sparse-matrix products: y <- A x and Y <- A X.

A thin binding over libspx.so (C ABI in include/spx.h).  Tensors must be on
the GPU; there is no CPU path, and importing an operation without the built
library raises.
"""
from ._lib import PlanOpts, SpxError, missing_symbols  # noqa: F401
from .ops import (BCSR, CSR, CSCIndex, CSCValueMap, Plan, bandwidth, banded_opts, bcsr_spmm, bcsr_spmv,  # noqa: F401
                  csc_value_map, default_opts, degree_order, from_coo, from_coo_host, permute, validate_host, values_to_csc,
                  probe, rcm, sddmm, sddmm_saved, spmm, spmv, spmv_save, spmv_t, tile_lines,
                  transpose_index, ucld, validate, vector_access, version)
from .autograd import GradContext, SpMVFunction, spmv_autograd  # noqa: F401
