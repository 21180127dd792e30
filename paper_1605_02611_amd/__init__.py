"""MI355X-native two-site ab initio DMRG (arXiv 1605.02611 hot path).

The compute lives in libdmrg.so (HIP kernels for gfx950 behind the C ABI of
include/dmrg.h); this package only marshals arguments to it.
"""

from ._lib import DMRG_BF16, DMRG_BF16X3, DMRG_FP32, DMRG_FP64, LIB_PATH, load  # noqa: F401
from .api import (Context, DmrgError, Mlp, Mpo, Mps, autotune, default_opts, mlp_features, two_site_index,  # noqa: F401
                  mlp_static, mlp_targets, sigma_model_flops, sweep_batched, tune_table, tune_table_load)
