"""ctypes binding of libdmrg.so (argument marshalling only).

Every function of include/dmrg.h is declared here with the same name.  The
library is loaded from this package directory; a missing or unloadable
library raises immediately -- there is no fallback implementation.
"""

from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdmrg.so")

c_int, c_int32, c_int64, c_double, c_void_p, c_char_p = (
    C.c_int, C.c_int32, C.c_int64, C.c_double, C.c_void_p, C.c_char_p)
P = C.POINTER

DMRG_FP64, DMRG_FP32, DMRG_BF16, DMRG_BF16X3 = 0, 1, 2, 3
STATUS = {0: "DMRG_OK", 1: "DMRG_E_INVAL", 2: "DMRG_E_NOMEM", 3: "DMRG_E_HIP",
          4: "DMRG_E_NOCONV", 5: "DMRG_E_NUMERIC", 6: "DMRG_E_STATE", 7: "DMRG_E_IO"}


class MpoOpts(C.Structure):
    _fields_ = [("switch_bond", c_int), ("compress_tol", c_double), ("basis", c_int)]


class SweepOpts(C.Structure):
    _fields_ = [("prec", c_int), ("dav_tol", c_double), ("dav_max_iter", c_int),
                ("dav_max_space", c_int), ("dav_keep", c_int), ("svd_cutoff", c_double),
                ("refine_tol", c_double), ("precond", c_int), ("collect", c_int), ("mlp", c_void_p)]


class SweepStat(C.Structure):
    _fields_ = [("energy", c_double), ("discarded", c_double), ("seconds", c_double),
                ("sigma_flops", c_double), ("sigma_seconds", c_double),
                ("sigma_calls", c_int64), ("gemm_seconds", c_double), ("gemm_launches", c_int64),
                ("dav_iters", c_int64), ("max_bond", c_int32),
                ("n_steps", c_int32), ("precond_fallbacks", c_int64), ("samples", c_int64),
                ("max_residual", c_double), ("unconverged", c_int64)]


ALLOC_FN = C.CFUNCTYPE(c_void_p, C.c_size_t, c_void_p)
FREE_FN = C.CFUNCTYPE(None, c_void_p, c_void_p)


class Allocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", c_void_p)]


# name -> (restype, argtypes)
SIGNATURES = {
    "dmrg_ctx_create": (c_int, [c_int, c_void_p, P(Allocator), P(c_void_p)]),
    "dmrg_ctx_destroy": (None, [c_void_p]),
    "dmrg_last_error": (c_char_p, [c_void_p]),
    "dmrg_build_mpo": (c_int, [c_void_p, P(c_double), P(c_double), c_int, c_int, c_int,
                               P(MpoOpts), P(c_void_p)]),
    "dmrg_build_sum_mpo": (c_int, [c_void_p, P(c_double), P(c_double), c_int, c_int, c_int, c_int,
                                   P(c_void_p)]),
    "dmrg_mpo_affine": (c_int, [c_void_p, c_void_p, c_double, c_double, P(c_void_p)]),
    "dmrg_debug_svd": (c_int, [c_void_p, c_int, P(c_int32), P(c_int32), P(c_double), P(c_double), P(c_double),
                               P(c_double), c_int]),
    "dmrg_mps_apply": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int, P(c_void_p),
                               P(c_double), P(c_double)]),
    "dmrg_mpo_bond_dims": (c_int, [c_void_p, P(c_int32)]),
    "dmrg_mpo_channels": (c_int, [c_void_p, c_int, P(c_int32)]),
    "dmrg_mpo_singular_values": (c_int, [c_void_p, c_int, P(c_int64), P(c_double)]),
    "dmrg_mpo_site_entries": (c_int, [c_void_p, c_int, P(c_int64), P(c_int32), P(c_double)]),
    "dmrg_mpo_free": (None, [c_void_p]),
    "dmrg_mps_n_values": (c_int, [c_void_p, c_int, P(c_int64)]),
    "dmrg_two_site_index": (c_int, [P(c_int32), c_int, P(c_int32), c_int, P(c_int64), P(c_int64)]),
    "dmrg_sigma_model_flops": (c_int, [c_void_p, c_int, P(c_int32), c_int, P(c_int32), c_int,
                                       P(c_double)]),
    "dmrg_mps_random": (c_int, [c_void_p, c_void_p, c_int, P(c_double), c_int64, P(c_void_p)]),
    "dmrg_mps_import": (c_int, [c_void_p, c_void_p, P(c_int32), P(c_int32), P(c_double), c_int64,
                                c_int, P(c_void_p)]),
    "dmrg_mps_bond": (c_int, [c_void_p, c_int, P(c_int32), P(c_int32)]),
    "dmrg_mps_center": (c_int, [c_void_p, P(c_int)]),
    "dmrg_mps_free": (None, [c_void_p]),
    "dmrg_mps_save": (c_int, [c_void_p, c_void_p, c_char_p]),
    "dmrg_mps_load": (c_int, [c_void_p, c_void_p, c_char_p, P(c_void_p)]),
    "dmrg_psi_size": (c_int, [c_void_p, P(c_int64)]),
    "dmrg_psi_export": (c_int, [c_void_p, c_void_p, P(c_double)]),
    "dmrg_sigma": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int, P(c_double)]),
    "dmrg_sigma_noalloc": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "dmrg_sigma_diag": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "dmrg_env_export": (c_int, [c_void_p, c_void_p, c_int, c_int, P(c_double)]),
    "dmrg_env_size": (c_int, [c_void_p, c_int, c_int, P(c_int64)]),
    "dmrg_env_import": (c_int, [c_void_p, c_void_p, c_int, c_int, P(c_double), c_int64]),
    "dmrg_debug_gemm": (c_int, [c_void_p, c_int, c_int, c_int, c_int, c_int, c_int, c_double,
                                c_void_p, c_int, c_void_p, c_int, c_void_p, c_int, c_int, c_int, c_int, c_int]),
    "dmrg_sweep_opts_default": (None, [P(SweepOpts)]),
    "dmrg_sweep": (c_int, [c_void_p, c_void_p, c_void_p, c_int, c_int, P(SweepOpts),
                           P(SweepStat), P(c_double)]),
    "dmrg_step": (c_int, [c_void_p, c_void_p, c_void_p, c_int, c_int, P(SweepOpts),
                          P(c_double), P(SweepStat)]),
    "dmrg_energy": (c_int, [c_void_p, c_void_p, c_void_p, P(c_double)]),
    "dmrg_mps_move": (c_int, [c_void_p, c_void_p, c_void_p, c_int]),
    "dmrg_sweep_batched": (c_int, [c_void_p, c_int, P(c_void_p), P(c_void_p), P(c_int), c_int,
                                   P(SweepOpts), P(SweepStat), P(c_double)]),
    "dmrg_psi_import": (c_int, [c_void_p, c_void_p, P(c_double)]),
    "dmrg_solve": (c_int, [c_void_p, c_void_p, c_void_p, P(SweepOpts), P(c_double), P(c_double),
                           P(SweepStat)]),
    "dmrg_autotune": (c_int, [c_void_p, c_void_p, c_void_p, c_int, c_int, c_char_p, c_int64]),
    "dmrg_tune_table": (c_int, [c_char_p, c_int64, P(c_int64)]),
    "dmrg_tune_table_load": (c_int, [c_char_p]),
    "dmrg_mlp_create": (c_int, [c_void_p, P(C.c_float), C.c_uint64, c_int64, P(c_void_p)]),
    "dmrg_mlp_free": (None, [c_void_p]),
    "dmrg_mlp_params": (c_int, [c_void_p, c_void_p, P(C.c_float)]),
    "dmrg_mlp_forward": (c_int, [c_void_p, c_void_p, c_void_p, c_int64, c_void_p]),
    "dmrg_mlp_loss_grad": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_int64, c_void_p,
                                   P(c_double)]),
    "dmrg_mlp_adam_step": (c_int, [c_void_p, c_void_p, c_void_p, c_double]),
    "dmrg_mlp_static": (c_int, [c_void_p, c_void_p, P(C.c_float)]),
    "dmrg_mlp_features": (c_int, [c_void_p, c_void_p, c_double, c_void_p, c_void_p, c_void_p]),
    "dmrg_mlp_targets": (c_int, [c_void_p, c_void_p, c_void_p, c_double, c_void_p, c_void_p, c_int64,
                                 c_void_p]),
    "dmrg_mlp_dataset": (c_int, [c_void_p, c_void_p, P(c_int64), P(C.c_float), P(C.c_float)]),
    "dmrg_mlp_train": (c_int, [c_void_p, c_void_p, c_int, c_int, c_double, C.c_uint64, P(c_double)]),
}
MLP_FEATURES, MLP_PARAMS = 12, 5057

_lib = None


def load():
    """Load libdmrg.so from the package directory (raises if absent)."""
    global _lib
    if _lib is not None:
        return _lib
    # torch ships its own HIP runtime; loading it first makes the library bind
    # to that same runtime instead of a second copy from the ROCm install
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libdmrg.so is not built (run __graft_entry__.build() or "
                           "python -m paper_1605_02611_amd.build); there is no fallback")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib
