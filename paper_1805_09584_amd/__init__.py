"""Python binding of libndtm (the HIP multi-shift twisted-mass solver for gfx950).

Argument marshalling only: every step runs in the library's HIP kernels.
PyTorch supplies device memory (complex128 CUDA tensors) and the current
stream.  Importing this package does not load the library; the first call
does, and raises if the shared library has not been built.
"""
from __future__ import annotations

from .binding import (  # noqa: F401
    NDTM_GUESS_LAGRANGE,
    NDTM_GUESS_MMS,
    NDTM_GUESS_MLP,
    NDTM_GUESS_PROJECTION,
    NDTM_GUESS_ZERO,
    NDTM_NMMS_AUTO,
    NDTM_OP_DFULL,
    NDTM_OP_HOP_EO,
    NDTM_OP_HOP_OE,
    NDTM_OP_QHAT,
    NDTM_OP_QHAT2,
    NDTM_OP_SHAT_SHIFT,
    NDTM_PREC_F16,
    NDTM_PREC_F32,
    NDTM_PREC_F32_H16,
    NDTM_PREC_F64,
    NDTM_SMOOTH_MR,
    NDTM_SMOOTH_SAP,
    Context,
    NdtmError,
    PROF_CLASSES,
    lib_path,
    hybrid_split,
    load_library,
    zolotarev,
)


def trained_weights_path():
    """Path of the shipped weights of the learned guess proposer (flat FP32, key 'w')."""
    import os

    return os.path.join(os.path.dirname(os.path.abspath(__file__)), "data", "guess_mlp.npz")
