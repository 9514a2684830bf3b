"""MI355X-native RBF neural fields on surfaces: Python binding of libnfr.so.

The computations run in the HIP library (paper_2504_13379_amd/libnfr.so, C ABI
in include/nfr.h); this package only marshals torch tensors into it.
"""
from ._lib import (EXP_MH, FORM_AUTO, FORM_ONTHEFLY_BF16X3, FORM_ONTHEFLY_FP16X3, FORM_ONTHEFLY_FP32,  # noqa: F401
                   FORM_ONTHEFLY_FP32_MFMA,  # noqa: F401
                   FORM_W_BF16X3, FORM_W_FP16X3, FORM_W_FP32,  # noqa: F401
                   GAUSS_MH, LIB_PATH, PROJ_ORIGIN, PROJ_ORTHOGONAL, PROJ_PLANES, NfrError, lib)
from .api import (Batch, Context, Firing, NeuralFieldRK4, Problem, kernel_struct, quad_weights, tune,  # noqa: F401
                  tune_load)
