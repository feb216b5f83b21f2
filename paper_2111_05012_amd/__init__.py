"""MI355X-native algebraic multigrid solver for the Wilson-clover Dirac
equation (arXiv:2111.05012): HIP kernels behind the C ABI of include/wcamg.h,
with a thin ctypes binding."""
from .wcamg import (Context, WcamgError, load_library, LIB_PATH, PREC_FP64, PREC_MIXED, DEVICE, HOST,  # noqa: F401
                    OK, NOT_CONVERGED, EINVAL, ESTATE, PC_AMG, PC_BICG32, SMOOTH_POST, SMOOTH_PRE,
                    SMOOTH_BOTH, BLOCK_MR, BLOCK_EO_MR)
