"""MI355X (gfx950) Jacobi-PCA for hyperspectral cubes.

The compute path is libpca.so (hand-written HIP kernels behind a C ABI,
include/pca.h); this package only marshals torch tensors into it.
"""

from ._lib import (  # noqa: F401
    COV_MODES,
    LIB_PATH,
    PCA_COV_BF16X3,
    PCA_COV_BF16X4,
    PCA_COV_FP16X3,
    PCA_COV_F32,
    PCA_IN_F32,
    PCA_IN_U16,
    PCA_IN_F32_BSQ,
    PCA_IN_U16_BSQ,
    PCA_JACOBI_FP64_ANGLES,
    PCA_JACOBI_OVERLAP_REPLAY,
    PCA_JACOBI_ONE_CU,
    PCA_JACOBI_BLOCK,
    JACOBI_FORMS,
    PCA_OP_CENTER,
    PCA_OP_COVARIANCE,
    PCA_OP_JACOBI,
    PCA_OP_BACKWARD,
    PCA_OP_PROJECT,
    PCAError,
    library,
    new_info,
    pca_backward,
    pca_center,
    pca_covariance,
    pca_jacobi_eigh,
    pca_jacobi_eigh_noalloc,
    pca_project,
    pca_workspace_size,
    read_info,
    set_wait_shift,
    workspace,
)
from ._lib import PCABatchTuning, PCACube, pca_batched, pca_batched_workspace_size  # noqa: F401
from .batched import BatchedPCA  # noqa: F401
from .api import DEFAULT_MAX_SWEEPS, DEFAULT_TOL, PCAFunction, PCAPipeline, PCAResult, PCAStream, pca_autograd, run  # noqa: F401
