"""FP64 CPU oracle for the Jacobi-PCA hot path.

TEST INFRASTRUCTURE ONLY. This package is the plain, slow reference that the
GPU library is checked against. Only the tests, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py`` may import it; the GPU product path
never does, and the two share no code (the seeded input generators in
``synth`` are the only common dependency, and they hold none of the method's
arithmetic).
"""

from .pca_oracle import (  # noqa: F401
    ORDERINGS,
    backward,
    band_mean,
    build_library,
    center,
    covariance,
    covariance_entries,
    jacobi_eigh,
    jacobi_raw,
    pca,
    project,
    project_rows,
    reconstruction_loss,
    sign_fix,
    sort_desc,
)
