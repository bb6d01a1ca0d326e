"""FP64 CPU oracle for Tucker-ALS (HOOI) -- test infrastructure only.

Imported by tests/, by ``__graft_entry__.smoke()`` and by the CPU-baseline leg of
bench.py; never by the library.  It shares no code with the HIP path.
"""

from .hooi_ref import (  # noqa: F401
    HooiResult,
    fit_from_norms,
    gram,
    hooi,
    hooi_update,
    identity_factors,
    leading_eigvecs,
    project_all,
    project_all_but,
    reconstruct,
    sign_fix,
    st_hosvd_factors,
    thosvd_factors,
    ttm,
    unfold,
    validate,
)
from .compare import compare, recon_diff, sin_theta_max, orthonormality_error  # noqa: F401
