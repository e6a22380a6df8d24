"""MI355X (gfx950) dashSVD: randomized truncated SVD with dynamic shifts and
PVE accuracy control (Feng, Yu, Xie, Tang), as hand-written HIP kernels behind
a C ABI (include/dashsvd.h).  This package is the thin Python binding."""
from .dashsvd import (  # noqa: F401
    BF16, F32, F64, DashSVD, DashSVDError, Info, k_cholqr, k_eig, k_eig_onesided, k_eig_prof, k_eig_tridiag,
    k_gaussian, k_gram, k_philox_raw, k_rescale, k_sort_index, k_spmm, k_spmm_static, k_transpose, lib, make_csr, workspace_size,
)
