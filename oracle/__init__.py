"""FP64 CPU oracle for per-pixel Kronecker STAP.

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain reference that the
GPU library is checked against.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import it; the library itself never
does, and shares no code with it.

Every function follows the paper (Greenewald, Zelnio & Hero, "Kronecker STAP
and SAR GMTI", SPIE 2016) step by step, in complex128, with NumPy/LAPACK
(`numpy.linalg.eigh`) as the only library primitives.  Readings adopted where
the paper is silent or garbled are listed at the top of `kron_stap.py`.

Pins (what fixes each function independently of itself) live in
`tests/test_oracle_pins.py`.  Parity unpinned: nothing in this package; the
Gotcha-data experiments and figure values of the paper are not reproduced.
"""
from .kron_stap import (  # noqa: F401
    OracleConfig,
    default_stencil,
    stencil_window,
    valid_region,
    snapshots,
    sample_covariance,
    rearrange,
    rearrange_direct,
    eig_truncate,
    top_eigvecs,
    lr_kron,
    kron_stap_statistic,
    gamma_upper_quantile,
    kron_stap_pixels,
    kron_stap_frame,
    relative_gaps,
)
