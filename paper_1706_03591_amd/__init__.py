"""MI355X-native compressive spectral clustering of static and dynamic graphs.

The compute path is the HIP library ``libcsc.so`` (C ABI in ``include/csc.h``); this
package only marshals arguments to it.  Build it with ``python -m paper_1706_03591_amd.build``.
"""

from .binding import (  # noqa: F401
    BF16, BF16S, BF16S_ITER, DAMP_JACKSON, DAMP_NONE, F16, F16S, F16S_ITER, F32, F64,
    LAP_COMBINATORIAL, LAP_NORMALIZED,
    CscError, DynamicCSC, Graph, cheb_coeffs, compressive_kmeans,
    cheb_filter, cheb_moments, dot, eigcount, gather_probe, eigcount_from_moments, filter_backward, kmeans,
    kmeans_assign, kmeans_seed, kmeans_update, lib, randn, timing_enable, timing_read,
    timing_reset, uniforms, version, weight_gradient, workspace,
)
from .autograd import ChebFilter, cheb_filter_autograd  # noqa: F401
