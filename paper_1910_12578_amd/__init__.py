"""MI355X-native SDC reactive-flow update (Castro, Sec. 2, Eq. 2).

`SDC` wraps a handle of libsdc.so: the advective term A(U), the reactive
source R(U), the per-zone Newton reaction solve, the node-to-node SDC sweep and
whole time steps, all computed by HIP kernels on the GPU.
"""
from ._binding import AMR, SDC, SDCError, SDC_FP64, SDC_MIXED, config_from_workload  # noqa: F401
