"""MI355X-native rational-Krylov (R-MATEX) transient solver for linear RC
power-distribution networks.

The compute path is the C-ABI library libmatex.so (HIP kernels for gfx950 plus
host C++ planning and factorisation); `matex` is its thin Python binding."""
