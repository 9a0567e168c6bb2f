"""ChASE on MI355X: Chebyshev-filtered subspace iteration with hand-written gfx950 HIP kernels."""
