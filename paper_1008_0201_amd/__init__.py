"""One-sided Jacobi eigensolver (trigonometric and hyperbolic, pointwise and
block) for AMD MI355X: a HIP library behind a C ABI (include/jevd.h) and a
thin ctypes binding (paper_1008_0201_amd.jevd)."""
