"""MI355X-native ML(n)BiCGStab: a HIP library (libmlbicgstab.so, C ABI in
include/mlbicgstab.h) and its Python binding.

    from paper_1106_3678_amd import binding
    dA = binding.to_device(A_scipy)
    s = binding.Solver(dA, n=4, tol=1e-10, maxit=2000)
    res = s.solve(b, x, Q)     # torch tensors on the GPU
"""
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libmlbicgstab.so")


def lib_built() -> bool:
    return os.path.exists(LIB_PATH)
