"""PackSELL sparse matrix-vector products on AMD MI355X (gfx950).

The computation lives in ``libpksell.so`` (HIP kernels behind the C ABI of
include/pksell.h); ``binding`` marshals torch tensors into it.  Importing
the package loads nothing; the first call into ``binding`` loads the library
and raises if it has not been built (there is no CPU fallback).

    from paper_2604_13433_amd import binding as B
    A = B.encode(rowptr, col, val, n, m, fmt="e8my", D=9)
    y = B.spmv(A, x)
"""

__all__ = ["binding", "autograd", "autotune", "workloads", "build"]
