"""Differentiable PackSELL product for torch.autograd.

``PackSELLLinear`` holds the CSR structure (rowptr, col) and the encoder
parameters; its ``values`` tensor is the differentiable quantity.  Forward
encodes the values into PackSELL words (cached until the values change) and
runs ``pksell_spmv``; backward runs ``pksell_spmv_t`` for grad_x = A_q^T g
and ``pksell_grad_values`` for d<g, A x>/d a_ij = g_i . x_j.  Quantisation is
treated as the identity in the value gradient (straight-through).  Both
adjoints read the same packed words as the forward product.
"""
from __future__ import annotations

import torch

from . import binding as B


class _SpMV(torch.autograd.Function):
    @staticmethod
    def forward(ctx, values, x, A, rowptr):
        ctx.A = A
        ctx.rowptr = rowptr
        ctx.save_for_backward(x)
        return B.spmv(A, x.contiguous())

    @staticmethod
    def backward(ctx, g):
        (x,) = ctx.saved_tensors
        g = g.contiguous()
        gv = gx = None
        if ctx.needs_input_grad[0]:
            gv = B.grad_values(ctx.A, ctx.rowptr, g, x.contiguous())
        if ctx.needs_input_grad[1]:
            gx = B.spmv_t(ctx.A, g)
        return gv, gx, None, None


class PackSELLLinear:
    """y = A(values) x with A stored in PackSELL on the GPU.

    ``rowptr`` (int64, n+1) and ``col`` (int32, nnz) fix the sparsity
    pattern; ``values`` (float32, nnz, may require grad) are the entries.
    Rows come out in the original order (implicit permutation).
    """

    def __init__(self, rowptr, col, values: torch.Tensor, n: int, m: int, fmt="e8my", D=9,
                 C=64, sigma=256):
        self.device = values.device
        self.rowptr = torch.as_tensor(rowptr, dtype=torch.int64).to(self.device)
        self.col = torch.as_tensor(col, dtype=torch.int32).to(self.device)
        self.values = values
        self.n, self.m = n, m
        self.params = dict(fmt=fmt, D=D, C=C, sigma=sigma)
        self._A = None
        self._version = None

    def matrix(self) -> B.PackSELLMatrix:
        """The encoded matrix, re-encoded when the values changed."""
        ver = (self.values.data_ptr(), self.values._version)
        if self._A is None or ver != self._version:
            with torch.no_grad():
                self._A = B.encode(self.rowptr, self.col, self.values.detach(), self.n, self.m,
                                   perm_mode=B.IMPLICIT, device=self.device, **self.params)
            self._version = ver
        return self._A

    def __call__(self, x: torch.Tensor) -> torch.Tensor:
        return _SpMV.apply(self.values, x, self.matrix(), self.rowptr)


def spmv(values: torch.Tensor, x: torch.Tensor, A: B.PackSELLMatrix, rowptr) -> torch.Tensor:
    """Functional form: y = A x, differentiable in ``values`` and ``x`` (the
    encoded ``A`` must hold ``values``)."""
    return _SpMV.apply(values, x, A, rowptr)
