"""Differentiable PackSELL product for torch.autograd.

``PackSELLLinear`` holds the CSR structure (rowptr, col) and the encoder
parameters; its ``values`` tensor is the differentiable quantity.  Forward
encodes the values into PackSELL words (cached until the values change) and
runs ``pksell_spmv``; backward computes grad_x = A_q^T g and
d<g, A x>/d a_ij = g_i . x_j (``pksell_grad_values``).  Quantisation is
treated as the identity in the value gradient (straight-through).

grad_x has two forms.  ``adjoint="atomic"`` runs ``pksell_spmv_t`` over the
forward product's own words (a float32 atomic scatter).  ``adjoint=
"transpose"`` (FP16 and E8MY only) keeps a second PackSELL matrix holding
(A_q)^T, encoded from the device transpose of the CSR, and runs the forward
product on it: no atomics, at the forward product's speed, for twice the
matrix memory.
"""
from __future__ import annotations

import torch

from . import binding as B


class _SpMV(torch.autograd.Function):
    @staticmethod
    def forward(ctx, values, x, A, rowptr, At=None):
        ctx.A = A
        ctx.At = At
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
            gx = B.spmv(ctx.At, g) if ctx.At is not None else B.spmv_t(ctx.A, g)
        return gv, gx, None, None, None


class PackSELLLinear:
    """y = A(values) x with A stored in PackSELL on the GPU.

    ``rowptr`` (int64, n+1) and ``col`` (int32, nnz) fix the sparsity
    pattern; ``values`` (float32, nnz, may require grad) are the entries.
    Rows come out in the original order (implicit permutation).
    """

    def __init__(self, rowptr, col, values: torch.Tensor, n: int, m: int, fmt="e8my", D=9,
                 C=64, sigma=256, adjoint="atomic"):
        if adjoint not in ("atomic", "transpose"):
            raise ValueError("adjoint must be 'atomic' or 'transpose'")
        if adjoint == "transpose" and fmt in ("fix", B.FIX):
            raise ValueError("FIX quantises per row: use adjoint='atomic'")
        self.device = values.device
        self.rowptr = torch.as_tensor(rowptr, dtype=torch.int64).to(self.device)
        self.col = torch.as_tensor(col, dtype=torch.int32).to(self.device)
        self.values = values
        self.n, self.m = n, m
        self.params = dict(fmt=fmt, D=D, C=C, sigma=sigma)
        self.adjoint = adjoint
        self._A = None
        self._At = None
        self._version = None

    def _refresh(self):
        ver = (self.values.data_ptr(), self.values._version)
        if self._A is None or ver != self._version:
            with torch.no_grad():
                v = self.values.detach()
                self._A = B.encode(self.rowptr, self.col, v, self.n, self.m,
                                   perm_mode=B.IMPLICIT, device=self.device, **self.params)
                if self.adjoint == "transpose":
                    self._At = B.encode_transpose(self.rowptr, self.col, v, self.n, self.m,
                                                  perm_mode=B.IMPLICIT, device=self.device,
                                                  **self.params)
            self._version = ver

    def matrix(self) -> B.PackSELLMatrix:
        """The encoded matrix, re-encoded when the values changed."""
        self._refresh()
        return self._A

    def transposed(self) -> B.PackSELLMatrix | None:
        """The encoded (A_q)^T (adjoint="transpose"), else None."""
        self._refresh()
        return self._At

    def __call__(self, x: torch.Tensor) -> torch.Tensor:
        A = self.matrix()
        return _SpMV.apply(self.values, x, A, self.rowptr, self._At)


def spmv(values: torch.Tensor, x: torch.Tensor, A: B.PackSELLMatrix, rowptr) -> torch.Tensor:
    """Functional form: y = A x, differentiable in ``values`` and ``x`` (the
    encoded ``A`` must hold ``values``)."""
    return _SpMV.apply(values, x, A, rowptr)
