"""CPU oracle for PackSELL SpMV -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously-correct CPU implementation of what the GPU library
computes, written from the paper (PackSELL: A Sparse Matrix Format for
Precision-Agnostic High-Performance SpMV, Suzuki & Iwashita):

* ``formats``  -- value quantisers (FP16, E8MY, fixed point) and the 32-bit
  word codec (sec. 4.2, the packing/unpacking listing and its two examples).
* ``packsell`` -- the encoder (delta encoding eq. 2 with the block-uniform
  left offset eq. 4, dummy insertion and SELL-C-sigma alignment, sec. 4.1 and
  4.3), the decoder, and the product of sec. 4.4 as a row-by-row decode
  followed by a float64 dot product.
* ``linalg``   -- float64 CSR SpMV / transposed SpMV / value gradients (the
  plain definitions y = A_q x), textbook CG and the inner-outer CG of
  sec. 5.2.2.
* ``csr_core.c`` -- the float64 CSR SpMV loop in C (built by ``build()``),
  used for sizes numpy loops cannot reach and timed as the CPU baseline.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import or run anything in this package.  It shares no code
with the GPU library (``paper_2604_13433_amd``) and imports nothing from it;
seeded inputs come from ``paper_2604_13433_amd.workloads``, which holds no
PackSELL arithmetic.

Readings of points the paper leaves open are listed in each function's
docstring.  Parity unpinned: the iteration counts of the inner-outer CG
against the paper (its convergence plots are not available).
"""
