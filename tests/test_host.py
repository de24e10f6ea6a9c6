"""Host-side behaviour that needs no GPU: the binding refuses to run without
the built library, and the extra generators have the structure they claim."""
import importlib

import numpy as np
import pytest

from paper_2604_13433_amd import workloads as W


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_2604_13433_amd import binding as B

    monkeypatch.setattr(B, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(B, "_lib", None)
    with pytest.raises(RuntimeError, match="missing"):
        B.lib()


def test_block_stencil_structure():
    a = W.block_stencil((5, 4, 3), 3, 1)
    assert a.n == 180
    # interior unknowns couple to 27 points x 3 unknowns
    assert a.row_lengths().max() == 81
    cols = a.col[a.rowptr[40]:a.rowptr[41]].astype(np.int64)
    runs = np.split(cols, np.nonzero(np.diff(cols) != 1)[0] + 1)
    assert all(len(r) % 3 == 0 for r in runs)
    assert np.allclose(np.add.reduceat(np.abs(a.val), a.rowptr[:-1]), 1.0)


def test_batch_generator_sizes():
    mats = W.m5_batch(count=6, n_lo=1000, n_hi=5000, seed=1)
    assert len(mats) == 6
    assert all(m.n == m.m for m in mats)
    assert mats[0].name.startswith("b0_5pt") and mats[1].name.startswith("b1_7pt")


_ARG_CHECKS = r"""
import torch, pytest
from paper_2604_13433_amd import binding as B
d = B.CMatrix(); d.n, d.m = 5, 10
A = B.PackSELLMatrix(d, {}, torch.device("cpu"))
cases = [
    (lambda: B.spmv(A, torch.zeros(9)), "10 rows"),
    (lambda: B.spmv(A, torch.zeros(10, dtype=torch.float64)), "torch.float32"),
    (lambda: B.spmv(A, torch.zeros(10)), "GPU tensor"),
    (lambda: B.spmv_t(A, torch.zeros(4)), "5 rows"),
    (lambda: B.spmv_f64(A, torch.zeros(10)), "torch.float64"),
]
for fn, msg in cases:
    try:
        fn()
    except ValueError as e:
        assert msg in str(e), (msg, str(e))
    else:
        raise SystemExit("no error for " + msg)
print("ok")
"""


@pytest.mark.parametrize("opt", [[], ["-O"]])
def test_binding_argument_errors_survive_optimised_python(opt):
    """Shape, dtype and device errors are raised before any library call,
    also under ``python -O`` (which strips asserts)."""
    import os
    import subprocess
    import sys

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, *opt, "-c", _ARG_CHECKS], cwd=root,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stderr[-2000:]
