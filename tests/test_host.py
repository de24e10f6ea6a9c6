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
