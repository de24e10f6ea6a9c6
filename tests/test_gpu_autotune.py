"""GPU checks of the autotuner: the byte model matches the built matrices,
the chosen configuration respects the precision floor, and the cache
returns the same answer without re-tuning."""
import os

import pytest
import torch

from paper_2604_13433_amd import autotune as T
from paper_2604_13433_amd import binding as B
from paper_2604_13433_amd import workloads as W

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def test_tune_stencil(tmp_path):
    a = W.stencil((40, 40, 40), "star", 2, 0.5)
    cache = os.path.join(tmp_path, "tune.json")
    r = T.tune(a.rowptr, a.col, a.val, a.n, a.m, "e8my", min_mantissa=13, cache_path=cache,
               sigma_list=(64, 256, 4096), device=DEV)
    assert 22 - r["D"] >= 13
    # the chosen configuration's byte model equals the built matrix's
    A = B.encode(a.rowptr, a.col, a.val, a.n, a.m, "e8my", r["D"], r["C"], r["sigma"],
                 B.IMPLICIT, DEV)
    assert A.bytes_per_spmv() == r["bytes"]
    timed = [c for c in r["candidates"] if "us" in c]
    assert timed and r["us"] == min(c["us"] for c in timed)
    again = T.tune(a.rowptr, a.col, a.val, a.n, a.m, "e8my", min_mantissa=13,
                   cache_path=cache, device=DEV)
    assert again == r


def test_tune_fp16_single_D():
    a = W.m1_poisson2d()
    r = T.tune(a.rowptr, a.col, a.val, a.n, a.m, "fp16", 10, sigma_list=(64, 256), device=DEV)
    assert r["D"] == 15
