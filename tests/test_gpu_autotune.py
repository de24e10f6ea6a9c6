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
                 B.IMPLICIT, DEV, split_words=r["split_words"])
    assert A.bytes_per_spmv() == r["bytes"]
    timed = [c for c in r["candidates"] + r["csr_candidates"] if "us" in c]
    assert timed and r["us"] == min(c["us"] for c in timed)
    again = T.tune(a.rowptr, a.col, a.val, a.n, a.m, "e8my", min_mantissa=13,
                   cache_path=cache, device=DEV)
    assert again == r


def test_tune_fp16_single_D():
    a = W.m1_poisson2d()
    r = T.tune(a.rowptr, a.col, a.val, a.n, a.m, "fp16", 10, sigma_list=(64, 256), device=DEV)
    assert r["D"] == 15


def test_tune_splits_wide_slices(tmp_path):
    """Power-law rows (n = 60,000, rows up to 5000 entries) in one sigma
    window: the split widths are timed, and the chosen configuration builds
    and multiplies correctly."""
    import numpy as np

    from helpers import FMTS, SPMV_TOL, normalised_error, oracle_product

    a = W.powerlaw(60_000, seed=9)
    cache = os.path.join(tmp_path, "tune.json")
    r = T.tune(a.rowptr, a.col, a.val, a.n, a.m, "fp16", 10, C_list=(64,), sigma_list=(65536,),
               split_list=(128, 256), time_top=1, cache_path=cache, device=DEV, csr_chunks=())
    top = r["candidates"][0]
    assert set(top["split_us"]) == {"128", "256"}  # both split some slice
    assert r["split_words"] in (0, 128, 256)
    assert r["us"] == min([top["us"]] + list(top["split_us"].values()))
    A = B.encode(a.rowptr, a.col, a.val, a.n, a.m, "fp16", r["D"], r["C"], r["sigma"],
                 B.IMPLICIT, DEV, split_words=r["split_words"])
    x = W.uniform_vector(a.m, 3)
    y = B.spmv(A, torch.from_numpy(x).to(DEV)).cpu().numpy()
    ref, q = oracle_product(a, FMTS["fp16"], 15, x)
    assert normalised_error(y, ref, a, q, x) <= SPMV_TOL
    assert T.tune(a.rowptr, a.col, a.val, a.n, a.m, "fp16", 10, C_list=(64,),
                  sigma_list=(65536,), split_list=(128, 256), time_top=1,
                  cache_path=cache, device=DEV, csr_chunks=()) == r


def test_tune_picks_csr_packing_for_power_law_rows():
    """On power-law rows the CSR-packed layout is timed beside split SELL;
    whichever wins, the chosen configuration rebuilds to the same bytes and
    multiplies correctly."""
    from helpers import FMTS, SPMV_TOL, normalised_error, oracle_product

    a = W.powerlaw(200_000, seed=9)
    r = T.tune(a.rowptr, a.col, a.val, a.n, a.m, "fp16", 10, C_list=(64,), sigma_list=(65536,),
               split_list=(128,), time_top=1, device=DEV, csr_chunks=(256, 512))
    c = r["csr_candidates"][0]
    assert set(c["chunk_us"]) == {"256", "512"} and c["C"] == 1 and c["sigma"] == 1
    timed = [c for c in r["candidates"] + r["csr_candidates"] if "us" in c]
    assert r["us"] == min(t["us"] for t in timed)
    A = B.encode(a.rowptr, a.col, a.val, a.n, a.m, "fp16", r["D"], r["C"], r["sigma"],
                 B.EXPLICIT, DEV, split_words=r["split_words"])
    assert A.bytes_per_spmv() == r["bytes"]
    x = W.uniform_vector(a.m, 4)
    y = B.spmv(A, torch.from_numpy(x).to(DEV)).cpu().numpy()
    ref, q = oracle_product(a, FMTS["fp16"], 15, x)
    assert normalised_error(y, ref, a, q, x) <= SPMV_TOL
