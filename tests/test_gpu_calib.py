"""The streaming-read measurement helper runs on any multiple of 16 bytes
and rejects other sizes."""
import ctypes

import pytest
import torch

from paper_2604_13433_amd import binding as B

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


@pytest.mark.parametrize("nbytes", [16, 4096, 1 << 20, (75_497_480 // 16) * 16])
@pytest.mark.parametrize("width,chunks", [(4, 7), (16, 8), (4, 1), (16, 4096)])
def test_stream_read_runs(nbytes, width, chunks):
    buf = torch.ones(nbytes // 4, dtype=torch.float32, device=DEV)
    rd = B.StreamRead(buf, width, chunks)
    rd()
    torch.cuda.synchronize()


@pytest.mark.parametrize("nbytes,width,chunks", [(20, 4, 7), (0, 4, 7), (64, 8, 7), (64, 4, 0),
                                                 (64, 4, 5000)])
def test_stream_read_rejects_bad_arguments(nbytes, width, chunks):
    buf = torch.ones(16, dtype=torch.float32, device=DEV)
    out = torch.empty(1, device=DEV)
    rc = B.lib().pksell_stream_read(ctypes.c_void_p(buf.data_ptr()), nbytes, width, chunks,
                                    ctypes.c_void_p(out.data_ptr()), None)
    assert rc == B.EINVAL
