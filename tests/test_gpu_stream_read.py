"""The read-only streaming probe (wh_stream_read): it reads every byte of the
buffer once, so its XOR of the buffer's 32-bit words must equal numpy's, for
sizes with and without a ragged tail of the grid-stride loop."""
import numpy as np
import pytest
import torch

from paper_1902_08018_amd import wh

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nbytes", [16, 4096, 16 * 1000003, 1 << 26])
def test_stream_read_xor(gpu_ctx, nbytes):
    rng = np.random.default_rng(nbytes % 1000)
    host = rng.integers(0, 2 ** 32, size=nbytes // 4, dtype=np.uint32)
    buf = torch.from_numpy(host.view(np.int32)).cuda()
    out = torch.zeros(1, dtype=torch.int32, device="cuda")
    wh.wh_stream_read(gpu_ctx, buf, out)
    torch.cuda.synchronize()
    want = np.bitwise_xor.reduce(host)
    assert int(out.cpu().numpy().view(np.uint32)[0]) == int(want)


def test_stream_read_rejects_ragged(gpu_ctx):
    buf = torch.zeros(5, dtype=torch.int32, device="cuda")       # 20 bytes: not a multiple of 16
    out = torch.zeros(1, dtype=torch.int32, device="cuda")
    with pytest.raises(wh.WhError) as ei:
        wh.wh_stream_read(gpu_ctx, buf, out)
    assert ei.value.status == wh.WH_ERR_INVALID
