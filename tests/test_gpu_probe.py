"""The random-read probe behind the H.v roofline: it runs, reports a plausible
rate, and leaves its buffer untouched."""
import pytest
import torch

pytestmark = pytest.mark.gpu


def test_random_read_probe_rate_and_no_writes():
    from paper_1804_05028_amd import _lib as L
    nbytes = 1 << 30
    buf = torch.arange(nbytes // 8, dtype=torch.int64, device="cuda").view(torch.uint8)
    before = int(buf.view(torch.int64).sum())
    for slot_bytes in (16, 32):
        rate = L.ed_probe_random_reads(buf, nbytes, 64, 2, torch.cuda.current_stream().cuda_stream,
                                       slot_bytes=slot_bytes)
        torch.cuda.synchronize()
        assert int(buf.view(torch.int64).sum()) == before
        # one slot per lane-iteration, one 128 B line each; HBM3E at 8 TB/s serves at most 6.25e10
        # lines per second
        assert 1e9 < rate < 2e11, (slot_bytes, rate)
