"""The streaming copy kernel (lb_stream_copy), which bench.py uses as the
plain-copy HBM probe and as the calibration of the byte counters: every
byte arrives, the tail of a size that is not a whole number of blocks too,
and nothing past `bytes` is written."""

import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nbytes", [16, 16 * 1023, 16 * (4 * 256 + 5), 1 << 20, (3 << 20) + 48])
def test_copy_is_exact_and_stops_at_the_end(lbgpu, nbytes):
    g = torch.Generator(device="cpu").manual_seed(nbytes)
    n = nbytes // 8 + 64
    src = torch.randint(-2**62, 2**62, (n,), dtype=torch.int64, generator=g).to("cuda")
    dst = torch.full((n,), -1, dtype=torch.int64, device="cuda")
    lbgpu.lb_stream_copy(dst, src, nbytes)
    torch.cuda.synchronize()
    k = nbytes // 8
    assert torch.equal(dst[:k], src[:k])
    assert bool((dst[k:] == -1).all())


def test_copy_on_another_stream(lbgpu):
    src = torch.arange(1 << 18, dtype=torch.float64, device="cuda")
    dst = torch.zeros_like(src)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    lbgpu.lb_stream_copy(dst, src, stream=s.cuda_stream)
    s.synchronize()
    assert torch.equal(dst, src)
