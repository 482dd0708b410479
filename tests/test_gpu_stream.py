"""The streaming probe (practical-bandwidth yardstick of the roofline figures): copy, read and
zero fill over buffers whose size is not a multiple of the workgroup's span, and beyond one
grid-stride pass."""
import pytest
import torch

pytestmark = pytest.mark.gpu

from paper_2209_01877_amd import stream_probe  # noqa: E402


@pytest.mark.parametrize("n16", [1, 37, 512 * 3 + 5, 65536 * 512 + 77])
def test_stream_probe_copy_and_fill(n16):
    g = torch.Generator(device="cuda").manual_seed(n16)
    src = torch.randint(-2**31, 2**31 - 1, (4 * n16,), dtype=torch.int32, device="cuda", generator=g)
    dst = torch.full_like(src, 7)
    guard = torch.full((8,), 5, dtype=torch.int32, device="cuda")
    stream_probe("copy", src, dst)
    torch.cuda.synchronize()
    assert torch.equal(dst, src)
    stream_probe("write", None, dst)
    torch.cuda.synchronize()
    assert torch.count_nonzero(dst).item() == 0
    stream_probe("read", src, guard)  # reads only; the guard is at most overwritten in its first 16 bytes
    stream_probe("read_cached", src, guard)
    torch.cuda.synchronize()
    assert torch.equal(guard[4:], torch.full((4,), 5, dtype=torch.int32, device="cuda"))


def test_stream_probe_partial_copy():
    """Copy of a prefix: dst's bytes decide the length, the source's tail is not read into dst."""
    src = torch.arange(4096, dtype=torch.int32, device="cuda")
    dst = torch.zeros(1024, dtype=torch.int32, device="cuda")
    stream_probe("copy", src, dst)
    torch.cuda.synchronize()
    assert torch.equal(dst, src[:1024])
