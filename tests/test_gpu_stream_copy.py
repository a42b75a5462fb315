"""The library's plain streaming copy (the bandwidth reference of the
benchmarks): exact bytes, a ragged tail, untouched guard bytes beyond the
destination, and refusal of misaligned sizes."""
import pytest

pytestmark = pytest.mark.gpu


def test_stream_copy_exact_with_ragged_tail():
    import torch
    from paper_2510_13726_amd import hlbm
    n = (16 << 20) + 48            # not a multiple of one workgroup's 16 KiB
    g = torch.Generator(device="cpu").manual_seed(11)
    src = torch.randint(0, 256, (n,), dtype=torch.uint8, generator=g).cuda()
    buf = torch.full((n + 4096,), 7, dtype=torch.uint8, device="cuda")
    hlbm.stream_copy(src, buf[:n])
    torch.cuda.synchronize()
    assert torch.equal(buf[:n], src)
    assert bool((buf[n:] == 7).all())


def test_stream_copy_refuses_misaligned_sizes():
    import torch
    from paper_2510_13726_amd import hlbm
    a = torch.zeros(40, dtype=torch.uint8, device="cuda")
    b = torch.zeros(40, dtype=torch.uint8, device="cuda")
    with pytest.raises(hlbm.HlbmError):
        hlbm.stream_copy(a, b)
