"""The streaming-ceiling kernels (gf_stream): every copy variant copies
exactly, an in-place pass (dst = src) leaves the data as it was, the read
pass sums what it reads, and bad arguments are refused.
Sizes include a ragged tail (not a multiple of one block's 16 KiB)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kind", ["copy", "copy_nt_load", "copy_nt_store", "copy_nt"])
def test_copy_is_exact(kind):
    import torch
    from paper_1212_5221_amd import gf
    n = (1 << 20) + 12  # floats: 4 MiB + 48 B
    x = torch.randn(n, dtype=torch.float32, device="cuda:0")
    y = torch.full_like(x, float("nan"))
    gf.stream(kind, y, x, n * 4)
    torch.cuda.synchronize()
    assert torch.equal(x, y)


@pytest.mark.parametrize("kind", ["copy", "copy_nt"])
def test_in_place_pass_keeps_the_data(kind):
    import torch
    from paper_1212_5221_amd import gf
    n = (1 << 20) + 12
    x = torch.randn(n, dtype=torch.float32, device="cuda:0")
    ref = x.clone()
    for _ in range(3):
        gf.stream(kind, x, x, n * 4)
    torch.cuda.synchronize()
    assert torch.equal(x, ref)


def test_read_sums_blocks():
    import torch
    from paper_1212_5221_amd import gf
    n = (1 << 18) + 20  # floats
    x = torch.ones(n, dtype=torch.float32, device="cuda:0")
    nb = gf.stream_blocks(n * 4)
    assert nb == (n * 4 + 16383) // 16384
    sink = torch.zeros(nb, dtype=torch.float32, device="cuda:0")
    gf.stream("read", sink, x, n * 4)
    torch.cuda.synchronize()
    s = sink.cpu().numpy()
    assert float(s.sum()) == float(n)
    np.testing.assert_array_equal(s[:-1], 4096.0)  # 16 KiB of ones per block


def test_bad_arguments():
    import ctypes
    from paper_1212_5221_amd import gf
    L = gf.load()
    assert L.gf_stream(None, 0, ctypes.c_void_p(256), ctypes.c_void_p(512), 10) == gf.E_INVALID  # not 16-byte units
    assert L.gf_stream(None, 9, ctypes.c_void_p(256), ctypes.c_void_p(512), 16) == gf.E_INVALID  # unknown kind
    assert L.gf_stream(None, 0, None, ctypes.c_void_p(512), 16) == gf.E_INVALID
    with pytest.raises(gf.GFError):
        gf.stream_blocks(10)
