"""The ceiling diagnostics behind the benchmark's rooflines do the memory
work they are priced at: the streaming copy copies every byte, the
streaming read and the random-access kernels leave the buffer unchanged."""
import pytest

pytestmark = pytest.mark.gpu


def test_stream_copy_copies_and_read_leaves_buffer():
    import torch
    import paper_2108_07232_amd as bht
    n = (1 << 20) + 12345                       # 16-byte words, a ragged last chunk
    src = torch.randint(-2**62, 2**62, (2 * n,), dtype=torch.int64, device="cuda")
    dst = torch.zeros_like(src)
    sink = torch.zeros(1, dtype=torch.int64, device="cuda")
    before = src.clone()
    bht.bht_diag_stream(src.data_ptr(), dst.data_ptr(), 16 * n, sink)
    torch.cuda.synchronize()
    assert torch.equal(dst, src)
    bht.bht_diag_stream(src.data_ptr(), None, 16 * n, sink)
    bht.bht_diag_gather(src.data_ptr(), 16 * n, 1 << 16, 128, 3, sink)
    bht.bht_diag_cas(src.data_ptr(), 16 * n, 1 << 16, 3, sink)
    torch.cuda.synchronize()
    assert torch.equal(src, before)
    # a byte count that is not a multiple of 16 copies the whole words only
    dst.zero_()
    bht.bht_diag_stream(src.data_ptr(), dst.data_ptr(), 16 * 1000 + 7, sink)
    torch.cuda.synchronize()
    assert torch.equal(dst[:2000], src[:2000]) and int(dst[2000:].abs().sum()) == 0
