"""The bandwidth probe behind the measured copy ceiling: an exact copy for
any length (whole 16-byte chunks plus a tail of 0-3 floats)."""
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_1309_1983_amd
    paper_1309_1983_amd.lib()


@pytest.mark.parametrize("n", [1, 3, 4, 1027, 1024 * 256, 1024 * 256 + 2, (1 << 22) + 5])
def test_copy_probe_copies_exactly(n):
    from paper_1309_1983_amd import copy_f32
    g = torch.Generator(device="cuda").manual_seed(n)
    a = torch.rand(n + 16, device="cuda", generator=g)
    b = torch.full((n + 16,), -1.0, device="cuda")
    copy_f32(a[:n], b)
    torch.cuda.synchronize()
    assert torch.equal(b[:n], a[:n])
    assert torch.all(b[n:] == -1.0)     # nothing written past n
