"""The reference streams (measurement context for the lifting kernels, not
part of the method): widen is the byte -> int16 zero extension and narrow
the int16 -> low byte truncation, elementwise; sizes span a ragged last
work-group, and the argument checks reject what the header excludes."""
import pytest

from conftest import gpu_available

pytestmark = pytest.mark.gpu

if not gpu_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import torch  # noqa: E402

import paper_1803_04880_amd as dwtfrag  # noqa: E402


@pytest.mark.parametrize("n", [16, 4096, 16 * 257 * 3, (1 << 20) + 16 * 5])
def test_widen_and_narrow_are_the_elementwise_conversions(n):
    g = torch.Generator().manual_seed(n)
    x = torch.randint(0, 256, (n,), dtype=torch.uint8, generator=g)
    v = torch.randint(-32768, 32768, (n,), dtype=torch.int16, generator=g)
    wide = torch.full((n,), -1, dtype=torch.int16, device="cuda")
    dwtfrag.ref_widen(x.cuda(), wide)
    assert torch.equal(wide.cpu(), x.to(torch.int16))
    back = torch.zeros(n, dtype=torch.uint8, device="cuda")
    dwtfrag.ref_narrow(wide, back)
    assert torch.equal(back.cpu(), x)
    low = torch.zeros(n, dtype=torch.uint8, device="cuda")
    dwtfrag.ref_narrow(v.cuda(), low)
    assert torch.equal(low.cpu(), (v.to(torch.int32) & 255).to(torch.uint8))


def test_reference_streams_reject_what_the_header_excludes():
    x = torch.zeros(64, dtype=torch.uint8, device="cuda")
    w = torch.zeros(64, dtype=torch.int16, device="cuda")
    lib = dwtfrag.lib()
    assert lib.dwtfrag_ref_widen(x.data_ptr(), w.data_ptr(), 40, None) == dwtfrag.DWTFRAG_EINVAL
    assert lib.dwtfrag_ref_widen(x.data_ptr() + 1, w.data_ptr(), 32, None) == dwtfrag.DWTFRAG_EINVAL
    assert lib.dwtfrag_ref_narrow(w.data_ptr(), x.data_ptr(), 0, None) == dwtfrag.DWTFRAG_EINVAL
    assert lib.dwtfrag_ref_narrow(None, x.data_ptr(), 32, None) == dwtfrag.DWTFRAG_EINVAL
    with pytest.raises(ValueError):
        dwtfrag.ref_widen(x, w[:32])
