"""The entry point that allocates nothing (dwtfrag_protect_noalloc) against
dwtfrag_protect, byte for byte, through the C ABI on cuda:0.

Two calls in a row share the library's static workspace, the second on a
smaller input, at depths above four levels (where the workspace is used);
a depth of at most four levels never touches it.  Both are also checked
against the oracle.
"""
import numpy as np
import pytest

from conftest import gpu_available

pytestmark = pytest.mark.gpu

if not gpu_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import torch  # noqa: E402

import paper_1803_04880_amd as dwtfrag  # noqa: E402
from oracle import fragment  # noqa: E402

DEV = "cuda:0"


def _run_both(n, width, levels, seed):
    print(f"noalloc case n={n} width={width} levels={levels} seed={seed}", flush=True)
    rng = np.random.default_rng(seed)
    buf = rng.integers(0, 256, n, dtype=np.uint8)
    key, nonce = rng.bytes(16), rng.bytes(16)
    x = torch.from_numpy(buf).to(DEV)
    g = dwtfrag.geometry(n, width, levels)
    priv_a, pub_a = dwtfrag.protect(x, width, levels, key, nonce)
    priv_b = torch.full((g["priv_bytes"],), 0xA5, dtype=torch.uint8, device=DEV)
    pub_b = torch.full((g["pub_bytes"] // 2,), -7, dtype=torch.int16, device=DEV)
    dwtfrag.protect_noalloc(x, width, levels, key, nonce, priv=priv_b, pub=pub_b)
    torch.cuda.synchronize()
    assert torch.equal(priv_a, priv_b), "private fragment differs from dwtfrag_protect"
    assert torch.equal(pub_a, pub_b), "public fragment differs from dwtfrag_protect"
    opriv, opub = fragment.protect(buf, width, levels, key, nonce)
    assert priv_b.cpu().numpy().tobytes() == opriv
    assert pub_b.cpu().numpy().tobytes() == opub
    return g["workspace_bytes"]


def test_noalloc_equals_protect_on_two_calls_second_smaller():
    ws1 = _run_both(700_001, 1031, 6, 71)
    ws2 = _run_both(100_003, 317, 5, 72)
    assert ws1 > ws2 > 0  # both used the static workspace, the second less of it


def test_noalloc_without_workspace_and_after_deep_call():
    _run_both(300_000, 1031, 8, 73)
    _run_both(262_144, 512, 3, 74)   # levels <= 4: no workspace
    _run_both(5000, 71, 5, 75)


def test_noalloc_geometry_errors_before_launch():
    L = dwtfrag.lib()
    x = torch.zeros(16, dtype=torch.uint8, device=DEV)
    # workspace of a 2^33-byte buffer at 6 levels is above the static 16 MiB
    n = 1 << 33
    assert dwtfrag.geometry(n, 1 << 16, 6)["workspace_bytes"] > 16 << 20
    rc = L.dwtfrag_protect_noalloc(x.data_ptr(), n, 1 << 16, 6, bytes(16), bytes(16),
                                   x.data_ptr(), x.data_ptr(), None, None)
    assert rc == dwtfrag.DWTFRAG_ESCRATCH
