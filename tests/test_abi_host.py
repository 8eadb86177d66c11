"""Host-side checks of the C ABI (no GPU needed, no kernel launched).

* the library loads and exports every function include/dwtfrag.h declares;
* geometry and default width agree with the oracle's bookkeeping;
* invalid arguments return the documented status codes before any launch.
"""
import ctypes
import os
import re

import pytest

from conftest import ROOT
from oracle import fragment

pkg = pytest.importorskip("paper_1803_04880_amd")

HEADER = os.path.join(ROOT, "include", "dwtfrag.h")


def _lib_or_skip():
    if not os.path.exists(pkg.LIB_PATH):
        pytest.skip("libdwtfrag.so not built")
    return pkg.lib()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dwtfrag_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    assert declared_functions() == sorted(pkg.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = _lib_or_skip()
    for name in declared_functions():
        assert hasattr(L, name), name
    nm = os.popen(f"nm -D --defined-only {pkg.LIB_PATH}").read()
    for name in declared_functions():
        assert re.search(rf"\bT {name}\b", nm), name


@pytest.mark.parametrize("n,width,levels", [
    (1, 1, 1), (7, 3, 2), (262144, 512, 1), (1 << 28, 32768, 3), (100003, 317, 3),
    (5000, 1, 4), (5000, 5000, 4), (12345, 64, 6), (1 << 20, 1024, 9), (3, 2, 32),
])
def test_geometry_matches_oracle(n, width, levels):
    _lib_or_skip()
    g = pkg.geometry(n, width, levels)
    o = fragment.geometry(n, width, levels)
    assert g["height"] == o["height"]
    assert (g["ll_h"], g["ll_w"]) == (o["ll_h"], o["ll_w"])
    assert g["priv_bytes"] == o["priv_bytes"] and g["pub_bytes"] == o["pub_bytes"]
    assert (g["workspace_bytes"] > 0) == (levels > 4)


def test_default_width_matches_oracle():
    _lib_or_skip()
    for n in list(range(1, 300)) + [4095, 4096, 4097, 1 << 24, (1 << 24) + 1, 1 << 26, 10 ** 9]:
        assert pkg.default_width(n) == fragment.default_width(n), n
    assert pkg.default_width(0) == 0


def test_geometry_errors():
    L = _lib_or_skip()
    g = pkg._Geom()
    assert L.dwtfrag_geometry(0, 4, 1, ctypes.byref(g)) == pkg.DWTFRAG_EINVAL
    assert L.dwtfrag_geometry(10, 0, 1, ctypes.byref(g)) == pkg.DWTFRAG_EINVAL
    assert L.dwtfrag_geometry(10, 4, 0, ctypes.byref(g)) == pkg.DWTFRAG_EINVAL
    assert L.dwtfrag_geometry(10, 4, 33, ctypes.byref(g)) == pkg.DWTFRAG_EINVAL
    assert L.dwtfrag_geometry(10, 4, 1, None) == pkg.DWTFRAG_EINVAL
    assert L.dwtfrag_geometry(10, 1 << 31, 1, ctypes.byref(g)) == pkg.DWTFRAG_ERANGE
    # the largest row / column count keeps 2^16 of int32 headroom for planning
    lim = (1 << 31) - (1 << 16)
    assert L.dwtfrag_geometry(10, lim, 1, ctypes.byref(g)) == pkg.DWTFRAG_OK
    assert L.dwtfrag_geometry(10, lim + 1, 1, ctypes.byref(g)) == pkg.DWTFRAG_ERANGE
    assert L.dwtfrag_geometry(lim, 1, 3, ctypes.byref(g)) == pkg.DWTFRAG_OK
    assert L.dwtfrag_geometry(lim + 1, 1, 3, ctypes.byref(g)) == pkg.DWTFRAG_ERANGE
    assert L.dwtfrag_geometry(1 << 40, 1, 1, ctypes.byref(g)) == pkg.DWTFRAG_ERANGE


def test_protect_restore_reject_bad_arguments_before_launch():
    L = _lib_or_skip()
    key = b"k" * 16
    fake = ctypes.c_void_p(0x10000)  # never dereferenced: validation fails first
    bad = [
        (None, 100, 10, 1, key, key, fake, fake, None, 0, None, None),   # null input
        (fake, 0, 10, 1, key, key, fake, fake, None, 0, None, None),     # n == 0
        (fake, 100, 0, 1, key, key, fake, fake, None, 0, None, None),    # width == 0
        (fake, 100, 10, 0, key, key, fake, fake, None, 0, None, None),   # levels == 0
        (fake, 100, 10, 33, key, key, fake, fake, None, 0, None, None),  # levels > 32
        (fake, 100, 10, 1, None, key, fake, fake, None, 0, None, None),  # null key
        (ctypes.c_void_p(0x10001), 100, 10, 1, key, key, fake, fake, None, 0, None, None),
    ]
    for args in bad:
        assert L.dwtfrag_protect(*args) == pkg.DWTFRAG_EINVAL
    # levels > 4 needs a workspace
    assert L.dwtfrag_protect(fake, 100000, 300, 6, key, key, fake, fake, None, 0, None,
                             None) == pkg.DWTFRAG_EWORKSPACE
    assert L.dwtfrag_restore(fake, fake, 100000, 300, 6, key, key, fake, None, 0, None,
                             None) == pkg.DWTFRAG_EWORKSPACE
    assert L.dwtfrag_restore(None, fake, 100, 10, 1, key, key, fake, None, 0, None,
                             None) == pkg.DWTFRAG_EINVAL
    assert L.dwtfrag_restore(fake, fake, 100, 10, 1, key, key, None, None, 0, None,
                             None) == pkg.DWTFRAG_EINVAL
    bad_launch = pkg.Launch(0, 12)
    assert L.dwtfrag_protect(fake, 100, 10, 1, key, key, fake, fake, None, 0,
                             ctypes.byref(bad_launch), None) == pkg.DWTFRAG_EINVAL
    assert L.dwtfrag_aes128_ctr(fake, fake, 0, key, key, 0, None) == pkg.DWTFRAG_EINVAL
    for code in (0, -1, -2, -3, -4, 7):
        assert pkg.strerror(code)


def test_alignment_contract_of_single_buffer_calls():
    """The header requires 16-byte aligned device buffers for protect and
    restore: each misaligned pointer is refused with EINVAL before any
    launch (the pointers are never dereferenced)."""
    L = _lib_or_skip()
    key = b"k" * 16
    A = 0x100000                                # 16-byte aligned fake addresses
    ok = dict(src=A, priv=A + 0x10000, pub=A + 0x20000, dst=A + 0x30000, ws=A + 0x40000)
    for name in ok:
        for off in (1, 2, 4, 8):
            p = dict(ok)
            p[name] += off
            v = {k: ctypes.c_void_p(x) for k, x in p.items()}
            # 6 levels: the workspace is used and checked too
            rc = L.dwtfrag_protect(v["src"], 100000, 300, 6, key, key, v["priv"], v["pub"],
                                   v["ws"], 1 << 20, None, None)
            if name != "dst":
                assert rc == pkg.DWTFRAG_EINVAL, (name, off)
            rc = L.dwtfrag_restore(v["priv"], v["pub"], 100000, 300, 6, key, key, v["dst"],
                                   v["ws"], 1 << 20, None, None)
            if name != "src":
                assert rc == pkg.DWTFRAG_EINVAL, (name, off)


def test_product_path_has_no_oracle_dependency():
    """The package never imports the oracle (or any CPU fallback)."""
    pdir = os.path.join(ROOT, "paper_1803_04880_amd")
    for dirpath, _, files in os.walk(pdir):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in re.sub(r"#.*|//.*", "", text), f


def _item(n, width, levels, base=1 << 20):
    from paper_1803_04880_amd.batch import Item
    it = Item()
    it.in_, it.out, it.priv, it.pub = base, base + (1 << 30), base + (2 << 30), base + (3 << 30)
    it.n, it.width, it.levels = n, width, levels
    return it


def test_batch_planner_host_logic():
    """Planning is host work: valid items give a plan and its device size;
    bad items are rejected before anything touches a device."""
    L = _lib_or_skip()
    from paper_1803_04880_amd.batch import Item
    items = (Item * 3)(_item(1000, 32, 1), _item(70000, 256, 4), _item(5, 2, 2))
    h = ctypes.c_void_p()
    assert L.dwtfrag_batch_create(ctypes.addressof(items), 3, None, 0, ctypes.byref(h)) == 0
    assert L.dwtfrag_batch_device_bytes(h) >= 256
    assert L.dwtfrag_batch_protect(h, None) == pkg.DWTFRAG_EINVAL   # not uploaded
    L.dwtfrag_batch_destroy(h)
    for bad in (_item(100, 10, 5), _item(100, 10, 0), _item(100, 0, 1), _item(100, 10, 1, base=8)):
        one = (Item * 1)(bad)
        h = ctypes.c_void_p()
        rc = L.dwtfrag_batch_create(ctypes.addressof(one), 1, None, 0, ctypes.byref(h))
        assert rc == pkg.DWTFRAG_EINVAL and not h.value
    assert L.dwtfrag_batch_create(None, 1, None, 0, ctypes.byref(h)) == pkg.DWTFRAG_EINVAL


def test_learned_geometry_pairs_and_limits():
    from oracle import learned
    import numpy as np
    from paper_1803_04880_amd import learned as GL
    _lib_or_skip()
    for n, w, lv in ((1, 1, 1), (1000, 1, 3), (12345, 97, 2), (4096 * 4096, 4096, 3)):
        _, pairs = GL.learned_geometry(n, w, lv)
        h = -(-n // w)
        if n <= 20000:
            ctx, t = learned.training_pairs(np.zeros((h, w), np.int64), lv)
            assert pairs == t.size
        assert pairs > 0 or (h == 1 and w == 1)
    with pytest.raises(pkg.DwtfragError):
        GL.learned_geometry(100, 10, 4)


def test_noalloc_rejects_workspace_above_static_buffer():
    L = _lib_or_skip()
    n, width, levels = 1 << 33, 1 << 16, 6
    assert pkg.geometry(n, width, levels)["workspace_bytes"] > 16 << 20
    # rejected on the host before any device call: the pointers are never used
    fake = 1 << 12
    assert L.dwtfrag_protect_noalloc(fake, n, width, levels, bytes(16), bytes(16), fake, fake,
                                     None, None) == pkg.DWTFRAG_ESCRATCH
    assert L.dwtfrag_protect_noalloc(None, n, width, levels, bytes(16), bytes(16), fake, fake,
                                     None, None) == pkg.DWTFRAG_EINVAL
    assert "16 MiB" in pkg.strerror(pkg.DWTFRAG_ESCRATCH)


@pytest.mark.parametrize("n,width", [(1, 8), (64, 8), (65, 8), (1000, 16), (12345, 96),
                                     (1 << 28, 32768), (3 * 257 * 64 + 1, 24)])
def test_se8_geometry_matches_oracle(n, width):
    _lib_or_skip()
    from oracle import se8
    g = pkg.se8_geometry(n, width)
    o = se8.geometry(n, width)
    for k in ("height", "block_rows", "block_cols", "blocks", "priv_bytes", "pub1_bytes",
              "pub2_bytes"):
        assert g[k] == o[k], k


def test_se8_errors_before_launch():
    L = _lib_or_skip()
    g = pkg._Se8Geom()
    assert L.dwtfrag_se8_geometry(0, 8, ctypes.byref(g)) == pkg.DWTFRAG_EINVAL
    assert L.dwtfrag_se8_geometry(64, 12, ctypes.byref(g)) == pkg.DWTFRAG_EINVAL
    assert L.dwtfrag_se8_geometry(64, 0, ctypes.byref(g)) == pkg.DWTFRAG_EINVAL
    assert L.dwtfrag_se8_geometry(64, 8, None) == pkg.DWTFRAG_EINVAL
    fake = 1 << 12
    # misaligned or null pointers are rejected on the host
    assert L.dwtfrag_se8_protect(fake + 8, 64, 8, bytes(16), bytes(16), fake, fake, fake,
                                 None) == pkg.DWTFRAG_EINVAL
    assert L.dwtfrag_se8_protect(fake, 64, 8, bytes(16), bytes(16), None, fake, fake,
                                 None) == pkg.DWTFRAG_EINVAL
    assert L.dwtfrag_se8_restore(fake, fake, fake + 4, 64, 8, bytes(16), bytes(16), fake,
                                 None) == pkg.DWTFRAG_EINVAL
