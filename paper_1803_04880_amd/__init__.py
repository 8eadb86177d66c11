"""dwtfrag: DWT-fragmentation protect / restore on one MI355X.

Thin ctypes binding over ``libdwtfrag.so`` (the HIP kernels and C ABI declared
in ``include/dwtfrag.h``).  This module only marshals arguments: every step of
protect / restore runs in the library's kernels.  PyTorch provides device
memory and the current stream.  If the library is missing the calls raise; no
other code path exists.

    priv, pub = protect(x_u8_cuda, width, levels, key, nonce)
    x2 = restore(priv, pub, n, width, levels, key, nonce)
"""
from __future__ import annotations

import ctypes
import os

import torch  # must load before the library so that both share one HIP runtime

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdwtfrag.so")

DWTFRAG_OK = 0
DWTFRAG_EINVAL = -1
DWTFRAG_ERANGE = -2
DWTFRAG_EDEVICE = -3
DWTFRAG_EWORKSPACE = -4
DWTFRAG_ESCRATCH = -5


class DwtfragError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {strerror(code)} ({code})")
        self.code = code


class _Geom(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint64), ("width", ctypes.c_uint32), ("height", ctypes.c_uint32),
                ("levels", ctypes.c_uint32), ("ll_h", ctypes.c_uint32), ("ll_w", ctypes.c_uint32),
                ("priv_bytes", ctypes.c_uint64), ("pub_bytes", ctypes.c_uint64),
                ("workspace_bytes", ctypes.c_uint64)]


class _Se8Geom(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint64), ("width", ctypes.c_uint32), ("height", ctypes.c_uint64),
                ("block_rows", ctypes.c_uint64), ("block_cols", ctypes.c_uint64),
                ("blocks", ctypes.c_uint64), ("priv_bytes", ctypes.c_uint64),
                ("pub1_bytes", ctypes.c_uint64), ("pub2_bytes", ctypes.c_uint64)]


class Launch(ctypes.Structure):
    """Optional launch shape; zero fields mean the library default."""
    _fields_ = [("seg_rows", ctypes.c_uint32), ("lane_cols", ctypes.c_uint32)]


_lib = None

EXPORTS = ("dwtfrag_geometry", "dwtfrag_default_width", "dwtfrag_protect",
           "dwtfrag_protect_noalloc", "dwtfrag_restore",
           "dwtfrag_aes128_ctr", "dwtfrag_strerror",
           "dwtfrag_learned_geometry", "dwtfrag_protect_learned", "dwtfrag_restore_learned",
           "dwtfrag_learned_pairs", "dwtfrag_trainer_workspace_bytes", "dwtfrag_trainer_init",
           "dwtfrag_trainer_step",
           "dwtfrag_batch_create", "dwtfrag_batch_device_bytes", "dwtfrag_batch_upload",
           "dwtfrag_batch_protect", "dwtfrag_batch_restore", "dwtfrag_batch_destroy",
           "dwtfrag_autotune",
           "dwtfrag_se8_geometry", "dwtfrag_se8_protect", "dwtfrag_se8_restore",
           "dwtfrag_ref_widen", "dwtfrag_ref_narrow")


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_1803_04880_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    u8p, i16p, vp = ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p
    L.dwtfrag_geometry.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                   ctypes.POINTER(_Geom)]
    L.dwtfrag_geometry.restype = ctypes.c_int
    L.dwtfrag_default_width.argtypes = [ctypes.c_uint64]
    L.dwtfrag_default_width.restype = ctypes.c_uint32
    L.dwtfrag_protect.argtypes = [u8p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                  ctypes.c_char_p, ctypes.c_char_p, u8p, i16p, vp,
                                  ctypes.c_uint64, ctypes.POINTER(Launch), vp]
    L.dwtfrag_protect.restype = ctypes.c_int
    L.dwtfrag_protect_noalloc.argtypes = [u8p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                          ctypes.c_char_p, ctypes.c_char_p, u8p, i16p,
                                          ctypes.POINTER(Launch), vp]
    L.dwtfrag_protect_noalloc.restype = ctypes.c_int
    L.dwtfrag_restore.argtypes = [u8p, i16p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                  ctypes.c_char_p, ctypes.c_char_p, u8p, vp, ctypes.c_uint64,
                                  ctypes.POINTER(Launch), vp]
    L.dwtfrag_restore.restype = ctypes.c_int
    L.dwtfrag_aes128_ctr.argtypes = [u8p, u8p, ctypes.c_uint64, ctypes.c_char_p, ctypes.c_char_p,
                                     ctypes.c_uint64, vp]
    L.dwtfrag_aes128_ctr.restype = ctypes.c_int
    L.dwtfrag_strerror.argtypes = [ctypes.c_int]
    L.dwtfrag_strerror.restype = ctypes.c_char_p
    u64, u32, cp = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_char_p
    L.dwtfrag_learned_geometry.argtypes = [u64, u32, u32, ctypes.POINTER(u64), ctypes.POINTER(u64)]
    L.dwtfrag_protect_learned.argtypes = [vp, u64, u32, u32, cp, cp, vp, vp, vp, vp, u64, vp]
    L.dwtfrag_restore_learned.argtypes = [vp, vp, u64, u32, u32, cp, cp, vp, vp, vp, u64, vp]
    L.dwtfrag_learned_pairs.argtypes = [vp, u64, u32, u32, vp, vp, vp, u64, vp]
    L.dwtfrag_trainer_workspace_bytes.argtypes = []
    L.dwtfrag_trainer_workspace_bytes.restype = u64
    L.dwtfrag_trainer_init.argtypes = [vp, vp, vp]
    L.dwtfrag_trainer_step.argtypes = [vp, vp, vp, u64, u64, ctypes.c_float, vp, u64, vp]
    for f in ("dwtfrag_learned_geometry", "dwtfrag_protect_learned", "dwtfrag_restore_learned",
              "dwtfrag_learned_pairs", "dwtfrag_trainer_init", "dwtfrag_trainer_step"):
        getattr(L, f).restype = ctypes.c_int
    L.dwtfrag_batch_create.argtypes = [vp, u32, vp, u32, ctypes.POINTER(vp)]
    L.dwtfrag_batch_device_bytes.argtypes = [vp]
    L.dwtfrag_batch_device_bytes.restype = u64
    L.dwtfrag_batch_upload.argtypes = [vp, vp, u64, vp]
    L.dwtfrag_batch_protect.argtypes = [vp, vp]
    L.dwtfrag_batch_restore.argtypes = [vp, vp]
    L.dwtfrag_batch_destroy.argtypes = [vp]
    L.dwtfrag_batch_destroy.restype = None
    L.dwtfrag_autotune.argtypes = [vp, u64, u32, u32, vp, u64, u32, ctypes.POINTER(Launch),
                                   ctypes.POINTER(ctypes.c_float), vp]
    for f in ("dwtfrag_batch_create", "dwtfrag_batch_upload", "dwtfrag_batch_protect",
              "dwtfrag_batch_restore", "dwtfrag_autotune"):
        getattr(L, f).restype = ctypes.c_int
    L.dwtfrag_se8_geometry.argtypes = [u64, u32, ctypes.POINTER(_Se8Geom)]
    L.dwtfrag_se8_protect.argtypes = [vp, u64, u32, cp, cp, vp, vp, vp, vp]
    L.dwtfrag_se8_restore.argtypes = [vp, vp, vp, u64, u32, cp, cp, vp, vp]
    for f in ("dwtfrag_se8_geometry", "dwtfrag_se8_protect", "dwtfrag_se8_restore"):
        getattr(L, f).restype = ctypes.c_int
    for f in ("dwtfrag_ref_widen", "dwtfrag_ref_narrow"):
        getattr(L, f).argtypes = [vp, vp, u64, vp]
        getattr(L, f).restype = ctypes.c_int
    _lib = L
    return L


def strerror(code: int) -> str:
    return lib().dwtfrag_strerror(code).decode()


def geometry(n: int, width: int, levels: int) -> dict:
    g = _Geom()
    rc = lib().dwtfrag_geometry(n, width, levels, ctypes.byref(g))
    if rc != DWTFRAG_OK:
        raise DwtfragError(rc, "dwtfrag_geometry")
    return {f: getattr(g, f) for f, _ in _Geom._fields_}


def default_width(n: int) -> int:
    return int(lib().dwtfrag_default_width(n))


def _key16(b: bytes, what: str) -> bytes:
    b = bytes(b)
    if len(b) != 16:
        raise ValueError(f"{what} must be 16 bytes")
    return b


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _launch(launch):
    if launch is None:
        return None
    if isinstance(launch, Launch):
        return ctypes.byref(launch)
    return ctypes.byref(Launch(*launch))


def _check_dev(t: torch.Tensor, dtype, name: str):
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous {dtype} CUDA tensor")


def workspace(n: int, width: int, levels: int, device=None):
    """Scratch tensor the library needs for levels > 4 (None when not needed)."""
    ws = geometry(n, width, levels)["workspace_bytes"]
    if not ws:
        return None
    return torch.empty(ws, dtype=torch.uint8, device=device or "cuda")


def protect(x: torch.Tensor, width: int, levels: int, key: bytes, nonce: bytes, *,
            priv: torch.Tensor | None = None, pub: torch.Tensor | None = None,
            ws: torch.Tensor | None = None, launch=None, stream=None):
    """(priv u8, pub int16) fragments of the bytes in ``x`` (uint8 CUDA tensor)."""
    _check_dev(x, torch.uint8, "x")
    n = x.numel()
    g = geometry(n, width, levels)
    if priv is None:
        priv = torch.empty(g["priv_bytes"], dtype=torch.uint8, device=x.device)
    if pub is None:
        pub = torch.empty(g["pub_bytes"] // 2, dtype=torch.int16, device=x.device)
    _check_dev(priv, torch.uint8, "priv")
    _check_dev(pub, torch.int16, "pub")
    # the C ABI takes no buffer sizes: a short tensor would be written past
    # its end on the device, so sizes are checked here
    if priv.numel() != g["priv_bytes"] or 2 * pub.numel() != g["pub_bytes"]:
        raise ValueError("fragment sizes do not match the geometry")
    if ws is None and g["workspace_bytes"]:
        ws = workspace(n, width, levels, x.device)
    if ws is not None and ws.numel() < g["workspace_bytes"]:
        raise ValueError("workspace smaller than the geometry needs")
    rc = lib().dwtfrag_protect(
        x.data_ptr(), n, width, levels, _key16(key, "key"), _key16(nonce, "nonce"),
        priv.data_ptr(), pub.data_ptr(), ws.data_ptr() if ws is not None else None,
        ws.numel() if ws is not None else 0, _launch(launch), _stream(stream))
    if rc != DWTFRAG_OK:
        raise DwtfragError(rc, "dwtfrag_protect")
    return priv, pub


def protect_noalloc(x: torch.Tensor, width: int, levels: int, key: bytes, nonce: bytes, *,
                    priv: torch.Tensor, pub: torch.Tensor, launch=None, stream=None):
    """``protect`` into caller-given fragment tensors through the entry point
    that allocates nothing (its workspace is the library's static array)."""
    _check_dev(x, torch.uint8, "x")
    _check_dev(priv, torch.uint8, "priv")
    _check_dev(pub, torch.int16, "pub")
    n = x.numel()
    g = geometry(n, width, levels)
    if priv.numel() != g["priv_bytes"] or 2 * pub.numel() != g["pub_bytes"]:
        raise ValueError("fragment sizes do not match the geometry")
    rc = lib().dwtfrag_protect_noalloc(
        x.data_ptr(), n, width, levels, _key16(key, "key"), _key16(nonce, "nonce"),
        priv.data_ptr(), pub.data_ptr(), _launch(launch), _stream(stream))
    if rc != DWTFRAG_OK:
        raise DwtfragError(rc, "dwtfrag_protect_noalloc")
    return priv, pub


def restore(priv: torch.Tensor, pub: torch.Tensor, n: int, width: int, levels: int,
            key: bytes, nonce: bytes, *, out: torch.Tensor | None = None,
            ws: torch.Tensor | None = None, launch=None, stream=None) -> torch.Tensor:
    """The original n bytes (uint8 CUDA tensor) from the two fragments."""
    _check_dev(priv, torch.uint8, "priv")
    _check_dev(pub, torch.int16, "pub")
    g = geometry(n, width, levels)
    if priv.numel() != g["priv_bytes"] or 2 * pub.numel() != g["pub_bytes"]:
        raise ValueError("fragment sizes do not match the geometry")
    if out is None:
        out = torch.empty(n, dtype=torch.uint8, device=priv.device)
    _check_dev(out, torch.uint8, "out")
    if out.numel() < n:
        raise ValueError("out holds fewer than n bytes")
    if ws is None and g["workspace_bytes"]:
        ws = workspace(n, width, levels, priv.device)
    if ws is not None and ws.numel() < g["workspace_bytes"]:
        raise ValueError("workspace smaller than the geometry needs")
    rc = lib().dwtfrag_restore(
        priv.data_ptr(), pub.data_ptr(), n, width, levels, _key16(key, "key"),
        _key16(nonce, "nonce"), out.data_ptr(), ws.data_ptr() if ws is not None else None,
        ws.numel() if ws is not None else 0, _launch(launch), _stream(stream))
    if rc != DWTFRAG_OK:
        raise DwtfragError(rc, "dwtfrag_restore")
    return out


def aes128_ctr(x: torch.Tensor, key: bytes, nonce: bytes, first_block: int = 0, *,
               out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """AES-128-CTR of a uint8 CUDA tensor (encryption == decryption)."""
    _check_dev(x, torch.uint8, "x")
    if out is None:
        out = torch.empty_like(x)
    rc = lib().dwtfrag_aes128_ctr(x.data_ptr(), out.data_ptr(), x.numel(), _key16(key, "key"),
                                  _key16(nonce, "nonce"), first_block, _stream(stream))
    if rc != DWTFRAG_OK:
        raise DwtfragError(rc, "dwtfrag_aes128_ctr")
    return out


def ref_widen(x: torch.Tensor, out: torch.Tensor, stream=None) -> torch.Tensor:
    """Reference stream (measurement context, not the method): out = x as
    int16, one-shot, the forward's traffic (read n bytes, write 2n)."""
    _check_dev(x, torch.uint8, "x")
    _check_dev(out, torch.int16, "out")
    if out.numel() != x.numel():
        raise ValueError("out must hold x.numel() int16 values")
    rc = lib().dwtfrag_ref_widen(x.data_ptr(), out.data_ptr(), x.numel(), _stream(stream))
    if rc != DWTFRAG_OK:
        raise DwtfragError(rc, "dwtfrag_ref_widen")
    return out


def ref_narrow(x: torch.Tensor, out: torch.Tensor, stream=None) -> torch.Tensor:
    """Reference stream (measurement context, not the method): out = low
    bytes of the int16 x, one-shot, the inverse's traffic (read 2n, write n)."""
    _check_dev(x, torch.int16, "x")
    _check_dev(out, torch.uint8, "out")
    if out.numel() != x.numel():
        raise ValueError("out must hold x.numel() bytes")
    rc = lib().dwtfrag_ref_narrow(x.data_ptr(), out.data_ptr(), x.numel(), _stream(stream))
    if rc != DWTFRAG_OK:
        raise DwtfragError(rc, "dwtfrag_ref_narrow")
    return out


# ---------------------------------------------------------------------------
# The per-8x8-block protection (SHA-2 keystreams over the public fragments,
# 10/11-bit packed records).

def se8_geometry(n: int, width: int) -> dict:
    g = _Se8Geom()
    rc = lib().dwtfrag_se8_geometry(n, width, ctypes.byref(g))
    if rc != DWTFRAG_OK:
        raise DwtfragError(rc, "dwtfrag_se8_geometry")
    return {f: getattr(g, f) for f, _ in _Se8Geom._fields_}


def se8_protect(x: torch.Tensor, width: int, key: bytes, nonce: bytes, *, out=None, stream=None):
    """(priv, pub1, pub2) uint8 fragments of the bytes in ``x``; ``out`` may
    pass the three tensors to fill."""
    _check_dev(x, torch.uint8, "x")
    n = x.numel()
    g = se8_geometry(n, width)
    sizes = (g["priv_bytes"], g["pub1_bytes"], g["pub2_bytes"])
    if out is None:
        out = tuple(torch.empty(s, dtype=torch.uint8, device=x.device) for s in sizes)
    for t, s, name in zip(out, sizes, ("priv", "pub1", "pub2")):
        _check_dev(t, torch.uint8, name)
        if t.numel() != s:
            raise ValueError(f"{name} holds {t.numel()} bytes, the geometry needs {s}")
    rc = lib().dwtfrag_se8_protect(x.data_ptr(), n, width, _key16(key, "key"),
                                   _key16(nonce, "nonce"), out[0].data_ptr(), out[1].data_ptr(),
                                   out[2].data_ptr(), _stream(stream))
    if rc != DWTFRAG_OK:
        raise DwtfragError(rc, "dwtfrag_se8_protect")
    return tuple(out)


def se8_restore(priv: torch.Tensor, pub1: torch.Tensor, pub2: torch.Tensor, n: int, width: int,
                key: bytes, nonce: bytes, *, out: torch.Tensor | None = None,
                stream=None) -> torch.Tensor:
    """The original n bytes from the three fragments."""
    g = se8_geometry(n, width)
    for t, s, name in zip((priv, pub1, pub2), (g["priv_bytes"], g["pub1_bytes"], g["pub2_bytes"]),
                          ("priv", "pub1", "pub2")):
        _check_dev(t, torch.uint8, name)
        if t.numel() != s:
            raise ValueError(f"{name} holds {t.numel()} bytes, the geometry needs {s}")
    if out is None:
        out = torch.empty(n, dtype=torch.uint8, device=priv.device)
    _check_dev(out, torch.uint8, "out")
    if out.numel() < n:
        raise ValueError("out holds fewer than n bytes")
    rc = lib().dwtfrag_se8_restore(priv.data_ptr(), pub1.data_ptr(), pub2.data_ptr(), n, width,
                                   _key16(key, "key"), _key16(nonce, "nonce"), out.data_ptr(),
                                   _stream(stream))
    if rc != DWTFRAG_OK:
        raise DwtfragError(rc, "dwtfrag_se8_restore")
    return out
