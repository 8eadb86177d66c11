"""Learned-predictor protect / restore and the GPU trainer (ctypes binding).

The predict step of the 5/3 lifting gains a correction from an integer
8-16-1 context network (declared with its exact formula in
``include/dwtfrag.h``).  This module marshals arguments only; the lifting,
the training-pair capture, the gradient sums, the Adam step and the
quantisation all run in ``libdwtfrag.so``.

    net = Predictor.from_arrays(w1, b1, w2, b2, shift)     # or Trainer(...).predictor()
    priv, pub = protect(x, width, levels, key, nonce, net)
    x2 = restore(priv, pub, n, width, levels, key, nonce, net)
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import DWTFRAG_OK, DwtfragError, _check_dev, _key16, _stream, lib

N_PARAMS = 161


class Predictor(ctypes.Structure):
    """dwtfrag_predictor: int8 w1[16][8], int8 w2[16], int32 b1[16], b2, shift."""
    _fields_ = [("w1", (ctypes.c_int8 * 8) * 16), ("w2", ctypes.c_int8 * 16),
                ("b1", ctypes.c_int32 * 16), ("b2", ctypes.c_int32), ("shift", ctypes.c_int32)]

    @staticmethod
    def from_arrays(w1, b1, w2, b2, shift) -> "Predictor":
        p = Predictor()
        ctypes.memmove(ctypes.addressof(p.w1), np.ascontiguousarray(w1, np.int8).tobytes(), 128)
        ctypes.memmove(ctypes.addressof(p.w2), np.ascontiguousarray(w2, np.int8).tobytes(), 16)
        ctypes.memmove(ctypes.addressof(p.b1), np.ascontiguousarray(b1, "<i4").tobytes(), 64)
        p.b2 = int(b2)
        p.shift = int(shift)
        return p

    @staticmethod
    def from_bytes(blob: bytes) -> "Predictor":
        if len(blob) != ctypes.sizeof(Predictor):
            raise ValueError("predictor blob must be 216 bytes")
        return Predictor.from_buffer_copy(blob)

    def to_bytes(self) -> bytes:
        return bytes(self)


assert ctypes.sizeof(Predictor) == 216


class _TrainerHead(ctypes.Structure):
    _fields_ = [("theta", ctypes.c_float * 161), ("m", ctypes.c_float * 161),
                ("v", ctypes.c_float * 161), ("grad", ctypes.c_float * 161),
                ("loss", ctypes.c_float), ("step", ctypes.c_int32), ("k1", ctypes.c_int32),
                ("k2", ctypes.c_int32), ("net", Predictor)]


TRAINER_BYTES = ctypes.sizeof(_TrainerHead)


def learned_geometry(n: int, width: int, levels: int) -> tuple[int, int]:
    """(workspace bytes, training pairs) of an n-byte buffer."""
    ws, pairs = ctypes.c_uint64(), ctypes.c_uint64()
    rc = lib().dwtfrag_learned_geometry(n, width, levels, ctypes.byref(ws), ctypes.byref(pairs))
    if rc != DWTFRAG_OK:
        raise DwtfragError(rc, "dwtfrag_learned_geometry")
    return ws.value, pairs.value


def workspace(n: int, width: int, levels: int, device=None) -> torch.Tensor:
    return torch.empty(learned_geometry(n, width, levels)[0], dtype=torch.uint8,
                       device=device or "cuda")


def protect(x, width, levels, key, nonce, net: Predictor, *, priv=None, pub=None, ws=None,
            stream=None):
    from . import geometry
    _check_dev(x, torch.uint8, "x")
    n = x.numel()
    g = geometry(n, width, levels)
    priv = torch.empty(g["priv_bytes"], dtype=torch.uint8, device=x.device) if priv is None else priv
    pub = torch.empty(g["pub_bytes"] // 2, dtype=torch.int16, device=x.device) if pub is None else pub
    ws = workspace(n, width, levels, x.device) if ws is None else ws
    _check_dev(priv, torch.uint8, "priv")
    _check_dev(pub, torch.int16, "pub")
    rc = lib().dwtfrag_protect_learned(x.data_ptr(), n, width, levels, _key16(key, "key"),
                                       _key16(nonce, "nonce"), ctypes.byref(net), priv.data_ptr(),
                                       pub.data_ptr(), ws.data_ptr(), ws.numel(), _stream(stream))
    if rc != DWTFRAG_OK:
        raise DwtfragError(rc, "dwtfrag_protect_learned")
    return priv, pub


def restore(priv, pub, n, width, levels, key, nonce, net: Predictor, *, out=None, ws=None,
            stream=None):
    from . import geometry
    _check_dev(priv, torch.uint8, "priv")
    _check_dev(pub, torch.int16, "pub")
    g = geometry(n, width, levels)
    if priv.numel() != g["priv_bytes"] or 2 * pub.numel() != g["pub_bytes"]:
        raise ValueError("fragment sizes do not match the geometry")
    out = torch.empty(n, dtype=torch.uint8, device=priv.device) if out is None else out
    ws = workspace(n, width, levels, priv.device) if ws is None else ws
    _check_dev(out, torch.uint8, "out")
    rc = lib().dwtfrag_restore_learned(priv.data_ptr(), pub.data_ptr(), n, width, levels,
                                       _key16(key, "key"), _key16(nonce, "nonce"),
                                       ctypes.byref(net), out.data_ptr(), ws.data_ptr(),
                                       ws.numel(), _stream(stream))
    if rc != DWTFRAG_OK:
        raise DwtfragError(rc, "dwtfrag_restore_learned")
    return out


def training_pairs(x, width, levels, *, ws=None, stream=None):
    """(ctx int8 (P, 8), target int32 (P,)) CUDA tensors of the buffer x."""
    _check_dev(x, torch.uint8, "x")
    n = x.numel()
    _, pairs = learned_geometry(n, width, levels)
    ctx = torch.empty((max(pairs, 1), 8), dtype=torch.int8, device=x.device)
    tgt = torch.empty(max(pairs, 1), dtype=torch.int32, device=x.device)
    ws = workspace(n, width, levels, x.device) if ws is None else ws
    rc = lib().dwtfrag_learned_pairs(x.data_ptr(), n, width, levels, ctx.data_ptr(),
                                     tgt.data_ptr(), ws.data_ptr(), ws.numel(), _stream(stream))
    if rc != DWTFRAG_OK:
        raise DwtfragError(rc, "dwtfrag_learned_pairs")
    return ctx[:pairs], tgt[:pairs]


class Trainer:
    """Device-resident quantisation-aware Adam trainer of the network."""

    def __init__(self, theta0, device="cuda", stream=None):
        self.state = torch.zeros(TRAINER_BYTES, dtype=torch.uint8, device=device)
        self.ws = torch.empty(int(lib().dwtfrag_trainer_workspace_bytes()), dtype=torch.uint8,
                              device=device)
        th = np.ascontiguousarray(theta0, dtype=np.float32)
        if th.size != N_PARAMS:
            raise ValueError("theta0 must hold 161 values")
        rc = lib().dwtfrag_trainer_init(self.state.data_ptr(),
                                        th.ctypes.data_as(ctypes.c_void_p), _stream(stream))
        if rc != DWTFRAG_OK:
            raise DwtfragError(rc, "dwtfrag_trainer_init")

    def step(self, ctx, target, lr, batch=0, n_batches=1, stream=None):
        """One Adam step on the interleaved batch ``batch`` of ``n_batches``:
        pairs batch, batch + n_batches, ..."""
        _check_dev(ctx, torch.int8, "ctx")
        _check_dev(target, torch.int32, "target")
        total = target.numel()
        if not 0 <= batch < n_batches or batch >= total:
            raise ValueError("batch index out of range")
        count = (total - batch + n_batches - 1) // n_batches
        rc = lib().dwtfrag_trainer_step(self.state.data_ptr(), ctx[batch:].data_ptr(),
                                        target[batch:].data_ptr(), count, n_batches, float(lr),
                                        self.ws.data_ptr(), self.ws.numel(), _stream(stream))
        if rc != DWTFRAG_OK:
            raise DwtfragError(rc, "dwtfrag_trainer_step")

    def read(self) -> _TrainerHead:
        """Host copy of the state (synchronises with the device)."""
        return _TrainerHead.from_buffer_copy(bytes(self.state.cpu().numpy().tobytes()))

    def predictor(self) -> Predictor:
        return Predictor.from_buffer_copy(bytes(self.read().net))
