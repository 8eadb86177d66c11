"""Batches of independent buffers and the launch-shape autotuner (ctypes).

A batch is planned once (``dwtfrag_batch_create``), its tables are copied
into a device tensor, and every protect / restore of the batch is one
persistent kernel launch draining one tile queue, which can be captured in a
HIP graph and replayed.  Marshalling only.

    b = Batch(buffers, widths, levels, keys, nonces)
    b.protect(); b.restore()          # b.privs / b.pubs / b.outs hold results
"""
from __future__ import annotations

import ctypes

import torch

from . import DWTFRAG_OK, DwtfragError, Launch, _check_dev, _key16, _stream, geometry, lib


class Item(ctypes.Structure):
    _fields_ = [("in_", ctypes.c_void_p), ("out", ctypes.c_void_p), ("priv", ctypes.c_void_p),
                ("pub", ctypes.c_void_p), ("n", ctypes.c_uint64), ("width", ctypes.c_uint32),
                ("levels", ctypes.c_uint32), ("key", ctypes.c_uint8 * 16),
                ("nonce", ctypes.c_uint8 * 16)]


class TuneEntry(ctypes.Structure):
    _fields_ = [("width", ctypes.c_uint32), ("levels", ctypes.c_uint32), ("launch", Launch)]


def autotune(x: torch.Tensor, width: int, levels: int, trials: int = 3, stream=None):
    """(Launch, microseconds per protect+restore) of the fastest launch shape
    for buffers like ``x`` (uint8 CUDA tensor)."""
    _check_dev(x, torch.uint8, "x")
    n = x.numel()
    g = geometry(n, width, levels)
    a = lambda v: (v + 255) // 256 * 256  # noqa: E731
    need = a(g["priv_bytes"]) + a(g["pub_bytes"]) + a(n) + g["workspace_bytes"]
    scratch = torch.empty(need + 256, dtype=torch.uint8, device=x.device)
    best, us = Launch(), ctypes.c_float()
    rc = lib().dwtfrag_autotune(x.data_ptr(), n, width, levels, scratch.data_ptr(), scratch.numel(),
                                trials, ctypes.byref(best), ctypes.byref(us), _stream(stream))
    if rc != DWTFRAG_OK:
        raise DwtfragError(rc, "dwtfrag_autotune")
    return best, float(us.value)


def tune_classes(buffers, widths, levels, trials: int = 2,
                 candidates=((64, 16), (128, 16), (256, 16)), stream=None):
    """Batch autotuner: for every (width, levels) class of the buffers, time a
    batched protect + restore of that class's buffers under each candidate
    tile shape (rows per tile, columns per lane; batch tiles always have 16
    columns per lane) with HIP events and keep the fastest.  Returns
    {(width, levels): Launch} for ``Batch(tune=...)``.

    Unlike ``autotune`` (one buffer alone, where finer tiles fill the device),
    this times the shapes where they will run: many buffers per launch, where
    coarser tiles save halo work."""
    groups = {}
    for i, (w, lv) in enumerate(zip(widths, levels)):
        groups.setdefault((w, lv), []).append(i)
    st = torch.cuda.current_stream() if stream is None else stream
    result = {}
    for key, idx in groups.items():
        xs = [buffers[i] for i in idx]
        best = None
        for rows, cols in candidates:
            b = Batch(xs, [key[0]] * len(xs), [key[1]] * len(xs), [bytes(16)] * len(xs),
                      [bytes(16)] * len(xs), tune={key: (rows, cols)})
            b.protect(stream=st)
            b.restore(stream=st)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(st)
            for _ in range(trials):
                b.protect(stream=st)
                b.restore(stream=st)
            e1.record(st)
            e1.synchronize()
            t = e0.elapsed_time(e1) / trials
            if best is None or t < best[0]:
                best = (t, rows, cols)
            b.close()
            del b
        result[key] = Launch(best[1], best[2])
    return result


class Batch:
    """A planned batch; owns the fragment and output tensors unless given."""

    def __init__(self, buffers, widths, levels, keys, nonces, *, privs=None, pubs=None, outs=None,
                 tune=None, device=None):
        count = len(buffers)
        if not (len(widths) == len(levels) == len(keys) == len(nonces) == count) or count == 0:
            raise ValueError("one width, level count, key and nonce per buffer")
        dev = device or buffers[0].device
        self.buffers = list(buffers)
        self.privs, self.pubs, self.outs = [], [], []
        items = (Item * count)()
        for i, x in enumerate(buffers):
            _check_dev(x, torch.uint8, "buffer")
            g = geometry(x.numel(), widths[i], levels[i])
            p = privs[i] if privs else torch.empty(g["priv_bytes"], dtype=torch.uint8, device=dev)
            q = pubs[i] if pubs else torch.empty(max(g["pub_bytes"] // 2, 1), dtype=torch.int16, device=dev)
            o = outs[i] if outs else torch.empty(x.numel(), dtype=torch.uint8, device=dev)
            # the plan carries pointers only: a short tensor would be written
            # (or read) past its end on the device, so sizes are checked here
            _check_dev(p, torch.uint8, "priv")
            _check_dev(q, torch.int16, "pub")
            _check_dev(o, torch.uint8, "out")
            if p.numel() != g["priv_bytes"] or 2 * q.numel() < g["pub_bytes"] or o.numel() < x.numel():
                raise ValueError(f"item {i}: fragment or output size does not match the geometry")
            self.privs.append(p)
            self.pubs.append(q[:g["pub_bytes"] // 2])
            self.outs.append(o)
            it = items[i]
            it.in_, it.out, it.priv, it.pub = x.data_ptr(), o.data_ptr(), p.data_ptr(), q.data_ptr()
            it.n, it.width, it.levels = x.numel(), widths[i], levels[i]
            ctypes.memmove(it.key, _key16(keys[i], "key"), 16)
            ctypes.memmove(it.nonce, _key16(nonces[i], "nonce"), 16)
        entries = None
        n_tune = 0
        if tune:
            entries = (TuneEntry * len(tune))()
            for k, ((w, lv), ln) in enumerate(tune.items()):
                entries[k].width, entries[k].levels = w, lv
                entries[k].launch = ln if isinstance(ln, Launch) else Launch(*ln)
            n_tune = len(tune)
        handle = ctypes.c_void_p()
        rc = lib().dwtfrag_batch_create(ctypes.addressof(items), count,
                                        ctypes.addressof(entries) if entries is not None else None,
                                        n_tune, ctypes.byref(handle))
        if rc != DWTFRAG_OK:
            raise DwtfragError(rc, "dwtfrag_batch_create")
        self._h = handle
        nbytes = int(lib().dwtfrag_batch_device_bytes(handle))
        self.plan = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        # the upload is asynchronous on the current stream
        self._upload_stream = torch.cuda.current_stream(dev)
        rc = lib().dwtfrag_batch_upload(handle, self.plan.data_ptr(), nbytes, _stream(None))
        if rc != DWTFRAG_OK:
            raise DwtfragError(rc, "dwtfrag_batch_upload")

    def _after_upload(self, stream):
        """Order a launch on `stream` after the plan's upload.  Under HIP graph
        capture on another stream the caller orders the two (a capture cannot
        wait for work outside it)."""
        s = stream if stream is not None else torch.cuda.current_stream(self.plan.device)
        if s != self._upload_stream and not torch.cuda.is_current_stream_capturing():
            s.wait_stream(self._upload_stream)

    def protect(self, stream=None):
        self._after_upload(stream)
        rc = lib().dwtfrag_batch_protect(self._h, _stream(stream))
        if rc != DWTFRAG_OK:
            raise DwtfragError(rc, "dwtfrag_batch_protect")

    def restore(self, stream=None):
        self._after_upload(stream)
        rc = lib().dwtfrag_batch_restore(self._h, _stream(stream))
        if rc != DWTFRAG_OK:
            raise DwtfragError(rc, "dwtfrag_batch_restore")

    def close(self):
        if getattr(self, "_h", None):
            lib().dwtfrag_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
