"""Benchmark: protect + restore throughput on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config large|small]

A step is one pass of the whole hot path over the workload: protect (view,
3-level 5/3 lifting, band scatter, AES-CTR of LL) then restore (AES-CTR,
inverse lifting, byte store), inputs resident in HBM.  Prints one JSON line.

value      = n * K / (sum of the K protect and K restore launch durations),
             each launch started cache-cold with clean caches (a 1 GiB buffer
             is overwritten and read back before each direction, outside the
             events)                                      [GB/s of user bytes]
             (512 x 512 workload: n * K / wall time of K warm steps)
cold_dirty = the same with the overwrite alone: the caches then hold 1 GiB of
             dirty lines, whose write-back lands inside the timed launch
warm       = the same K steps back to back, value = n * K / wall time
roofline   = algorithmic bytes per launch (n + 2*H*W: read the bytes, write
             the int16 fragments; restore reads them back and writes bytes)
             / average launch duration of the dominant kernel (cold steps),
             against 8 TB/s HBM peak.  Durations come from HIP events
             recorded on the stream the kernels run on.
cpu_baseline = the CPU oracle on a bounded sample of the same workload, over
             a process pool of the host's cores (one-process time beside it),
             with openssl's AES-128-CTR rate on the same host as context.
"""
from __future__ import annotations

import argparse
import contextlib
import hashlib
import json
import multiprocessing
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PROFILES = os.path.join(ROOT, "profiles")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


@contextlib.contextmanager
def _closing_pool(processes: int):
    """A fork pool whose workers leave by finishing their queue (close and
    join) rather than by SIGTERM (a plain `with Pool()` terminates them):
    under a profiler that traps signals in every process, a terminated worker
    can hang in the profiler's handler and the join with it."""
    pool = multiprocessing.get_context("fork").Pool(processes)
    try:
        yield pool
    finally:
        pool.close()
        pool.join()


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = (len(xs) - 1) * q / 100.0
    lo, hi = int(k), min(int(k) + 1, len(xs) - 1)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


# sources of the kernels and launch planning the plain protect / restore runs
PLAIN_PATH_SOURCES = ("api.hip", "common.h", "fwd.hip", "inv.hip", "lift.h", "pack.h")
BATCH_PATH_SOURCES = PLAIN_PATH_SOURCES + ("batch.h", "batch.hip")


def source_hash(sources=PLAIN_PATH_SOURCES) -> str:
    """Hash of the kernel sources of a path; stored HBM-traffic figures are
    only used while it matches the one recorded with them."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1803_04880_amd", "csrc")
    for f in sources:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def stored_traffic(workload_key: str, sources=PLAIN_PATH_SOURCES):
    """Counter-measured HBM bytes per launch of a workload's kernels, from
    profiles/hbm_traffic.json, if recorded for the current sources (an entry
    with its own source_hash, else the file's)."""
    path = os.path.join(PROFILES, "hbm_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    entry = rec.get(workload_key)
    if not isinstance(entry, dict):
        return None
    if entry.get("source_hash", rec.get("source_hash")) != source_hash(sources):
        return None
    return entry


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            return next(l.split(":", 1)[1].strip() for l in f if l.startswith("model name"))
    except (OSError, StopIteration):
        return "unknown CPU"


def _host_cores() -> int:
    """Host cores this process may use, capped at 16 (a one-GPU share)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


# Process-pool run of the oracle: the sample's arrays live in anonymous shared
# memory mapped before the pool forks, and each task applies the oracle's own
# 1-D pass (or its keystream) to a block of rows or columns of them.
_SH = {}


def _shared_i64(name, count):
    import mmap

    import numpy as np
    mm = mmap.mmap(-1, max(8, 8 * count))
    _SH[name] = np.frombuffer(mm, dtype=np.int64, count=count)


def _rows_task(args):
    from oracle import dwt53
    src, dst, h, w, r0, r1, inverse = args
    a = _SH[src][:h * w].reshape(h, w)
    b = _SH[dst][:h * w].reshape(h, w)
    b[r0:r1] = (dwt53.inv_1d if inverse else dwt53.fwd_1d)(a[r0:r1])
    return r1 - r0


def _cols_task(args):
    from oracle import dwt53
    src, dst, h, w, c0, c1, inverse = args
    a = _SH[src][:h * w].reshape(h, w)
    b = _SH[dst][:h * w].reshape(h, w)
    b[:, c0:c1] = (dwt53.inv_1d if inverse else dwt53.fwd_1d)(a[:, c0:c1].T).T
    return c1 - c0


def _ctr_task(args):
    import numpy as np

    from oracle import aes128
    key, nonce, nbytes, b0, b1 = args
    buf = _SH["ctr"].view(np.uint8)
    lo, hi = 16 * b0, min(nbytes, 16 * b1)
    buf[lo:hi] ^= aes128.ctr_keystream(key, nonce, hi - lo, offset_blocks=b0)
    return hi - lo


def _blocks(total, parts):
    step = -(-total // parts)
    return [(i, min(total, i + step)) for i in range(0, total, step)]


def _pool_protect_restore(pool, cores, sample, w, levels, key, nonce):
    """Oracle protect then restore of `sample`, each 1-D pass split over the
    pool (row blocks for the row pass, column blocks for the column pass, one
    barrier per pass) and the counter-mode keystream split by block ranges.
    Returns (priv, pub, restored bytes)."""
    import numpy as np

    from oracle import fragment
    g = fragment.geometry(sample.size, w, levels)
    h0 = g["height"]
    A, B = _SH["a"], _SH["b"]
    A[:h0 * w] = fragment.view(sample, w).reshape(-1)
    details = []
    h, ww = h0, w
    for _ in range(levels):   # forward: rows into b, columns back into a
        pool.map(_rows_task, [("a", "b", h, ww, r0, r1, False) for r0, r1 in _blocks(h, cores)])
        pool.map(_cols_task, [("b", "a", h, ww, c0, c1, False) for c0, c1 in _blocks(ww, cores)])
        m = A[:h * ww].reshape(h, ww)
        hl, wl = (h + 1) // 2, (ww + 1) // 2
        details.append((m[:hl, wl:].copy(), m[hl:, :wl].copy(), m[hl:, wl:].copy()))
        ll = m[:hl, :wl].copy()
        A[:hl * wl] = ll.reshape(-1)
        h, ww = hl, wl
    ll = A[:h * ww].reshape(h, ww).copy()
    priv_plain, pub = fragment.serialize(ll, details)

    def ctr(data):
        n = len(data)
        nblk = -(-n // 16)
        _SH["ctr"].view(np.uint8)[:n] = np.frombuffer(data, np.uint8)
        pool.map(_ctr_task, [(key, nonce, n, b0, b1) for b0, b1 in _blocks(nblk, cores)])
        return _SH["ctr"].view(np.uint8)[:n].tobytes()

    priv = ctr(priv_plain)
    # restore: keystream, then levels L..1 (columns inverse into b, rows into a)
    ll, dets = fragment.deserialize(ctr(priv), pub, g)
    cur = ll
    for lvl in range(levels, 0, -1):
        hlb, lhb, hhb = dets[lvl - 1]
        top = np.concatenate([cur, hlb], axis=1)
        full = np.concatenate([top, np.concatenate([lhb, hhb], axis=1)], axis=0)
        h, ww = full.shape
        A[:h * ww] = full.reshape(-1)
        pool.map(_cols_task, [("a", "b", h, ww, c0, c1, True) for c0, c1 in _blocks(ww, cores)])
        pool.map(_rows_task, [("b", "a", h, ww, r0, r1, True) for r0, r1 in _blocks(h, cores)])
        cur = A[:h * ww].reshape(h, ww).copy()
    out = (cur.reshape(-1)[:sample.size] & 0xFF).astype(np.uint8).tobytes()
    return priv, pub, out


def _openssl_ctr(cores: int):
    """`openssl speed -evp aes-128-ctr` on 16 KiB blocks, one process and
    `cores` processes (GB/s), or None without the tool."""
    import re
    import shutil
    import subprocess

    if not shutil.which("openssl"):
        return None
    out = {}
    for procs in sorted({1, cores}):
        cmd = ["openssl", "speed", "-bytes", "16384", "-seconds", "2", "-evp", "aes-128-ctr"]
        if procs > 1:
            cmd[2:2] = ["-multi", str(procs)]
        try:
            txt = subprocess.run(cmd, capture_output=True, text=True, timeout=120).stdout
        except (OSError, subprocess.SubprocessError):
            return None
        m = re.findall(r"^(?:aes-128-ctr|evp)\s+([0-9.]+)k", txt, flags=re.I | re.M)
        if not m:
            return None
        out[f"procs_{procs}"] = round(float(m[-1]) * 1e3 / 1e9, 3)
    return dict(unit="GB/s", block_bytes=16384, **out)


def cpu_baseline(cfg, rows: int = 2048, row0: int = 2048):
    """The CPU oracle (as it stands) on `rows` rows of the workload: protect +
    restore in one process, then the same over a process pool of the host's
    cores; plus openssl's AES-128-CTR rate on the same host as context."""
    import multiprocessing

    import numpy as np
    from oracle import fragment
    w, lv, key, nonce = cfg["width"], cfg["levels"], cfg["key"], cfg["nonce"]
    sample = np.ascontiguousarray(cfg["buf"][row0 * w:(row0 + rows) * w])
    t0 = time.perf_counter()
    priv, pub = fragment.protect(sample, w, lv, key, nonce)
    back = fragment.restore(priv, pub, sample.size, w, lv, key, nonce)
    dt1 = time.perf_counter() - t0
    assert back == sample.tobytes()
    cores = _host_cores()
    cells = rows * w
    _shared_i64("a", cells)
    _shared_i64("b", cells)
    _shared_i64("ctr", -(-2 * cells // 8) + 2)
    with _closing_pool(cores) as pool:
        pool.map(_rows_task, [("a", "b", 1, 1, 0, 1, False)] * cores)  # workers up
        t0 = time.perf_counter()
        ppriv, ppub, pback = _pool_protect_restore(pool, cores, sample, w, lv, key, nonce)
        dtp = time.perf_counter() - t0
    _SH.clear()
    assert (ppriv, ppub, pback) == (priv, pub, sample.tobytes()), "pooled oracle differs"
    # the 512 x 512, one-level workload whole, one process (a fraction of a second)
    import synth
    small = synth.config_small()
    t0 = time.perf_counter()
    spriv, spub = fragment.protect(small["buf"], small["width"], small["levels"], small["key"],
                                   small["nonce"])
    sback = fragment.restore(spriv, spub, small["buf"].size, small["width"], small["levels"],
                             small["key"], small["nonce"])
    dts = time.perf_counter() - t0
    assert sback == small["buf"].tobytes()
    return dict(value=round(sample.size / dtp / 1e9, 4), unit="GB/s", cores=cores, kind="oracle",
                cpu_model=_cpu_model(),
                small_workload=dict(value=round(small["buf"].size / dts / 1e9, 5),
                                    seconds=round(dts, 4), workload=small["name"],
                                    processes=1),
                one_process=dict(value=round(sample.size / dt1 / 1e9, 4), seconds=round(dt1, 2)),
                openssl_aes128_ctr=_openssl_ctr(cores),
                sample=f"rows {row0}..{row0 + rows} of the {w}-wide workload "
                       f"({sample.size / 2**20:.0f} MiB, {lv} levels), protect+restore, NumPy "
                       f"oracle over a pool of {cores} processes ({dtp:.1f} s; one process "
                       f"{dt1:.1f} s) on {_cpu_model()}; pooled fragments equal the "
                       f"one-process ones")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", choices=["large", "small", "learned", "serve", "batch", "se8"],
                    default="large")
    ap.add_argument("--count", type=int, default=2048, help="batch config: number of buffers")
    ap.add_argument("--batch-subset", default="",
                    help="batch config, for counter runs: LEVELS,MIN_BYTES,MAX_ITEMS[,KIND] keeps "
                         "only the buffers of that depth and at least that size (and content kind: "
                         "smooth, markov, uniform), at most that many")
    ap.add_argument("--no-tune", action="store_true", help="batch config: default tile shapes")
    ap.add_argument("--duration", type=float, default=30.0, help="serve config: seconds of arrivals")
    ap.add_argument("--rate", type=float, default=2000.0, help="serve config: arrivals per second")
    ap.add_argument("--learned-streams", type=int, default=16,
                    help="learned config: streams the per-image calls are spread over")
    ap.add_argument("--images", type=int, default=0,
                    help="learned config: number of 4096x4096 images (default 64)")
    ap.add_argument("--seg-rows", type=int, default=0)
    ap.add_argument("--lane-cols", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-small", action="store_true",
                    help="large config: skip the 512 x 512 latency measurement")
    ap.add_argument("--no-parity", action="store_true")
    ap.add_argument("--profile-run", action="store_true",
                    help="no timing: 2 plain device copies of n bytes and 2 of n/4 bytes "
                         "(counter calibration), then 2 protect and 2 restore launches, for "
                         "rocprofv3")
    ap.add_argument("--print-source-hash", action="store_true")
    args = ap.parse_args()

    if args.print_source_hash:
        print(source_hash())                      # plain path
        print(source_hash(BATCH_PATH_SOURCES))    # batch path
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(buffers are independent, so several GPUs would each take whole buffers).",
              file=sys.stderr)
        sys.exit(2)

    if args.config == "learned":
        return run_learned(args)
    if args.config == "serve":
        return run_serve(args)
    if args.config == "batch":
        return run_batch(args)
    if args.config == "se8":
        return run_se8(args)

    import numpy as np
    import torch

    import paper_1803_04880_amd as dwtfrag
    import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    t0 = time.time()
    cfg = synth.config_large() if args.config == "large" else synth.config_small()
    buf = cfg["buf"]
    n, width, levels, key, nonce = buf.size, cfg["width"], cfg["levels"], cfg["key"], cfg["nonce"]
    log(f"workload {cfg['name']}: n={n} generated in {time.time() - t0:.1f}s")
    g = dwtfrag.geometry(n, width, levels)
    H = g["height"]
    launch = dwtfrag.Launch(args.seg_rows, args.lane_cols) if (args.seg_rows or args.lane_cols) else None

    x = torch.from_numpy(buf).to(dev)
    priv = torch.empty(g["priv_bytes"], dtype=torch.uint8, device=dev)
    pub = torch.empty(g["pub_bytes"] // 2, dtype=torch.int16, device=dev)
    out = torch.empty(n, dtype=torch.uint8, device=dev)
    ws = dwtfrag.workspace(n, width, levels, dev)

    def protect():
        dwtfrag.protect(x, width, levels, key, nonce, priv=priv, pub=pub, ws=ws, launch=launch)

    def restore():
        dwtfrag.restore(priv, pub, n, width, levels, key, nonce, out=out, ws=ws, launch=launch)

    if args.profile_run:
        for _ in range(2):
            out.copy_(x)  # plain copy kernel: reads n bytes, writes n bytes
        torch.cuda.synchronize()
        for _ in range(2):  # a second size for the counters' calibration
            out[:n // 4].copy_(x[n // 4:n // 2])
        torch.cuda.synchronize()
        for _ in range(2):
            protect()
            restore()
        torch.cuda.synchronize()
        log(f"profile run done: n={n} bytes, {n + 2 * H * width} algorithmic bytes per launch")
        return

    # parity gate: fragments against the oracle's stored digests, restore exact
    protect()
    restore()
    torch.cuda.synchronize()
    bit_exact = bool(torch.equal(out, x))
    if not args.no_parity:
        with open(os.path.join(ROOT, "tests", "golden", "oracle_digests.json")) as f:
            gold = json.load(f)[args.config]
        bit_exact &= hashlib.sha256(priv.cpu().numpy().tobytes()).hexdigest() == gold["priv_sha256"]
        bit_exact &= hashlib.sha256(pub.cpu().numpy().tobytes()).hexdigest() == gold["pub_sha256"]
    log(f"parity vs oracle: {'bit-exact' if bit_exact else 'MISMATCH'}")

    for _ in range(args.warmup):
        protect()
        restore()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    alg_bytes = n + 2 * H * width  # per launch, each direction

    scratch = None
    evict_sum = torch.zeros((), dtype=torch.int64, device=dev)

    def evict(clean: bool, k: int):
        """Outside the events: overwrite a 1 GiB scratch buffer, so the
        Infinity Cache and the L2s hold none of the workload's data; clean:
        then read it back, so they hold no dirty lines either (otherwise the
        write-back of the fill's 1 GiB lands inside the next timed launch)."""
        scratch.fill_(k & 255)
        if clean:
            evict_sum.add_(scratch.view(torch.int64).sum())

    def run_steps(cold: bool, clean: bool = True):
        """K steps; cold: evict(clean) before each direction."""
        ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        for k in range(args.steps):
            if cold:
                evict(clean, 2 * k + 1)
            ev[k][0].record(stream)
            protect()
            ev[k][1].record(stream)
            if cold:
                evict(clean, 2 * k + 2)
            ev[k][2].record(stream)
            restore()
            ev[k][3].record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
        tp = [ev[k][0].elapsed_time(ev[k][1]) * 1e3 for k in range(args.steps)]  # us
        tr = [ev[k][2].elapsed_time(ev[k][3]) * 1e3 for k in range(args.steps)]
        tpair = [a + b for a, b in zip(tp, tr)]
        avg_p, avg_r = sum(tp) / len(tp), sum(tr) / len(tr)
        dom = "fwd_kernel" if avg_p >= avg_r else "inv_kernel"
        dom_us = max(avg_p, avg_r)
        return dict(
            wall=wall, busy_us=sum(tpair), dominant=dom, dom_us=dom_us,
            achieved=alg_bytes / (dom_us * 1e-6) / 1e9,
            pair_frac=2 * alg_bytes / (avg_p + avg_r) / 1e3 / HBM_PEAK_GBS,
            latency={"protect_p50": round(percentile(tp, 50), 1),
                     "protect_p99": round(percentile(tp, 99), 1),
                     "restore_p50": round(percentile(tr, 50), 1),
                     "restore_p99": round(percentile(tr, 99), 1),
                     "pair_p50": round(percentile(tpair, 50), 1),
                     "pair_p99": round(percentile(tpair, 99), 1)},
            avg_us={"protect": round(avg_p, 2), "restore": round(avg_r, 2)})

    # headline of the 256 MiB workload: cache-cold steps (clean caches), value
    # = n * K / (sum of the protect and restore launch durations); cold steps
    # behind a fill alone (dirty caches) and warm back-to-back steps as
    # footnotes.  The 512 x 512 workload is a latency measurement of data
    # that stays in the caches: warm steps, value = n * K / wall time.
    warm = run_steps(False)
    cold_dirty = None
    if args.config == "large":
        scratch = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        evict(True, 0)  # the reduction's first call sets itself up (host time)
        torch.cuda.synchronize()
        cold = run_steps(True)
        cold_dirty = run_steps(True, clean=False)
        value = n * args.steps / (cold["busy_us"] * 1e-6) / 1e9
    else:
        cold = dict(warm, busy_us=warm["wall"] * 1e6)
        value = n * args.steps / warm["wall"] / 1e9
    traffic = stored_traffic(args.config)
    roofline = {"bound": "hbm", "achieved": round(cold["achieved"], 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(cold["achieved"] / HBM_PEAK_GBS, 4),
                "traffic": traffic.get(cold["dominant"]) if traffic else None,
                "kernel": cold["dominant"], "bytes_per_launch": alg_bytes,
                "avg_launch_us": round(cold["dom_us"], 2)}

    # context for the HBM fraction: the rate of a plain device copy of the
    # same n bytes (read n, write n) on this GPU, timed the same way as the
    # headline launches (cold, clean caches: one event pair per copy), and
    # back to back as well
    spare = torch.empty_like(x)
    spare.copy_(x)
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0.record(stream)
    for _ in range(20):
        spare.copy_(x)
    c1.record(stream)
    torch.cuda.synchronize()
    copy_warm_us = c0.elapsed_time(c1) * 1e3 / 20
    copy_us = copy_dirty_us = copy_warm_us

    def cold_copies(clean: bool, op=lambda: spare.copy_(x)) -> float:
        cev = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(20)]
        for k in range(20):
            evict(clean, k)
            cev[k][0].record(stream)
            op()
            cev[k][1].record(stream)
        torch.cuda.synchronize()
        return sum(a.elapsed_time(b) for a, b in cev) * 1e3 / 20

    shaped = None
    if scratch is not None:
        copy_us = cold_copies(True)
        copy_dirty_us = cold_copies(False)
        # the library's reference streams: the same bytes as the forward
        # (widen: read n, write 2n) and the inverse (narrow: read 2n, write
        # n) in one-shot launches, timed as the headline launches
        wide = torch.empty(n, dtype=torch.int16, device=dev)
        dwtfrag.ref_widen(x, wide)
        dwtfrag.ref_narrow(wide, spare)
        torch.cuda.synchronize()
        assert torch.equal(spare, x), "reference streams do not round trip"
        widen_us = cold_copies(True, lambda: dwtfrag.ref_widen(x, wide))
        narrow_us = cold_copies(True, lambda: dwtfrag.ref_narrow(wide, spare))
        del wide
        like = widen_us if cold["dominant"] == "fwd_kernel" else narrow_us
        shaped = {"widen_u8_to_i16": {"us": round(widen_us, 1),
                                      "gbps": round(alg_bytes / (widen_us * 1e-6) / 1e9, 1)},
                  "narrow_i16_to_u8": {"us": round(narrow_us, 1),
                                       "gbps": round(alg_bytes / (narrow_us * 1e-6) / 1e9, 1)},
                  "dominant_kernel_frac_of_same_shape": round(like / cold["dom_us"], 4)}
        del scratch
    del spare
    copy_gbps = 2 * n / (copy_us * 1e-6) / 1e9
    device_copy = {"us": round(copy_us, 1), "gbps": round(copy_gbps, 1),
                   "cache": "as the headline launches",
                   "cold_dirty_gbps": round(2 * n / (copy_dirty_us * 1e-6) / 1e9, 1),
                   "warm_back_to_back_gbps": round(2 * n / (copy_warm_us * 1e-6) / 1e9, 1),
                   "dominant_kernel_frac_of_copy": round(cold["achieved"] / copy_gbps, 4)}
    if shaped is not None:
        device_copy["same_traffic_shape"] = shaped

    result = {
        "metric": "protect+restore GB/s on 1 MI355X (% HBM roofline), bit-exact; p50/p99 latency",
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(cold["busy_us"] / args.steps / 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int16/int32",
        "data": "synthetic",
        "config": {"workload": cfg["name"], "n_bytes": n, "rows": H, "width": width,
                   "levels": levels,
                   "cache": ("cold (1 GiB overwritten, then read back, before each direction)"
                             if args.config == "large" else "warm (back to back)"),
                   "launch": {"seg_rows": args.seg_rows, "lane_cols": args.lane_cols}},
        "bit_exact": bit_exact,
        "latency_us": cold["latency"],
        "roofline": roofline,
        "pair_hbm_frac": round(cold["pair_frac"], 4),
        "warm": {"value": round(n * args.steps / warm["wall"] / 1e9, 2),
                 "ms_per_step": round(warm["wall"] / args.steps * 1e3, 4),
                 "latency_us": warm["latency"], "avg_launch_us": warm["avg_us"],
                 "roofline_frac": round(warm["achieved"] / HBM_PEAK_GBS, 4),
                 "pair_hbm_frac": round(warm["pair_frac"], 4),
                 "note": "K protect + restore steps back to back (inputs and fragments partly "
                         "cached); value = n * K / wall time"},
        "device_copy": device_copy,
        "cpu_baseline": None,
    }
    if cold_dirty is not None:
        result["cold_dirty"] = {
            "value": round(n * args.steps / (cold_dirty["busy_us"] * 1e-6) / 1e9, 2),
            "latency_us": cold_dirty["latency"], "avg_launch_us": cold_dirty["avg_us"],
            "roofline_frac": round(cold_dirty["achieved"] / HBM_PEAK_GBS, 4),
            "note": "1 GiB overwritten (not read back) before each direction: the caches hold "
                    "1 GiB of dirty lines, whose write-back falls inside the timed launch"}
    if args.config == "small" or not args.no_small:
        result["small_latency_us"] = small_latency(dev, stream)
    if not args.no_cpu_baseline and args.config == "large":
        log("timing the CPU oracle on a bounded sample ...")
        result["cpu_baseline"] = cpu_baseline(cfg)
    print(json.dumps(result), flush=True)


def small_latency(dev, stream, steps: int = 1000, warmup: int = 50):
    """Latency of the 512 x 512, one-level workload (inputs resident, warm):
    p50 / p99 of protect, restore and the pair from HIP events, after a
    byte-for-byte check against the oracle's stored digests."""
    import torch

    import paper_1803_04880_amd as dwtfrag
    import synth
    cfg = synth.config_small()
    buf = cfg["buf"]
    n, w, lv, key, nonce = buf.size, cfg["width"], cfg["levels"], cfg["key"], cfg["nonce"]
    g = dwtfrag.geometry(n, w, lv)
    x = torch.from_numpy(buf).to(dev)
    priv = torch.empty(g["priv_bytes"], dtype=torch.uint8, device=dev)
    pub = torch.empty(g["pub_bytes"] // 2, dtype=torch.int16, device=dev)
    out = torch.empty(n, dtype=torch.uint8, device=dev)
    dwtfrag.protect(x, w, lv, key, nonce, priv=priv, pub=pub)
    dwtfrag.restore(priv, pub, n, w, lv, key, nonce, out=out)
    torch.cuda.synchronize()
    with open(os.path.join(ROOT, "tests", "golden", "oracle_digests.json")) as f:
        gold = json.load(f)["small"]
    exact = (hashlib.sha256(priv.cpu().numpy().tobytes()).hexdigest() == gold["priv_sha256"]
             and hashlib.sha256(pub.cpu().numpy().tobytes()).hexdigest() == gold["pub_sha256"]
             and bool(torch.equal(out, x)))
    for _ in range(warmup):
        dwtfrag.protect(x, w, lv, key, nonce, priv=priv, pub=pub)
        dwtfrag.restore(priv, pub, n, w, lv, key, nonce, out=out)
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    torch.cuda.synchronize()
    for k in range(steps):
        ev[k][0].record(stream)
        dwtfrag.protect(x, w, lv, key, nonce, priv=priv, pub=pub)
        ev[k][1].record(stream)
        dwtfrag.restore(priv, pub, n, w, lv, key, nonce, out=out)
        ev[k][2].record(stream)
    torch.cuda.synchronize()
    tp = [ev[k][0].elapsed_time(ev[k][1]) * 1e3 for k in range(steps)]
    tr = [ev[k][1].elapsed_time(ev[k][2]) * 1e3 for k in range(steps)]
    tq = [a + b for a, b in zip(tp, tr)]
    # Context: one-shot streams of the same bytes (protect's traffic, read n
    # and write 2n; restore's, read 2n and write n), launched and timed the
    # same way.  At this size both are launch-bound, so these are the floor
    # a launch of the path reaches under the same events and calls.
    wide = torch.empty(n, dtype=torch.int16, device=dev)
    narrow = torch.empty(n, dtype=torch.uint8, device=dev)
    for _ in range(warmup):
        dwtfrag.ref_widen(x, wide)
        dwtfrag.ref_narrow(wide, narrow)
    torch.cuda.synchronize()
    for k in range(steps):
        ev[k][0].record(stream)
        dwtfrag.ref_widen(x, wide)
        ev[k][1].record(stream)
        dwtfrag.ref_narrow(wide, narrow)
        ev[k][2].record(stream)
    torch.cuda.synchronize()
    sw = [ev[k][0].elapsed_time(ev[k][1]) * 1e3 for k in range(steps)]
    sn = [ev[k][1].elapsed_time(ev[k][2]) * 1e3 for k in range(steps)]
    return {"workload": cfg["name"], "steps": steps, "bit_exact": exact,
            "protect_p50": round(percentile(tp, 50), 1), "protect_p99": round(percentile(tp, 99), 1),
            "restore_p50": round(percentile(tr, 50), 1), "restore_p99": round(percentile(tr, 99), 1),
            "pair_p50": round(percentile(tq, 50), 1), "pair_p99": round(percentile(tq, 99), 1),
            "one_shot_streams": {
                "widen_p50": round(percentile(sw, 50), 1), "widen_p99": round(percentile(sw, 99), 1),
                "narrow_p50": round(percentile(sn, 50), 1), "narrow_p99": round(percentile(sn, 99), 1),
                "note": "same bytes and traffic as protect / restore, one-shot, timed the same way"}}


# Algorithmic VALU instructions per 8x8 block of the blocked protection: the
# operations of the definitions, each counted as the gfx950 instructions it
# needs at least (a 32-bit rotate is one funnel shift, a 64-bit rotate, shift
# or add two instructions, three-input XOR / choose / majority one bit
# operation, three-term sums one three-input add):
#   SHA-256: 64 rounds x 14 + 48 schedule words x 10 + 8 = 1384
#   SHA-512: 80 rounds x 34 + 64 schedule words x 22 + 16 = 4144
#   lifting, two levels: 3 per sample and pass (predict or update), 160 = 480
#   bytes in (64), records out (2 per coefficient, 128), hash messages (20)
#   AES-128-CTR: 5/16 of a T-table block (about 232) per 8x8 block = 72
SE8_OPS_PER_BLOCK = 1384 + 4144 + 480 + 64 + 128 + 20 + 72
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12   # int32 VALU lane instructions per second (T)


def run_se8(args):
    """Blocked (per-8x8) protection of the 256 MiB workload: two-level block
    lifting, SHA-256 / SHA-512 keystreams over the public fragments, packed
    10/11-bit records, AES-128-CTR private fragment; protect + restore."""
    import numpy as np
    import torch

    import paper_1803_04880_amd as dwtfrag
    import synth
    from oracle import aes128, se8

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    cfg = synth.config_large()
    buf = cfg["buf"]
    n, width, key, nonce = buf.size, cfg["width"], cfg["key"], cfg["nonce"]
    g = dwtfrag.se8_geometry(n, width)
    x = torch.from_numpy(buf).to(dev)
    frags = tuple(torch.empty(g[k], dtype=torch.uint8, device=dev)
                  for k in ("priv_bytes", "pub1_bytes", "pub2_bytes"))
    out = torch.empty(n, dtype=torch.uint8, device=dev)

    def protect():
        dwtfrag.se8_protect(x, width, key, nonce, out=frags)

    def restore():
        dwtfrag.se8_restore(*frags, n, width, key, nonce, out=out)

    protect()
    restore()
    torch.cuda.synchronize()
    ok = bool(torch.equal(out, x))
    # sampled blocks against the oracle's per-block definition (the whole
    # buffer is 4 M blocks: too many for the oracle)
    rng = np.random.default_rng(8)
    wb = g["block_cols"]
    for b in sorted({0, 255, 256, g["blocks"] - 1} | set(int(v) for v in
                                                        rng.integers(0, g["blocks"], 12))):
        by, bx = divmod(b, wb)
        rows = np.stack([buf[(8 * by + r) * width + 8 * bx:(8 * by + r) * width + 8 * bx + 8]
                         for r in range(8)])
        bands = se8.block_bands(rows)
        pr = se8.record(bands, "priv")
        p1 = se8.record(bands, "pub1") ^ se8.pub1_keystream(pr, key, nonce, b)
        p2 = se8.record(bands, "pub2") ^ se8.pub2_keystream(p1, key, nonce, b)
        j0 = (5 * b) // 16
        ks = aes128.ctr_keystream(key, nonce, 32, offset_blocks=j0).tobytes()
        enc = bytes(a ^ k for a, k in zip(pr.to_bytes(5, "little"), ks[5 * b - 16 * j0:]))
        lo = (124 * b) // 8
        seg = int.from_bytes(frags[1][lo:lo + 17].cpu().numpy().tobytes(), "little")
        ok &= frags[0][5 * b:5 * b + 5].cpu().numpy().tobytes() == enc
        ok &= (seg >> (124 * b - 8 * lo)) & ((1 << 124) - 1) == p1
        ok &= int.from_bytes(frags[2][60 * b:60 * b + 60].cpu().numpy().tobytes(), "little") == p2
    log(f"blocked protection: round trip and sampled blocks vs oracle: {'exact' if ok else 'MISMATCH'}")
    steps = args.steps if args.steps != 50 else 20
    warmup = args.warmup if args.warmup != 5 else 2
    for _ in range(warmup):
        protect()
        restore()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    w0 = time.perf_counter()
    for k in range(steps):
        ev[k][0].record(stream)
        protect()
        ev[k][1].record(stream)
        restore()
        ev[k][2].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    tp = [ev[k][0].elapsed_time(ev[k][1]) * 1e3 for k in range(steps)]
    tr = [ev[k][1].elapsed_time(ev[k][2]) * 1e3 for k in range(steps)]
    avg_p, avg_r = sum(tp) / steps, sum(tr) / steps
    dom = "se8_protect_kernel" if avg_p >= avg_r else "se8_restore_kernel"
    dom_us = max(avg_p, avg_r)
    ops = SE8_OPS_PER_BLOCK * g["blocks"]
    achieved = ops / (dom_us * 1e-6) / 1e12
    frag_bytes = g["priv_bytes"] + g["pub1_bytes"] + g["pub2_bytes"]
    result = {
        "metric": "blocked (8x8, SHA-2 keyed) protect+restore GB/s on 1 MI355X, exact",
        "value": round(n * steps / wall / 1e9, 2), "unit": "GB/s", "n_gpus": 1, "steps": steps,
        "warmup": warmup, "ms_per_step": round(wall / steps * 1e3, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int32/u32", "data": "synthetic",
        "config": {"workload": cfg["name"] + ", per-8x8-block protection", "n_bytes": n,
                   "width": width, "blocks": g["blocks"]},
        "exact": ok,
        "latency_us": {"protect_p50": round(percentile(tp, 50), 1),
                       "restore_p50": round(percentile(tr, 50), 1)},
        "roofline": {"bound": "alu", "achieved": round(achieved, 2),
                     "peak": round(VALU_PEAK_TOPS, 1), "unit": "T lane-instructions/s (int32 VALU)",
                     "frac": round(achieved / VALU_PEAK_TOPS, 4), "traffic": None,
                     "kernel": dom, "ops_per_launch": ops, "avg_launch_us": round(dom_us, 2),
                     "hbm_frac": round((n + frag_bytes) / (dom_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)},
        "cpu_baseline": None,
    }
    print(json.dumps(result), flush=True)


def _batch_item(spec):
    import synth
    return synth.batch_buffer(spec)


def run_batch(args):
    """Uneven batch: --count buffers (default 2048), sizes floor(exp U(ln 2^12,
    ln 2^26)), content kinds and levels U{1..4} from the seeded specs of
    synth.batch_specs, default widths, mixed content from synth.batch_buffer.
    Rows per tile are autotuned per (width, levels) class before timing.  A
    step is one batched protect + one batched restore of every buffer, each
    one persistent kernel launch; the timed steps replay the two directions
    as captured HIP graphs (eager steps reported beside them)."""
    import multiprocessing

    import numpy as np
    import torch

    import synth
    from oracle import fragment
    from paper_1803_04880_amd import batch as B

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    specs = synth.batch_specs(args.count)
    if args.batch_subset:
        fields = args.batch_subset.split(",")
        lv, min_n, most = (int(v) for v in fields[:3])
        kind = fields[3] if len(fields) > 3 else None
        specs = [s for s in specs if s["levels"] == lv and s["n"] >= min_n
                 and (kind is None or s["kind"] == kind)][:most]
    t0 = time.time()
    xs = []
    with _closing_pool(_host_cores()) as pool:
        for buf in pool.imap(_batch_item, specs, chunksize=4):
            xs.append(torch.from_numpy(buf).to(dev))
    total = sum(s["n"] for s in specs)
    log(f"{len(specs)} buffers, {total / 1e9:.2f} GB of mixed content in {time.time() - t0:.1f}s")
    widths = [s["width"] for s in specs]
    levels = [s["levels"] for s in specs]
    keys = [np.random.default_rng(s["seed"] + 10**6).bytes(16) for s in specs]
    nonces = [s["nonce"] for s in specs]
    t0 = time.time()
    tune = {}
    if not args.no_tune:
        tune = B.tune_classes(xs, widths, levels)
        log(f"tuned {len(tune)} classes in {time.time() - t0:.1f}s: "
            + ", ".join(f"{k}->({v.seg_rows},{v.lane_cols})" for k, v in sorted(tune.items())))
    b = B.Batch(xs, widths, levels, keys, nonces, tune=tune)
    b.protect()
    b.restore()
    torch.cuda.synchronize()
    ok = all(bool(torch.equal(o, x)) for o, x in zip(b.outs, xs))
    # fragments of a sample of items against the oracle (the small ones:
    # the oracle takes seconds per MB)
    small = sorted(range(len(specs)), key=lambda i: specs[i]["n"])[:6] + [
        i for i in range(len(specs)) if specs[i]["n"] < (1 << 20)][-2:]
    for i in small:
        buf = xs[i].cpu().numpy()
        opriv, opub = fragment.protect(buf, widths[i], levels[i], keys[i], nonces[i])
        ok &= b.privs[i].cpu().numpy().tobytes() == opriv
        ok &= b.pubs[i].cpu().numpy().tobytes() == opub
    log(f"batch: round trip of every item and {len(small)} items' fragments vs oracle: "
        f"{'exact' if ok else 'MISMATCH'}")
    steps = args.steps if args.steps != 50 else 10
    warmup = args.warmup if args.warmup != 5 else 2
    for _ in range(warmup):
        b.protect()
        b.restore()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()

    def timed(fp, fr):
        ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        for k in range(steps):
            ev[k][0].record(stream)
            fp()
            ev[k][1].record(stream)
            fr()
            ev[k][2].record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
        tp = [ev[k][0].elapsed_time(ev[k][1]) for k in range(steps)]
        tr = [ev[k][1].elapsed_time(ev[k][2]) for k in range(steps)]
        return wall, tp, tr

    wall_e, tp_e, tr_e = timed(b.protect, b.restore)
    # each direction captured as a HIP graph of its one launch, replayed
    side = torch.cuda.Stream()
    side.wait_stream(stream)
    gp, gr = torch.cuda.CUDAGraph(), torch.cuda.CUDAGraph()
    with torch.cuda.stream(side):
        with torch.cuda.graph(gp, stream=side):
            b.protect(stream=side)
        with torch.cuda.graph(gr, stream=side):
            b.restore(stream=side)
    stream.wait_stream(side)
    torch.cuda.synchronize()
    gp.replay()
    gr.replay()
    torch.cuda.synchronize()
    ok &= all(bool(torch.equal(o, x)) for o, x in zip(b.outs, xs))
    wall, tp, tr = timed(gp.replay, gr.replay)
    torch.cuda.synchronize()
    ok &= all(bool(torch.equal(o, x)) for o, x in zip(b.outs, xs))
    alg = sum(s["n"] + 2 * (-(-s["n"] // s["width"])) * s["width"] for s in specs)  # per direction
    # counter traffic is recorded for the default tile heights of the full
    # batch (tuned heights vary with the tuner's timings)
    traffic = (stored_traffic("batch_default_tiles", BATCH_PATH_SOURCES)
               if args.no_tune and args.count == 2048 and not args.batch_subset else None)
    avg_p, avg_r = sum(tp) / steps, sum(tr) / steps
    dom = "fwd_batch_kernel" if avg_p >= avg_r else "inv_batch_kernel"
    dom_ms = max(avg_p, avg_r)
    result = {
        "metric": "batched protect+restore GB/s on 1 MI355X, bit-exact",
        "value": round(total * steps / wall / 1e9, 2), "unit": "GB/s", "n_gpus": 1, "steps": steps,
        "warmup": warmup, "ms_per_step": round(wall / steps * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int16/int32", "data": "synthetic",
        "config": {"workload": f"{len(specs)} uneven buffers ({total / 1e9:.2f} GB, mixed content), "
                               "1-4 levels, one persistent launch per direction replayed as HIP graphs, "
                               + ("default tile heights" if args.no_tune else
                                  "tile heights tuned per (width, levels) class"),
                   "buffers": len(specs), "bytes": total, "classes": len(tune),
                   "subset": args.batch_subset or None},
        "bit_exact": ok,
        "latency_ms": {"protect_p50": round(percentile(tp, 50), 3),
                       "restore_p50": round(percentile(tr, 50), 3)},
        "eager": {"value": round(total * steps / wall_e / 1e9, 2),
                  "protect_p50_ms": round(percentile(tp_e, 50), 3),
                  "restore_p50_ms": round(percentile(tr_e, 50), 3)},
        "roofline": {"bound": "hbm", "achieved": round(alg / (dom_ms * 1e-3) / 1e9, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(alg / (dom_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "traffic": traffic.get(dom) if traffic else None,
                     "kernel": dom, "bytes_per_launch": alg, "avg_launch_ms": round(dom_ms, 3)},
        "cpu_baseline": None,
    }
    print(json.dumps(result), flush=True)


def _launch_stats(log):
    """p50 / p99 / max of launch -> retire (host clock) over the server's
    launches; for the slowest: its planning time, its kernels' device time,
    requests and bytes."""
    if not log:
        return None
    d = [(r - l) * 1e3 for _, l, r, _, _, _ in log]
    g = [gm for _, _, _, gm, _, _ in log]
    worst = max(range(len(log)), key=lambda i: d[i])
    p0, l0, _, gm, nreq, nb = log[worst]
    return {"p50": round(percentile(d, 50), 3), "p99": round(percentile(d, 99), 3),
            "max": round(d[worst], 3), "max_at_s": round(l0, 3),
            "max_planning_ms": round((l0 - p0) * 1e3, 3), "max_device_ms": round(gm, 3),
            "max_requests": nreq, "max_bytes": nb,
            "device_ms_p50": round(percentile(g, 50), 3), "device_ms_max": round(max(g), 3),
            "planning_ms_max": round(max((l - p) * 1e3 for p, l, _, _, _, _ in log), 3)}


def run_serve(args):
    """Serving workload: Poisson arrivals (seed 5) at --rate per second for
    --duration seconds; sizes log-uniform in 16 KiB .. 256 MiB drawn from a
    pool of 256 device-resident buffers (random bytes from a seeded device
    generator, the default width, 1..4 levels); half the requests protect a
    pool buffer, half restore its pre-protected fragments."""
    import math

    import numpy as np
    import torch

    import paper_1803_04880_amd as dwtfrag
    import synth
    from paper_1803_04880_amd import serve

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(5)
    gen = torch.Generator(device=dev)
    gen.manual_seed(5)
    pool = []
    for i in range(256):
        n = int(math.exp(rng.uniform(math.log(16 << 10), math.log(256 << 20))))
        lv = int(rng.integers(1, 5))
        w = synth.default_width(n)
        x = torch.randint(0, 256, (n,), dtype=torch.uint8, device=dev, generator=gen)
        key, nonce = rng.bytes(16), rng.bytes(16)
        p, q = dwtfrag.protect(x, w, lv, key, nonce)
        pool.append((n, w, lv, key, nonce, x, p, q))
    torch.cuda.synchronize()
    log(f"pool of {len(pool)} buffers, {sum(e[0] for e in pool) / 1e9:.2f} GB")
    reqs, t = [], 0.0
    while True:
        t += float(rng.exponential(1.0 / args.rate))
        if t >= args.duration:
            break
        n, w, lv, key, nonce, x, p, q = pool[int(rng.integers(0, len(pool)))]
        op = "protect" if rng.random() < 0.5 else "restore"
        reqs.append(serve.Request(len(reqs), op, t, n, w, lv, key, nonce,
                                  x=x if op == "protect" else None,
                                  priv=p if op == "restore" else None,
                                  pub=q if op == "restore" else None))
    srv = serve.Server(budget_bytes=64 << 30, max_batch=512)
    # results are released as requests complete, except a sample that is
    # kept and checked after the run against the lone calls that made the
    # pool (a check inside the loop would synchronise the device under it)
    stride = max(1, len(reqs) // 50)
    kept = []

    def on_complete(r):
        if r.rid % stride == 0:
            kept.append((r, r.out_priv, r.out_pub, r.out))
        r.out_priv = r.out_pub = r.out = None

    srv.on_complete = on_complete
    srv.warmup()
    wall = srv.run(reqs)
    torch.cuda.synchronize()
    checks = []
    for r, p, q, o in kept:
        e = next(e for e in pool if e[3] == r.key and e[4] == r.nonce)
        if r.op == "protect":
            checks.append(bool(torch.equal(p, e[6]) and torch.equal(q, e[7])))
        else:
            checks.append(bool(torch.equal(o, e[5])))
    del kept
    lat = [(r.done - r.arrival) * 1e3 for r in reqs]
    total = sum(r.n for r in reqs)
    ok = bool(checks) and all(checks)
    result = {
        "metric": "serving: arrival-to-completion latency and sustained GB/s on 1 MI355X",
        "value": round(total / wall / 1e9, 2), "unit": "GB/s", "n_gpus": 1, "steps": len(reqs),
        "warmup": 0, "ms_per_step": round(wall / max(len(reqs), 1) * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int16/int32",
        "data": "synthetic",
        "config": {"workload": f"Poisson {args.rate:.0f}/s for {args.duration:.0f}s, sizes 16 KiB-256 MiB "
                               "log-uniform (pool of 256), 50/50 protect/restore, 64 GB budget",
                   "requests": len(reqs), "offered_gbps": round(total / args.duration / 1e9, 2)},
        "bit_exact_sample": ok,
        "latency_ms": {"p50": round(percentile(lat, 50), 3), "p99": round(percentile(lat, 99), 3),
                       "max": round(max(lat), 3)},
        "launches": srv.batches_launched, "wall_s": round(wall, 3),
        "launch_to_retire_ms": _launch_stats(srv.launch_log),
        "host_loop_max_ms": round(srv.max_gap[0] * 1e3, 3), "host_loop_max_at_s": round(srv.max_gap[1], 3),
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(result), flush=True)


def _entropy_bits(pub):
    """Zeroth-order entropy (bits per coefficient) of int16 coefficients."""
    import torch
    counts = torch.bincount((pub.to(torch.int64) + 32768).reshape(-1), minlength=65536)
    p = counts[counts > 0].double() / pub.numel()
    return float(-(p * torch.log2(p)).sum())


def run_learned(args):
    """Learned-predictor workload: 64 smooth 4096 x 4096 images (1 GiB), 3
    levels.  Trains the network on the GPU, then times learned and plain
    protect + restore over all images with the oracle-trained network of
    tests/golden (a fixed input, so the fragments can be checked against the
    oracle's digest).  Learned calls are one per image, spread over four
    streams; the plain path runs as one batch."""
    import multiprocessing

    import torch

    import paper_1803_04880_amd as dwtfrag
    import synth
    from paper_1803_04880_amd import learned as GL

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    steps = args.steps if args.steps != 50 else 10
    warmup = args.warmup if args.warmup != 5 else 2
    nimg = args.images or synth.LEARNED_IMAGES
    if args.learned_streams < 1:
        raise SystemExit("--learned-streams must be at least 1")
    W, L, n = 4096, 3, 4096 * 4096
    t0 = time.time()
    if nimg <= 8:   # few images (profiler runs): no worker processes
        imgs = [synth.learned_image(i) for i in range(nimg)]
    else:
        with _closing_pool(8) as pool:
            imgs = pool.map(synth.learned_image, range(nimg))
    log(f"{nimg} images of 4096x4096 generated in {time.time() - t0:.1f}s")
    xs = [torch.from_numpy(im).to(dev) for im in imgs]
    del imgs
    kn = [synth.learned_key_nonce(i) for i in range(nimg)]
    with open(os.path.join(ROOT, "tests", "golden", "predictor_smooth.json")) as f:
        rec = json.load(f)
    gold_net = GL.Predictor.from_arrays(rec["w1"], rec["b1"], rec["w2"], rec["b2"], rec["shift"])
    g = dwtfrag.geometry(n, W, L)
    privs = [torch.empty(g["priv_bytes"], dtype=torch.uint8, device=dev) for _ in range(nimg)]
    pubs = [torch.empty(g["pub_bytes"] // 2, dtype=torch.int16, device=dev) for _ in range(nimg)]
    outs = [torch.empty(n, dtype=torch.uint8, device=dev) for _ in range(nimg)]
    # The images are independent calls: they go round-robin to a few streams
    # (--learned-streams, sixteen by default; all at the default priority),
    # each with its own workspace, forked from and
    # joined back into the current stream, so that one image's small levels
    # overlap another's large one.  Image i's restore runs on the stream of
    # its protect.
    main = torch.cuda.current_stream()
    n_streams = args.learned_streams
    side = [torch.cuda.Stream(device=dev) for _ in range(n_streams)]
    wss = [GL.workspace(n, W, L, dev) for _ in range(n_streams)]

    def fan_out(call):
        fork = torch.cuda.Event()
        fork.record(main)
        for st in side:
            st.wait_event(fork)
        for i in range(nimg):
            call(i, side[i % n_streams], wss[i % n_streams])
        for st in side:
            join = torch.cuda.Event()
            join.record(st)
            main.wait_event(join)

    def protect_all(net):
        fan_out(lambda i, st, ws: GL.protect(xs[i], W, L, kn[i][0], kn[i][1], net, priv=privs[i],
                                             pub=pubs[i], ws=ws, stream=st))

    def restore_all(net):
        fan_out(lambda i, st, ws: GL.restore(privs[i], pubs[i], n, W, L, kn[i][0], kn[i][1], net,
                                             out=outs[i], ws=ws, stream=st))

    from paper_1803_04880_amd import batch as B
    plain = B.Batch(xs, [W] * nimg, [L] * nimg, [k for k, _ in kn], [v for _, v in kn],
                    privs=privs, pubs=pubs, outs=outs)

    def plain_protect_all():
        plain.protect()

    def plain_restore_all():
        plain.restore()

    # parity: image 0 against the oracle's digest, every image round trips
    protect_all(gold_net)
    restore_all(gold_net)
    torch.cuda.synchronize()
    with open(os.path.join(ROOT, "tests", "golden", "oracle_digests.json")) as f:
        gold = json.load(f)["learned"]
    bit_exact = hashlib.sha256(privs[0].cpu().numpy().tobytes()).hexdigest() == gold["priv_sha256"]
    bit_exact &= hashlib.sha256(pubs[0].cpu().numpy().tobytes()).hexdigest() == gold["pub_sha256"]
    bit_exact &= all(bool(torch.equal(outs[i], xs[i])) for i in range(nimg))
    log(f"parity vs oracle (image 0) and round trips: {'bit-exact' if bit_exact else 'MISMATCH'}")
    ent_learned = sum(_entropy_bits(p) for p in pubs) / nimg

    # training on the GPU: pairs of the 512x512 image and of rows 0..256 of
    # the 256 MiB workload, the recipe of the stored network
    small = synth.config_small()["buf"]
    big = synth.config_large()
    part = big["buf"][:256 * big["width"]].copy()
    del big
    c1, t1 = GL.training_pairs(torch.from_numpy(small).to(dev), 512, 3)
    c2, t2 = GL.training_pairs(torch.from_numpy(part).to(dev), 32768, 3)
    ctx, tgt = torch.cat([c1, c2]), torch.cat([t1, t2])
    trainer = GL.Trainer(synth.mlp_init(161, 4), dev)
    nb = max(tgt.numel() // 65536, 1)
    torch.cuda.synchronize()
    tt0 = time.perf_counter()
    for s_ in range(300):
        trainer.step(ctx, tgt, 0.01, s_ % nb, nb)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - tt0
    st = trainer.read()
    gpu_net = GL.Predictor.from_buffer_copy(bytes(st.net))
    # entropy with the GPU-trained network, round trip checked
    protect_all(gpu_net)
    torch.cuda.synchronize()
    ent_gpu = sum(_entropy_bits(p) for p in pubs) / nimg
    restore_all(gpu_net)
    torch.cuda.synchronize()
    bit_exact &= all(bool(torch.equal(outs[i], xs[i])) for i in range(nimg))

    stream = torch.cuda.current_stream()

    def timed(fp, fr):
        for _ in range(warmup):
            fp()
            fr()
        torch.cuda.synchronize()
        ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
        w0 = time.perf_counter()
        for k in range(steps):
            ev[k][0].record(stream)
            fp()
            ev[k][1].record(stream)
            fr()
            ev[k][2].record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
        tp = [ev[k][0].elapsed_time(ev[k][1]) * 1e3 for k in range(steps)]
        tr = [ev[k][1].elapsed_time(ev[k][2]) * 1e3 for k in range(steps)]
        return wall, tp, tr

    plain_protect_all()
    torch.cuda.synchronize()
    ent_plain = sum(_entropy_bits(p) for p in pubs) / nimg
    wall_p, tp_p, tr_p = timed(plain_protect_all, plain_restore_all)
    wall, tp, tr = timed(lambda: protect_all(gold_net), lambda: restore_all(gold_net))
    total = n * nimg
    value = total * steps / wall / 1e9
    # Roofline of the learned passes: int8 multiply-accumulates of the network
    # (8x16 + 16 per predicted sample) over all predict steps of both
    # directions, as operations (2 per MAC) against the dense int8 matrix-core
    # peak (5.0 POP/s), with the VALU v_dot4 rate (4 MACs per lane per cycle)
    # and the HBM fraction of the algorithmic bytes (3 per element each way)
    # beside it
    _, pairs = GL.learned_geometry(n, W, L)
    macs = 2 * pairs * 144 * nimg
    pair_us = (sum(tp) + sum(tr)) / steps
    achieved = macs / (pair_us * 1e-6) / 1e12
    peak = 256 * 64 * 2.4e9 * 4 / 1e12
    result = {
        "metric": "learned-predictor protect+restore GB/s on 1 MI355X, bit-exact",
        "value": round(value, 2), "unit": "GB/s", "n_gpus": 1, "steps": steps, "warmup": warmup,
        "ms_per_step": round(wall / steps * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int8/int32", "data": "synthetic",
        "config": {"workload": f"{nimg} smooth 4096x4096 images ({total / 2**30:.2f} GiB), 3 levels, "
                               "context network trained by the oracle", "images": nimg,
                   "width": W, "levels": L, "streams": n_streams},
        "bit_exact": bool(bit_exact),
        "latency_us": {"protect_all_p50": round(percentile(tp, 50), 1),
                       "restore_all_p50": round(percentile(tr, 50), 1)},
        "plain_53_batched": {"value": round(total * steps / wall_p / 1e9, 2), "unit": "GB/s",
                     "protect_all_p50_us": round(percentile(tp_p, 50), 1),
                     "restore_all_p50_us": round(percentile(tr_p, 50), 1)},
        "entropy_bits": {"plain_53": round(ent_plain, 4), "learned_oracle_net": round(ent_learned, 4),
                         "learned_gpu_trained": round(ent_gpu, 4)},
        "training": {"pairs": int(tgt.numel()), "steps": 300, "seconds": round(train_s, 3),
                     "final_batch_loss": round(float(st.loss), 4),
                     "oracle_loss_end_full_set": rec["loss_end"]},
        "roofline": {"bound": "mfma", "achieved": round(2 * achieved, 3), "peak": 5000.0,
                     "unit": "T int8 ops/s (multiply and add)",
                     "frac": round(2 * achieved / 5000.0, 5),
                     "traffic": None, "kernel": "all learned passes of protect+restore",
                     "macs_per_step": macs,
                     "valu_dot4_frac": round(achieved / peak, 4),
                     "hbm_frac": round(2 * (n + 2 * n) * nimg / (pair_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)},
        "cpu_baseline": None,
    }
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
