"""GPU parity of batched protect / restore (persistent tile-queue launches),
their HIP-graph replay, and the launch-shape autotuner.

Every item of a batch must produce exactly the fragments of the oracle on that
item alone (integer work: byte for byte), and restore must return the input.
"""
import numpy as np
import pytest

from conftest import gpu_available

pytestmark = pytest.mark.gpu

if not gpu_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import torch  # noqa: E402

import paper_1803_04880_amd as dwtfrag  # noqa: E402
import synth  # noqa: E402
from oracle import fragment  # noqa: E402
from paper_1803_04880_amd import batch as B  # noqa: E402

DEV = "cuda:0"


def _say(msg):
    print(msg, flush=True)


def _specs(count, seed, lo=1, hi=200000):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(np.exp(rng.uniform(np.log(lo), np.log(hi))))
        lv = int(rng.integers(1, 5))
        w = synth.default_width(n)
        out.append(dict(n=n, width=w, levels=lv, buf=rng.integers(0, 256, n, dtype=np.uint8),
                        key=rng.bytes(16), nonce=rng.bytes(16)))
    return out


def _make_batch(specs, tune=None):
    xs = [torch.from_numpy(s["buf"]).to(DEV) for s in specs]
    return B.Batch(xs, [s["width"] for s in specs], [s["levels"] for s in specs],
                   [s["key"] for s in specs], [s["nonce"] for s in specs], tune=tune)


def _check_against_oracle(b, specs):
    for i, s in enumerate(specs):
        opriv, opub = fragment.protect(s["buf"], s["width"], s["levels"], s["key"], s["nonce"])
        assert b.privs[i].cpu().numpy().tobytes() == opriv, f"item {i} priv"
        assert b.pubs[i].cpu().numpy().tobytes() == opub, f"item {i} pub"


@pytest.mark.parametrize("count,seed", [(1, 1), (7, 2), (64, 3), (300, 4)])
def test_batch_matches_oracle_and_roundtrips(count, seed):
    specs = _specs(count, seed)
    _say(f"batch count={count} seed={seed} bytes={sum(s['n'] for s in specs)}")
    b = _make_batch(specs)
    b.protect()
    torch.cuda.synchronize()
    _check_against_oracle(b, specs)
    b.restore()
    torch.cuda.synchronize()
    for i, s in enumerate(specs):
        assert b.outs[i].cpu().numpy().tobytes() == s["buf"].tobytes(), f"item {i} restore"
    b.close()


_CFG3 = {}


def _cfg3_specs():
    """Items of the uneven-batch workload's shapes: sizes from 4 MiB to just
    over 16 MiB, so the default width is 4096 (several column windows per
    item), levels 1..4 (four levels run 16-column tiles), content from the
    workload's generators (smooth / markov / uniform thirds), ragged tails."""
    sizes = [(16 << 20) + 12345, (9 << 20) - 777, (6 << 20) + 1, (4 << 20) + 4097,
             (5 << 20) + 3, (7 << 20) - 5]
    levels = [4, 3, 2, 1, 3, 1]
    kinds = ["smooth", "markov", "uniform", "smooth", "markov", "uniform"]
    if "specs" in _CFG3:
        return _CFG3["specs"]
    rng = np.random.default_rng(31)
    specs = []
    for i, (n, lv, kind) in enumerate(zip(sizes, levels, kinds)):
        spec = dict(seed=7000 + i, n=n, kind=kind, levels=lv, width=synth.default_width(n),
                    nonce=rng.bytes(16))
        spec["buf"] = synth.batch_buffer(spec)
        spec["key"] = rng.bytes(16)
        # the oracle's fragments, computed once for both parametrisations
        spec["oracle"] = fragment.protect(spec["buf"], spec["width"], lv, spec["key"], spec["nonce"])
        specs.append(spec)
    _CFG3["specs"] = specs
    return specs


def _first_diff(a, b):
    a = np.frombuffer(a, np.uint8)
    b = np.frombuffer(b, np.uint8)
    if a.size != b.size:
        return f"sizes {a.size} != {b.size}"
    idx = np.flatnonzero(a != b)
    return "equal" if idx.size == 0 else f"{idx.size} bytes differ, first at byte {idx[0]}"


@pytest.mark.parametrize("tuned", [False, True])
def test_batch_workload_shapes_match_oracle(tuned):
    """Batch items at the uneven-batch workload's shapes (width 4096,
    multi-window drains, 8- and 16-column tiles, tuned tile heights) against
    the oracle, element by element, and restored exactly."""
    specs = _cfg3_specs()
    assert all(s["width"] == 4096 for s in specs)
    tune = None
    if tuned:   # 16-column tiles for the 1..3-level classes, other heights
        tune = {(4096, 1): (64, 16), (4096, 2): (256, 16), (4096, 3): (256, 8), (4096, 4): (64, 16)}
    _say(f"workload-shaped batch tuned={tuned}: " +
         ", ".join(f"n={s['n']} L={s['levels']} {s['kind']}" for s in specs))
    b = _make_batch(specs, tune=tune)
    b.protect()
    b.restore()
    torch.cuda.synchronize()
    for i, s in enumerate(specs):
        opriv, opub = s["oracle"]
        gpriv = b.privs[i].cpu().numpy().tobytes()
        gpub = b.pubs[i].cpu().numpy().tobytes()
        assert gpriv == opriv, f"item {i} priv: {_first_diff(gpriv, opriv)}"
        assert gpub == opub, f"item {i} pub: {_first_diff(gpub, opub)}"
        assert np.array_equal(b.outs[i].cpu().numpy(), s["buf"]), f"item {i} restore"
    b.close()


def test_batch_degenerate_items():
    rng = np.random.default_rng(9)
    specs = []
    for n, w, lv in [(1, 1, 1), (2, 1, 4), (3, 2, 2), (1, 1, 4), (17, 17, 3), (4096, 4096, 1)]:
        specs.append(dict(n=n, width=w, levels=lv, buf=rng.integers(0, 256, n, dtype=np.uint8),
                          key=rng.bytes(16), nonce=rng.bytes(16)))
    _say("batch degenerate items")
    b = _make_batch(specs)
    b.protect()
    b.restore()
    torch.cuda.synchronize()
    _check_against_oracle(b, specs)
    for i, s in enumerate(specs):
        assert b.outs[i].cpu().numpy().tobytes() == s["buf"].tobytes()


def test_batch_rejects_bad_items():
    x = torch.zeros(100, dtype=torch.uint8, device=DEV)
    with pytest.raises(Exception):
        B.Batch([x], [10], [5], [bytes(16)], [bytes(16)])    # more than one fused stage
    with pytest.raises(Exception):
        B.Batch([x[1:]], [9], [1], [bytes(16)], [bytes(16)])  # misaligned input


def test_batch_graph_replays_match_eager():
    """Capture protect + restore of a batch in a HIP graph; replay it several
    times with eager work and synchronisation in between; every replay gives
    the eager fragments and outputs."""
    specs = _specs(40, 11)
    b = _make_batch(specs)
    b.protect()
    b.restore()
    torch.cuda.synchronize()
    want_priv = [p.clone() for p in b.privs]
    want_pub = [q.clone() for q in b.pubs]
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        for p, q, o in zip(b.privs, b.pubs, b.outs):
            p.zero_()
            q.zero_()
            o.zero_()
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=s):
            b.protect(stream=s)
            b.restore(stream=s)
    torch.cuda.synchronize()
    for rep in range(4):
        for p, q, o in zip(b.privs, b.pubs, b.outs):   # eager work between replays
            p.fill_(7)
            q.fill_(-3)
            o.fill_(1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        _say(f"graph replay {rep}")
        for i, spec in enumerate(specs):
            assert torch.equal(b.privs[i], want_priv[i]), f"replay {rep} item {i} priv"
            assert torch.equal(b.pubs[i], want_pub[i]), f"replay {rep} item {i} pub"
            assert b.outs[i].cpu().numpy().tobytes() == spec["buf"].tobytes(), f"replay {rep} item {i}"


def test_autotune_and_tuned_batch():
    specs = _specs(24, 12, lo=20000, hi=400000)
    classes = {}
    for s in specs:
        classes.setdefault((s["width"], s["levels"]), s)
    tune = {}
    for key, s in classes.items():
        ln, us = B.autotune(torch.from_numpy(s["buf"]).to(DEV), s["width"], s["levels"], trials=2)
        assert ln.lane_cols in (8, 16) and us > 0
        tune[key] = ln
    _say(f"autotuned {len(tune)} classes")
    b = _make_batch(specs, tune=tune)
    b.protect()
    b.restore()
    torch.cuda.synchronize()
    _check_against_oracle(b, specs)
    for i, s in enumerate(specs):
        assert b.outs[i].cpu().numpy().tobytes() == s["buf"].tobytes()


def test_serving_loop_results_equal_oracle_and_lone_calls():
    """Requests arriving over time, served by continuous batching, give the
    oracle's bytes: every served protect equals the oracle's fragments of its
    buffer, every served restore equals the oracle's restore of the oracle's
    fragments; the lone GPU calls that made the restore inputs agree too."""
    from paper_1803_04880_amd import serve
    rng = np.random.default_rng(21)
    reqs, lone = [], []
    pool = _specs(12, 22, lo=1000, hi=300000)
    frag, ofrag = [], []
    for s in pool:   # fragments for restore requests, made by lone calls
        x = torch.from_numpy(s["buf"]).to(DEV)
        p, q = dwtfrag.protect(x, s["width"], s["levels"], s["key"], s["nonce"])
        frag.append((x, p, q))
        opriv, opub = fragment.protect(s["buf"], s["width"], s["levels"], s["key"], s["nonce"])
        oback = fragment.restore(opriv, opub, s["n"], s["width"], s["levels"], s["key"], s["nonce"])
        ofrag.append((opriv, opub, oback))
    torch.cuda.synchronize()
    for (x, p, q), (opriv, opub, _) in zip(frag, ofrag):
        assert p.cpu().numpy().tobytes() == opriv and q.cpu().numpy().tobytes() == opub
    t = 0.0
    for rid in range(60):
        t += float(rng.exponential(0.002))
        k = int(rng.integers(0, len(pool)))
        s, (x, p, q) = pool[k], frag[k]
        op = "protect" if rng.random() < 0.5 else "restore"
        r = serve.Request(rid, op, t, s["n"], s["width"], s["levels"], s["key"], s["nonce"],
                          x=x if op == "protect" else None, priv=p if op == "restore" else None,
                          pub=q if op == "restore" else None)
        reqs.append(r)
        lone.append(k)
    srv = serve.Server(budget_bytes=1 << 28, max_batch=16)
    wall = srv.run(reqs)
    torch.cuda.synchronize()
    _say(f"served {len(reqs)} requests in {wall:.3f}s, {srv.batches_launched} launches")
    assert srv.batches_launched > 1   # requests were admitted over several batches
    for r, k in zip(reqs, lone):
        x, p, q = frag[k]
        opriv, opub, oback = ofrag[k]
        assert r.done is not None and r.done >= r.arrival
        if r.op == "protect":
            assert r.out_priv.cpu().numpy().tobytes() == opriv, f"request {r.rid} priv vs oracle"
            assert r.out_pub.cpu().numpy().tobytes() == opub, f"request {r.rid} pub vs oracle"
            assert torch.equal(r.out_priv, p) and torch.equal(r.out_pub, q), f"request {r.rid}"
        else:
            assert r.out.cpu().numpy().tobytes() == oback, f"request {r.rid} restore vs oracle"
            assert torch.equal(r.out, x), f"request {r.rid}"


def test_batch_class_tuner_and_tuned_batch():
    specs = _specs(30, 13, lo=5000, hi=300000)
    xs = [torch.from_numpy(s["buf"]).to(DEV) for s in specs]
    tune = B.tune_classes(xs, [s["width"] for s in specs], [s["levels"] for s in specs], trials=1)
    assert set(tune) == {(s["width"], s["levels"]) for s in specs}
    for (w, lv), ln in tune.items():
        assert ln.lane_cols in (8, 16) and ln.seg_rows in (64, 128, 256)
        assert lv < 4 or ln.lane_cols == 16
    _say(f"class tuner: {len(tune)} classes")
    b = _make_batch(specs, tune=tune)
    b.protect()
    b.restore()
    torch.cuda.synchronize()
    _check_against_oracle(b, specs)
    for i, s in enumerate(specs):
        assert b.outs[i].cpu().numpy().tobytes() == s["buf"].tobytes()
