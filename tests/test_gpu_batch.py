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


def test_serving_loop_results_equal_lone_calls():
    """Requests arriving over time, served by continuous batching, give the
    same bytes as each request processed alone."""
    from paper_1803_04880_amd import serve
    rng = np.random.default_rng(21)
    reqs, lone = [], []
    pool = _specs(12, 22, lo=1000, hi=300000)
    frag = []
    for s in pool:   # fragments for restore requests, made by lone calls
        x = torch.from_numpy(s["buf"]).to(DEV)
        p, q = dwtfrag.protect(x, s["width"], s["levels"], s["key"], s["nonce"])
        frag.append((x, p, q))
    torch.cuda.synchronize()
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
    for r, k in zip(reqs, lone):
        x, p, q = frag[k]
        assert r.done is not None and r.done >= r.arrival
        if r.op == "protect":
            assert torch.equal(r.out_priv, p) and torch.equal(r.out_pub, q), f"request {r.rid}"
        else:
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
