"""GPU parity of the learned-predictor path and its trainer against the oracle.

Protect / restore / training pairs are integer work: compared byte for byte.
The trainer's gradient is exact integer sums scaled once, so it must equal
the oracle's fp64 gradient to float32 rounding (relative 1e-6); the Adam step
runs in float32 (relative 1e-5 of the step size); the quantisation is exact
(power-of-two scales) and compared bit for bit.
"""
import numpy as np
import pytest

from conftest import gpu_available

pytestmark = pytest.mark.gpu

if not gpu_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import torch  # noqa: E402

import synth  # noqa: E402
from oracle import fragment  # noqa: E402
from oracle import learned as OL  # noqa: E402
from paper_1803_04880_amd import learned as GL  # noqa: E402

DEV = "cuda:0"


def _say(msg):
    print(msg, flush=True)


def _nets(seed):
    raw = synth.random_predictor(seed)
    return OL.Predictor(*raw), GL.Predictor.from_arrays(*raw)


def _protect(buf, width, levels, key, nonce, gnet):
    x = torch.from_numpy(np.ascontiguousarray(buf)).to(DEV)
    priv, pub = GL.protect(x, width, levels, key, nonce, gnet)
    torch.cuda.synchronize()
    return priv.cpu().numpy().tobytes(), pub.cpu().numpy().tobytes()


def _restore(priv, pub, n, width, levels, key, nonce, gnet):
    p = torch.from_numpy(np.frombuffer(priv, np.uint8).copy()).to(DEV)
    q = torch.from_numpy(np.frombuffer(pub, "<i2").copy()).to(DEV)
    out = GL.restore(p, q, n, width, levels, key, nonce, gnet)
    torch.cuda.synchronize()
    return out.cpu().numpy().tobytes()


# (n, width, levels): degenerate and ragged shapes; levels spanning several
# 64 x 128 tiles of the protect / restore kernels in either direction, with
# ragged last tiles and odd dimensions at every level; rows spanning several
# 2048-sample segments of the training-pair capture.
CASES = [
    (1, 1, 1), (2, 1, 2), (2, 2, 1), (5, 2, 3), (9, 3, 2), (100, 7, 3), (1000, 1, 3),
    (4097, 64, 3), (12345, 97, 2), (200 * 130 - 17, 130, 3), (70 * 2049, 2049, 1),
    (3 * 4500 + 11, 4500, 3), (262144, 512, 1), (300000, 1031, 2), (333 * 261 - 5, 261, 3),
    (129 * 257, 257, 2), (3 * 20000 + 7, 20000, 2), (5000 * 4 + 1, 4, 3), (257 * 516, 516, 3),
]


@pytest.mark.parametrize("n,width,levels", CASES)
def test_learned_protect_matches_oracle_and_roundtrips(n, width, levels):
    rng = np.random.default_rng(n * 17 + width * 3 + levels)
    buf = rng.integers(0, 256, n, dtype=np.uint8)
    key, nonce = rng.bytes(16), rng.bytes(16)
    onet, gnet = _nets(n + levels)
    _say(f"learned case n={n} width={width} levels={levels}")
    priv, pub = _protect(buf, width, levels, key, nonce, gnet)
    opriv, opub = OL.protect(buf, width, levels, key, nonce, onet)
    assert priv == opriv, "private fragment differs"
    assert pub == opub, "public fragment differs"
    assert _restore(priv, pub, n, width, levels, key, nonce, gnet) == buf.tobytes()


# The last two take the restore's vector tile loads (even band widths at
# every level), with int32 intermediate LL bands between levels.
@pytest.mark.parametrize("n,width,levels", [(9, 3, 2), (12345, 97, 3), (200 * 130 - 17, 130, 2),
                                            (64 * 256, 256, 3), (300 * 512 - 100, 512, 2)])
def test_learned_restore_of_arbitrary_fragments(n, width, levels):
    rng = np.random.default_rng(3 * n + levels)
    g = fragment.geometry(n, width, levels)
    priv = rng.integers(0, 256, g["priv_bytes"], dtype=np.uint8).tobytes()
    pub = rng.integers(-32768, 32768, g["pub_bytes"] // 2).astype("<i2").tobytes()
    key, nonce = rng.bytes(16), rng.bytes(16)
    onet, gnet = _nets(7 * n)
    _say(f"learned restore n={n} width={width} levels={levels}")
    assert _restore(priv, pub, n, width, levels, key, nonce, gnet) == \
        OL.restore(priv, pub, n, width, levels, key, nonce, onet)


def test_zero_network_equals_plain_fragments():
    rng = np.random.default_rng(44)
    buf = rng.integers(0, 256, 50000, dtype=np.uint8)
    key, nonce = rng.bytes(16), rng.bytes(16)
    zero = GL.Predictor()
    assert _protect(buf, 250, 3, key, nonce, zero) == fragment.protect(buf, 250, 3, key, nonce)


def test_saturating_network_edges():
    """Huge biases: every correction clamps at +-255 and every hidden unit
    sits at the bias limit."""
    rng = np.random.default_rng(45)
    buf = np.where(rng.random(40 * 70) < 0.5, 0, 255).astype(np.uint8)
    key, nonce = rng.bytes(16), rng.bytes(16)
    for sign in (1, -1):
        w1 = np.full((16, 8), 127 * sign, np.int8)
        b1 = np.full(16, 65536, np.int32)
        w2 = np.full(16, 127 * sign, np.int8)
        raw = (w1, b1, w2, sign * (1 << 26), 0)
        onet, gnet = OL.Predictor(*raw), GL.Predictor.from_arrays(*raw)
        got = _protect(buf, 70, 3, key, nonce, gnet)
        assert got == OL.protect(buf, 70, 3, key, nonce, onet)
        assert _restore(*got, buf.size, 70, 3, key, nonce, gnet) == buf.tobytes()


def test_rejects_out_of_range_network():
    x = torch.zeros(64, dtype=torch.uint8, device=DEV)
    bad = GL.Predictor()
    bad.shift = 31
    with pytest.raises(Exception):
        GL.protect(x, 8, 1, bytes(16), bytes(16), bad)
    bad = GL.Predictor()
    bad.b1[3] = (1 << 16) + 1
    with pytest.raises(Exception):
        GL.protect(x, 8, 1, bytes(16), bytes(16), bad)
    with pytest.raises(Exception):
        GL.protect(x, 8, 4, bytes(16), bytes(16), GL.Predictor())


@pytest.mark.parametrize("h,w,levels", [(1, 1, 1), (1, 9, 2), (9, 1, 2), (33, 70, 3),
                                        (130, 2100, 2), (512, 512, 1)])
def test_training_pairs_match_oracle(h, w, levels):
    img = synth.smooth(h, w, 50 + h)
    ctx, tgt = GL.training_pairs(torch.from_numpy(img.reshape(-1).copy()).to(DEV), w, levels)
    octx, otgt = OL.training_pairs(img.astype(np.int64), levels)
    _say(f"pairs h={h} w={w} levels={levels}: {len(otgt)}")
    assert tgt.numel() == len(otgt)
    assert np.array_equal(tgt.cpu().numpy(), otgt)
    assert np.array_equal(ctx.cpu().numpy().astype(np.int64), octx)


def _oracle_pairs():
    img = synth.smooth(160, 200, 61)
    return img, OL.training_pairs(img.astype(np.int64), 2)


def test_trainer_init_quantisation_is_exact():
    theta0 = synth.mlp_init(OL.N_PARAMS, 70)
    tr = GL.Trainer(theta0, DEV)
    st = tr.read()
    assert np.array_equal(np.frombuffer(bytes(st.theta), np.float32), theta0)
    want = OL.quantize(theta0)
    assert bytes(st.net) == want.to_bytes()
    for scale in (1e-4, 3.0, 300.0):        # other exponent ranges, incl. negative k
        th = (theta0 * scale).astype(np.float32)
        assert bytes(GL.Trainer(th, DEV).read().net) == OL.quantize(th).to_bytes()


@pytest.mark.parametrize("batch,n_batches", [(0, 1), (2, 5)])
def test_trainer_step_matches_oracle(batch, n_batches):
    _, (octx, otgt) = _oracle_pairs()
    ctx = torch.from_numpy(octx.astype(np.int8)).to(DEV)
    tgt = torch.from_numpy(otgt.astype(np.int32)).to(DEV)
    theta0 = synth.mlp_init(OL.N_PARAMS, 71)
    tr = GL.Trainer(theta0, DEV)
    lr = 0.01
    tr.step(ctx, tgt, lr, batch, n_batches)
    st = tr.read()
    loss, g = OL.loss_grad(OL.fake_quant(theta0), octx[batch::n_batches], otgt[batch::n_batches])
    got_g = np.frombuffer(bytes(st.grad), np.float32).astype(np.float64)
    assert np.allclose(got_g, g, rtol=1e-6, atol=1e-12)
    assert st.loss == pytest.approx(loss, rel=1e-6)
    th1, _, _ = OL.adam_step(theta0.astype(np.float64), g, np.zeros(161), np.zeros(161), 1, lr)
    got = np.frombuffer(bytes(st.theta), np.float32).astype(np.float64)
    assert np.allclose(got, th1, rtol=0, atol=1e-5 * lr + 1e-6 * np.abs(th1).max())
    assert st.step == 1


def test_trainer_lowers_loss_and_roundtrips():
    img, (octx, otgt) = _oracle_pairs()
    ctx = torch.from_numpy(octx.astype(np.int8)).to(DEV)
    tgt = torch.from_numpy(otgt.astype(np.int32)).to(DEV)
    tr = GL.Trainer(synth.mlp_init(OL.N_PARAMS, 72), DEV)
    losses = []
    for s in range(60):
        tr.step(ctx, tgt, 0.01, s % 4, 4)
        losses.append(tr.read().loss)
    assert losses[-1] < losses[0]
    net = tr.predictor()
    buf = img.reshape(-1)
    key, nonce = bytes(range(16)), bytes(range(16, 32))
    priv, pub = _protect(buf, 200, 2, key, nonce, net)
    assert _restore(priv, pub, buf.size, 200, 2, key, nonce, net) == buf.tobytes()


def test_golden_predictor_full_size_image():
    """One 4096 x 4096 smooth image at 3 levels with the oracle-trained
    network of tests/golden: element-wise against the oracle."""
    import json
    import os
    from conftest import GOLDEN
    rec = json.load(open(os.path.join(GOLDEN, "predictor_smooth.json")))
    raw = (np.array(rec["w1"]), np.array(rec["b1"]), np.array(rec["w2"]), rec["b2"], rec["shift"])
    onet, gnet = OL.Predictor(*raw), GL.Predictor.from_arrays(*raw)
    img = synth.smooth(4096, 4096, 4000).reshape(-1)
    key, nonce = synth.key_nonce(104, 204)
    _say("golden predictor 4096x4096 L3")
    got = _protect(img, 4096, 3, key, nonce, gnet)
    assert got == OL.protect(img, 4096, 3, key, nonce, onet)
    assert _restore(*got, img.size, 4096, 3, key, nonce, gnet) == img.tobytes()


def _entropy(values):
    _, counts = np.unique(np.asarray(values).reshape(-1), return_counts=True)
    p = counts / counts.sum()
    return float(-(p * np.log2(p)).sum())


def test_gpu_trained_network_lowers_detail_entropy():
    """What training gains: a network trained on the GPU from a smooth image's
    own (context, target) pairs gives lower zeroth-order entropy of the
    detail bands (eq. (5.6)) than the plain lifting, round trip exact."""
    img = synth.smooth(512, 512, 77).reshape(-1)
    x = torch.from_numpy(img).to(DEV)
    ctx, tgt = GL.training_pairs(x, 512, 3)
    tr = GL.Trainer(synth.mlp_init(OL.N_PARAMS, 78), DEV)
    nb = max(tgt.numel() // 16384, 1)
    for s in range(200):
        tr.step(ctx, tgt, 0.01, s % nb, nb)
    net = tr.predictor()
    key, nonce = bytes(range(16)), bytes(range(32, 48))
    priv, pub = _protect(img, 512, 3, key, nonce, net)
    _, pub0 = _protect(img, 512, 3, key, nonce, GL.Predictor())
    e_learned = _entropy(np.frombuffer(pub, "<i2"))
    e_plain = _entropy(np.frombuffer(pub0, "<i2"))
    _say(f"detail entropy plain {e_plain:.4f} learned {e_learned:.4f} bits")
    assert e_learned < e_plain
    assert _restore(priv, pub, img.size, 512, 3, key, nonce, net) == img.tobytes()
