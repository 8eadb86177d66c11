"""Write tests/golden/predictor_smooth.json: a context network trained by the
ORACLE (``oracle.learned.train``), used as a fixed input of the learned-path
parity tests and benchmark.

Calls only ``oracle`` and the seeded generators in ``synth``: no value stored
here comes from the GPU path.  Run from the repository root:

    python tests/golden/make_predictor.py

Recipe: training pairs of the 512 x 512 smooth image (seed 1) and of rows
0..256 of the 256 MiB mixed workload (its smooth third) (both decomposed to 3 levels),
concatenated; start from ``synth.mlp_init(161, 4)``; 300 quantisation-aware
Adam steps, learning rate 0.01, interleaved batches of about 65536 pairs.
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import synth  # noqa: E402
from oracle import dwt53  # noqa: E402
from oracle import learned as L  # noqa: E402


def main():
    t0 = time.time()
    img = synth.smooth(512, 512, 1).astype(np.int64)
    big = synth.config_large()
    w = big["width"]
    part = big["buf"][0:256 * w].reshape(256, w).astype(np.int64)
    del big
    c1, t1 = L.training_pairs(img, 3)
    c2, t2 = L.training_pairs(part, 3)
    ctx, tgt = np.concatenate([c1, c2]), np.concatenate([t1, t2])
    theta0 = synth.mlp_init(L.N_PARAMS, 4)
    theta = L.train(theta0, ctx, tgt, steps=300, lr=0.01, batch=65536)
    net = L.quantize(theta)
    _, det = L.fwd_multilevel(img, 3, net)
    _, det0 = dwt53.fwd_multilevel(img, 3)
    rec = dict(
        recipe=__doc__.split("Recipe: ")[1].strip(),
        pairs=int(tgt.size),
        loss_start=float(L.loss_grad(L.fake_quant(theta0), ctx, tgt)[0]),
        loss_end=float(L.loss_grad(L.fake_quant(theta), ctx, tgt)[0]),
        entropy_plain_512=L.detail_entropy(det0),
        entropy_learned_512=L.detail_entropy(det),
        w1=net.w1.tolist(), b1=net.b1.tolist(), w2=net.w2.tolist(), b2=net.b2, shift=net.shift,
        seconds=round(time.time() - t0, 1),
    )
    path = os.path.join(ROOT, "tests", "golden", "predictor_smooth.json")
    with open(path, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps({k: v for k, v in rec.items() if k not in ("w1", "b1", "w2")}))


if __name__ == "__main__":
    main()
