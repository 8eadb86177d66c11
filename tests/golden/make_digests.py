"""Write tests/golden/oracle_digests.json: SHA-256 of the oracle's fragments.

Calls only ``oracle`` (and the seeded input generators in ``synth``): no value
stored here comes from the GPU path.  Run from the repository root:

    python tests/golden/make_digests.py

It covers the 512x512 one-level workload, the 256 MiB three-level workload
(~20 GB of host memory and a few minutes) and image 0 of the learned-predictor
workload (4096 x 4096, 3 levels, the oracle-trained network stored in
predictor_smooth.json).  ``--only KEY`` recomputes one entry.
"""
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import synth  # noqa: E402
from oracle import fragment  # noqa: E402


def digest_config(cfg):
    buf = np.ascontiguousarray(cfg["buf"])
    t0 = time.time()
    priv, pub = fragment.protect(buf, cfg["width"], cfg["levels"], cfg["key"], cfg["nonce"])
    return dict(name=cfg["name"], n=int(buf.size), width=cfg["width"], levels=cfg["levels"],
                input_sha256=hashlib.sha256(buf.tobytes()).hexdigest(),
                priv_sha256=hashlib.sha256(priv).hexdigest(),
                pub_sha256=hashlib.sha256(pub).hexdigest(),
                priv_bytes=len(priv), pub_bytes=len(pub),
                oracle_seconds=round(time.time() - t0, 1))


def digest_learned():
    from oracle import learned
    with open(os.path.join(ROOT, "tests", "golden", "predictor_smooth.json")) as f:
        rec = json.load(f)
    net = learned.Predictor(np.array(rec["w1"]), np.array(rec["b1"]), np.array(rec["w2"]),
                            rec["b2"], rec["shift"])
    buf = synth.learned_image(0)
    key, nonce = synth.learned_key_nonce(0)
    t0 = time.time()
    priv, pub = learned.protect(buf, 4096, 3, key, nonce, net)
    return dict(name="learned-predictor image 0 (4096x4096 smooth), 3 levels", n=int(buf.size),
                width=4096, levels=3, input_sha256=hashlib.sha256(buf.tobytes()).hexdigest(),
                predictor_sha256=hashlib.sha256(net.to_bytes()).hexdigest(),
                priv_sha256=hashlib.sha256(priv).hexdigest(),
                pub_sha256=hashlib.sha256(pub).hexdigest(),
                priv_bytes=len(priv), pub_bytes=len(pub),
                oracle_seconds=round(time.time() - t0, 1))


def main():
    path = os.path.join(ROOT, "tests", "golden", "oracle_digests.json")
    only = sys.argv[sys.argv.index("--only") + 1] if "--only" in sys.argv else None
    out = {}
    if only and os.path.exists(path):
        with open(path) as f:
            out = json.load(f)
    makers = {"small": lambda: digest_config(synth.config_small()),
              "large": lambda: digest_config(synth.config_large()),
              "learned": digest_learned}
    for key, make in makers.items():
        if only and key != only:
            continue
        out[key] = make()
        print(key, out[key], flush=True)
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
