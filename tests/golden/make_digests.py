"""Write tests/golden/oracle_digests.json: SHA-256 of the oracle's fragments.

Calls only ``oracle`` (and the seeded input generators in ``synth``): no value
stored here comes from the GPU path.  Run from the repository root:

    python tests/golden/make_digests.py

It covers the 512x512 one-level workload and the 256 MiB three-level workload
(the latter needs ~20 GB of host memory and a few minutes).
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


def main():
    out = {}
    for key, make in (("small", synth.config_small), ("large", synth.config_large)):
        cfg = make()
        out[key] = digest_config(cfg)
        print(key, out[key], flush=True)
        del cfg
    path = os.path.join(ROOT, "tests", "golden", "oracle_digests.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
