"""Write tests/golden/batch256_f32.json: the oracle's result on every field of
the uneven 2D batch (256 Gaussian-peak fields, sizes log-uniform in
[256, 4096] per axis, relative bound from {1e-2, 1e-3, 1e-4}, master seed
256): per field, the sha256 of f, fhat and the corrected field, and every
statistic.

Calls only the CPU oracle and the seeded input generator (host synthesis,
reproducible bit for bit)."""
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402


def sha(a):
    return hashlib.sha256(np.ascontiguousarray(a).view(np.uint8)).hexdigest()


def main():
    t0 = time.time()
    rec = synth.batch_recipe(256, 256)
    cases = synth.batch_cases(256, 256)
    print("generated in %.1f s" % (time.time() - t0), flush=True)
    t0 = time.time()
    fields = []
    for c, (f, fhat, xi) in zip(rec, cases):
        f, fhat = f.numpy(), fhat.numpy()
        g, st = oracle.correct(f, fhat, xi)
        fields.append({"nx": c["nx"], "ny": c["ny"], "rel_eps": c["rel_eps"], "seed": c["seed"],
                       "xi": xi, "sha256_f": sha(f), "sha256_fhat": sha(fhat),
                       "sha256_g": sha(g), "stats": st})
    print("oracle in %.1f s on %d threads" % (time.time() - t0, oracle.threads()), flush=True)
    out = {"workload": "256 uneven 2D Gaussian-peak fields, float32, master seed 256",
           "made_by": "tests/golden/make_golden_batch.py (oracle only)", "fields": fields}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "batch256_f32.json")
    with open(path, "w") as fh:
        json.dump(out, fh)
    print("wrote", path, flush=True)


if __name__ == "__main__":
    main()
