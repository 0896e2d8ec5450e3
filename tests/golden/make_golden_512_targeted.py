"""Write tests/golden/perlin512_f32_targeted.json: the oracle's result with the
targeted edit on the 512^3 binary32 Perlin workload (6 octaves, 8 cells,
eps = 1e-4, seed 512), and its halving statistics beside it for the
iteration / edit comparison.

Calls only the CPU oracle and the seeded input generator.
"""
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
    f, fhat, xi = synth.large_perlin_case()
    f, fhat = f.numpy(), fhat.numpy()
    print("generated in %.1f s" % (time.time() - t0), flush=True)
    t0 = time.time()
    g, st = oracle.correct(f, fhat, xi, mode="targeted")
    print("oracle (targeted) in %.1f s: %s" % (time.time() - t0, st), flush=True)
    edited = int(np.count_nonzero(g != fhat))
    out = {
        "workload": "perlin 512^3 float32, 6 octaves, 8 cells, eps 1e-4, seed 512",
        "made_by": "tests/golden/make_golden_512_targeted.py (oracle only)",
        "edit": "targeted",
        "sha256_f": sha(f), "sha256_fhat": sha(fhat), "sha256_g": sha(g),
        "stats": st, "vertices_edited": edited, "xi": xi,
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)),
                        "perlin512_f32_targeted.json")
    with open(path, "w") as fh:
        json.dump(out, fh)
    print("wrote", path)


if __name__ == "__main__":
    main()
