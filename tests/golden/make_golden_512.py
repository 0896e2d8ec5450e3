"""Write tests/golden/perlin512_f32.json: the oracle's result on the 512^3
binary32 Perlin workload (6 octaves, 8 cells, eps = 1e-4, seed 512).

Calls only the CPU oracle and the seeded input generator.  The stored hashes
let the GPU test compare its full-size result bit for bit without rerunning
the oracle (minutes of CPU time) on the GPU host.
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
    g, st = oracle.correct(f, fhat, xi)
    print("oracle in %.1f s: %s" % (time.time() - t0, st), flush=True)
    d = oracle.directions(f)
    rng = np.random.default_rng(4242)
    idx = np.sort(rng.choice(f.size, size=4096, replace=False))
    mx, mn = oracle.labels_at(f, idx)
    out = {
        "workload": "perlin 512^3 float32, 6 octaves, 8 cells, eps 1e-4, seed 512",
        "made_by": "tests/golden/make_golden_512.py (oracle only)",
        "sha256_f": sha(f), "sha256_fhat": sha(fhat), "sha256_g": sha(g),
        "sha256_dirs_f": sha(d), "stats": st, "xi": xi,
        "label_sample_idx": idx.tolist(), "label_sample_max": mx.tolist(),
        "label_sample_min": mn.tolist(),
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "perlin512_f32.json")
    with open(path, "w") as fh:
        json.dump(out, fh)
    print("wrote", path)


if __name__ == "__main__":
    main()
