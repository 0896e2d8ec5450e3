"""Write tests/golden/grf1024x1024x768_f64.json: the oracle's result on the
large binary64 workload (Gaussian random field with a k^-3 spectrum,
1024 x 1024 x 768, relative bound 1e-5, seed 1024).

Calls only the CPU oracle and the seeded input generator (host synthesis,
reproducible bit for bit).  About 25 GB of host memory and a few minutes of
CPU time; the stored hashes let the GPU test compare its full-size result bit
for bit without rerunning the oracle on the GPU host.
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
    f, fhat, xi = synth.grf_case()
    f, fhat = f.numpy(), fhat.numpy()
    print("generated in %.1f s" % (time.time() - t0), flush=True)
    t0 = time.time()
    g, st = oracle.correct(f, fhat, xi)
    print("oracle in %.1f s on %d threads: %s" % (time.time() - t0, oracle.threads(), st),
          flush=True)
    out = {
        "workload": "grf k^-3 1024x1024x768 float64, relative eps 1e-5, seed 1024",
        "made_by": "tests/golden/make_golden_grf.py (oracle only)",
        "shape": list(f.shape), "xi": xi,
        "sha256_f": sha(f), "sha256_fhat": sha(fhat), "sha256_g": sha(g), "stats": st,
    }
    del g, fhat
    d = oracle.directions(f)
    out["sha256_dirs_f"] = sha(d)
    del d
    rng = np.random.default_rng(7681)
    idx = np.sort(rng.choice(f.size, size=4096, replace=False))
    mx, mn = oracle.labels_at(f, idx)
    out.update({"label_sample_idx": idx.tolist(), "label_sample_max": mx.tolist(),
                "label_sample_min": mn.tolist()})
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "grf1024x1024x768_f64.json")
    with open(path, "w") as fh:
        json.dump(out, fh)
    print("wrote", path, "in %.1f s" % (time.time() - t0), flush=True)


if __name__ == "__main__":
    main()
