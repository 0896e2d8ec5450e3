"""The large binary64 workload on the GPU: a 1024 x 1024 x 768 Gaussian random
field (k^-3 spectrum, relative bound 1e-5, 6.4 GB per array).  The input is
synthesised on the host, bit-reproducibly, and checked against the hashes
the oracle's golden records before anything else; the corrected field, the
direction bytes of f and every statistic must then equal the oracle's bit for
bit (tests/golden/grf1024x1024x768_f64.json, written by
tests/golden/make_golden_grf.py from the oracle alone), and the labels at the
golden's sampled vertices must equal the oracle's walked labels."""
import hashlib
import json
import os

import numpy as np
import pytest
import torch

import paper_2601_01787_amd as pmsz
import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "grf1024x1024x768_f64.json")
STAT_KEYS = ("iterations", "steps_applied", "flagged_final", "stalled_flags",
             "mismatch_initial", "status")


def sha(t):
    torch.cuda.synchronize()
    return hashlib.sha256(t.cpu().numpy().view(np.uint8)).hexdigest()


def test_grf_1024x1024x768_f64_matches_the_oracle():
    ref = json.load(open(GOLDEN))
    f, fhat, xi = synth.grf_case()
    assert tuple(f.shape) == tuple(ref["shape"]) and f.dtype == torch.float64
    assert xi == ref["xi"]
    # the host synthesis reproduced the oracle's input
    assert hashlib.sha256(f.numpy().view(np.uint8)).hexdigest() == ref["sha256_f"]
    assert hashlib.sha256(fhat.numpy().view(np.uint8)).hexdigest() == ref["sha256_fhat"]
    print("input matches the golden", flush=True)
    f, g = f.to(DEV), fhat.to(DEV)
    del fhat
    d = pmsz.directions(f)
    assert sha(d) == ref["sha256_dirs_f"]
    _, st = pmsz.correct(f, g, xi, inplace=True)
    assert [st[k] for k in STAT_KEYS] == [ref["stats"][k] for k in STAT_KEYS], st
    assert sha(g) == ref["sha256_g"]
    print("corrected field matches the golden: %s" % st, flush=True)
    mx, mn = pmsz.labels(d)
    idx = torch.tensor(ref["label_sample_idx"], dtype=torch.int64, device=DEV)
    assert mx.view(-1)[idx].cpu().tolist() == ref["label_sample_max"]
    assert mn.view(-1)[idx].cpu().tolist() == ref["label_sample_min"]
