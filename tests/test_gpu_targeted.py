"""GPU parity of the targeted-edit variant (pmsz_correct_mode with
PMSZ_EDIT_TARGETED) against the oracle's targeted mode, bit for bit: ragged
shapes over several tiles, ties, binary32 and binary64, the Perlin and
Gaussian-peak workloads, a round limit, and the worked ascending example."""
import numpy as np
import pytest

import oracle
import paper_2601_01787_amd as pmsz
import synth
from test_gpu_parity import SHAPES, STAT_KEYS, dev, host, random_case, same_bits

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("shape", SHAPES[:-1], ids=lambda s: "x".join(map(str, s)))
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("ties", [False, True])
def test_targeted_matches_oracle(shape, dtype, ties):
    f, fhat, xi = random_case(shape, dtype, seed=5 * sum(shape) + ties, ties=ties)
    g_ref, st_ref = oracle.correct(f, fhat, xi, mode="targeted")
    g, st = pmsz.correct(dev(f), dev(fhat), xi, mode="targeted")
    for k in STAT_KEYS:
        assert st[k] == st_ref[k], (k, st, st_ref)
    assert same_bits(host(g), g_ref)


def test_targeted_small_perlin_and_peaks():
    f, fhat, xi = synth.small_perlin_case()
    f, fhat = f.numpy(), fhat.numpy()
    g_ref, st_ref = oracle.correct(f, fhat, xi, mode="targeted")
    g, st = pmsz.correct(dev(f), dev(fhat), xi, mode="targeted")
    assert [st[k] for k in STAT_KEYS] == [st_ref[k] for k in STAT_KEYS]
    assert same_bits(host(g), g_ref)
    f, fhat, xi = synth.make_2d_case(613, 401, 1e-3, 99)
    f, fhat = f.numpy(), fhat.numpy()
    g_ref, st_ref = oracle.correct(f, fhat, xi, mode="targeted")
    g, st = pmsz.correct(dev(f), dev(fhat), xi, mode="targeted")
    assert [st[k] for k in STAT_KEYS] == [st_ref[k] for k in STAT_KEYS]
    assert same_bits(host(g), g_ref)


@pytest.mark.parametrize("k", [0, 1, 2])
def test_targeted_round_limit(k):
    f, fhat, xi = random_case((33, 40, 70), np.float32, seed=77)
    g_ref, st_ref = oracle.correct(f, fhat, xi, max_iters=k, mode="targeted")
    g, st = pmsz.correct(dev(f), dev(fhat), xi, max_iters=k, mode="targeted")
    assert [st[k2] for k2 in STAT_KEYS] == [st_ref[k2] for k2 in STAT_KEYS]
    assert same_bits(host(g), g_ref)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_targeted_ascending_example(dtype):
    f = np.array([[0, 1, 0.5]], dtype)
    fh = np.array([[0, 0.75, 1.0]], dtype)
    g, st = pmsz.correct(dev(f), dev(fh), 0.5, mode="targeted")
    assert st["status"] == "OK" and st["iterations"] == 1
    assert host(g)[0, 2] == np.nextafter(dtype(0.75), dtype(-np.inf))


def test_unknown_mode_rejected():
    f = np.zeros((4, 4), np.float32)
    with pytest.raises(KeyError):
        pmsz.correct(dev(f), dev(f), 0.1, mode="bogus")


def test_targeted_full_size_perlin_512():
    """512^3 binary32 Perlin with the targeted edit: the corrected field and
    statistics against the hash and counts the oracle wrote."""
    import hashlib
    import json
    import os
    import torch
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                        "perlin512_f32_targeted.json")
    gold = json.load(open(path))
    f, fhat, xi = synth.large_perlin_case(device="cuda:0")
    sha = lambda t: hashlib.sha256(host(t).view(np.uint8)).hexdigest()  # noqa: E731
    assert sha(fhat) == gold["sha256_fhat"], "input generator differs on this host"
    g, st = pmsz.correct(f, fhat, xi, mode="targeted")
    for k in STAT_KEYS:
        assert st[k] == gold["stats"][k], (k, st, gold["stats"])
    assert sha(g) == gold["sha256_g"]
    assert int(torch.count_nonzero(g != fhat)) == gold["vertices_edited"]
