"""The tile-height policy and its autotuner on the GPU: results and statistics
are bit-identical to the oracle at every tiles-per-field target (3D and 2D,
single fields and a batch), and the tuner leaves its inputs unchanged,
returns one of the candidates and installs it."""
import numpy as np
import pytest
import torch

import oracle
import paper_2601_01787_amd as pmsz
import synth
from test_gpu_parity import STAT_KEYS, dev, host, random_case, same_bits

pytestmark = pytest.mark.gpu

TARGETS = [1, 256, 2048, 1 << 20]


@pytest.fixture(autouse=True)
def default_targets():
    yield
    for nd in (2, 3):
        for dt in (torch.float32, torch.float64):
            pmsz.set_tiles_target(nd, dt, 0)


@pytest.mark.parametrize("shape,dtype", [((40, 33, 70), np.float32), ((21, 50, 130), np.float64),
                                         ((300, 517), np.float32), ((1000, 77), np.float64)])
def test_results_do_not_depend_on_tile_height(shape, dtype):
    f, fhat, xi = random_case(shape, dtype, seed=sum(shape))
    g_ref, st_ref = oracle.correct(f, fhat, xi)
    tdt = torch.float32 if dtype == np.float32 else torch.float64
    for t in TARGETS:
        pmsz.set_tiles_target(len(shape), tdt, t)
        g, st = pmsz.correct(dev(f), dev(fhat), xi)
        for k in STAT_KEYS:
            assert st[k] == st_ref[k], (t, k, st, st_ref)
        assert same_bits(host(g), g_ref), t


def test_batch_results_do_not_depend_on_tile_height():
    cases = [synth.make_2d_case(n, m, rel, seed) for n, m, rel, seed in
             ((256, 300, 1e-3, 1), (700, 257, 1e-2, 2), (64, 1100, 1e-4, 3))]
    refs = [oracle.correct(f.numpy(), fh.numpy(), xi) for f, fh, xi in cases]
    for t in TARGETS:
        pmsz.set_tiles_target(2, torch.float32, t)
        fields = [(dev(f.numpy()), dev(fh.numpy()), xi) for f, fh, xi in cases]
        stats = pmsz.correct_batched(fields)
        for (f, g, _), st, (g_ref, st_ref) in zip(fields, stats, refs):
            assert [st[k] for k in STAT_KEYS] == [st_ref[k] for k in STAT_KEYS]
            assert same_bits(host(g), g_ref)


def test_tuner_installs_a_candidate_and_keeps_inputs(tmp_path, monkeypatch):
    """The tuner installs the fastest candidate, leaves fhat alone and records
    every target in the tune cache named by PMSZ_TUNE_CACHE."""
    import json
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("PMSZ_TUNE_CACHE", str(cache))
    cases = [synth.make_2d_case(n, n, 1e-3, 10 + n) for n in (256, 512, 1024)]
    fields = [(dev(f.numpy()), dev(fh.numpy()), xi) for f, fh, xi in cases]
    keep = [fh.clone() for _, fh, _ in fields]
    cands = (256, 2048, 16384)
    best, ms = pmsz.tune_tiles(fields, candidates=cands, reps=1)
    assert best in cands and set(ms) == set(cands) and all(v > 0 for v in ms.values())
    assert pmsz.get_tiles_target(2, torch.float32) == best
    assert json.loads(cache.read_text())["2d_f32"] == best
    for (_, fh, _), k in zip(fields, keep):
        assert torch.equal(fh, k)


def test_default_rule_by_batch_size():
    """Without a set or tuned target a batch of n fields takes 2048 / n tiles
    per field, between 32 and 256: a 256-wide strip field of 512 rows is cut
    into 256 tiles alone (2 rows each) and into 32 tiles (16 rows each) in a
    batch of 64 such fields; the results match the field alone."""
    assert pmsz.get_tiles_target(2, torch.float32) == 0
    f, fhat, xi = synth.make_2d_case(256, 512, 1e-3, 5)
    g1, st1 = pmsz.correct(f.to("cuda:0"), fhat.to("cuda:0"), xi)
    assert pmsz.last_timing()["tiles"] == 256
    fields = [(f.to("cuda:0"), fhat.to("cuda:0"), xi) for _ in range(64)]
    stats = pmsz.correct_batched(fields)
    assert pmsz.last_timing()["tiles"] == 64 * 32
    for (_, g, _), st in zip(fields, stats):
        assert st == st1 and torch.equal(g, g1)
