"""GPU parity: the HIP path (through the C ABI) against the CPU oracle, bit for
bit, on seeded inputs that span several tiles with ragged tails, plus the
edge cases of the method (stall, out-of-rounds, validation failures,
subnormal values, degenerate grids)."""
import json
import os

import numpy as np
import pytest
import torch

import oracle
import paper_2601_01787_amd as pmsz
import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
STAT_KEYS = ("iterations", "steps_applied", "flagged_final", "stalled_flags",
             "mismatch_initial", "status")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def same_bits(a, b):
    a, b = np.ascontiguousarray(a), np.ascontiguousarray(b)
    return a.shape == b.shape and a.dtype == b.dtype and np.array_equal(a.view(np.uint8),
                                                                       b.view(np.uint8))


def random_case(shape, dtype, seed, ties=False, xi=0.05):
    rng = np.random.default_rng(seed)
    if ties:
        f = (rng.integers(0, 8, size=shape) * 0.125).astype(dtype)
    else:
        f = rng.uniform(0, 1, size=shape)
        f = (f + np.roll(f, 1, axis=-1) + np.roll(f, 1, axis=0)) / 3.0
        f = f.astype(dtype)
    lb, ub = oracle.bounds(f, xi)
    fhat = (f.astype(np.float64) + rng.uniform(-xi, xi, size=shape)).astype(dtype)
    if ties:
        fhat[rng.uniform(size=shape) < 0.3] = dtype(0.5)
    fhat = np.minimum(np.maximum(fhat, lb), ub)
    return f, fhat, xi


SHAPES = [(64, 64, 64), (7, 9, 70), (3, 130, 67), (33, 1, 65), (1, 5, 300), (70, 2, 3),
          (300, 517), (1, 1000), (1000, 1), (257, 255), (1, 1)]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("ties", [False, True])
def test_directions_match_oracle(shape, dtype, ties):
    f, fhat, _ = random_case(shape, dtype, seed=sum(shape) + ties, ties=ties)
    for h in (f, fhat):
        d = host(pmsz.directions(dev(h)))
        assert same_bits(d, oracle.directions(h))


@pytest.mark.parametrize("shape", SHAPES[:-1], ids=lambda s: "x".join(map(str, s)))
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("ties", [False, True])
def test_correct_matches_oracle(shape, dtype, ties):
    f, fhat, xi = random_case(shape, dtype, seed=3 * sum(shape) + ties, ties=ties)
    g_ref, st_ref = oracle.correct(f, fhat, xi)
    g, st = pmsz.correct(dev(f), dev(fhat), xi)
    g = host(g)
    for k in STAT_KEYS:
        assert st[k] == st_ref[k], (k, st, st_ref)
    assert same_bits(g, g_ref)


def test_small_perlin_workload():
    """64^3 float32 Perlin, eps = 1e-3 (the small workload the oracle finishes
    in seconds)."""
    f, fhat, xi = synth.small_perlin_case()
    f, fhat = f.numpy(), fhat.numpy()
    g_ref, st_ref = oracle.correct(f, fhat, xi)
    g, st = pmsz.correct(dev(f), dev(fhat), xi)
    assert st_ref["iterations"] > 2
    for k in STAT_KEYS:
        assert st[k] == st_ref[k], (k, st, st_ref)
    assert same_bits(host(g), g_ref)


def test_gaussian_peaks_2d_and_grf_3d():
    f, fhat, xi = synth.make_2d_case(613, 401, 1e-3, 99)
    f, fhat = f.numpy(), fhat.numpy()
    g_ref, st_ref = oracle.correct(f, fhat, xi)
    g, st = pmsz.correct(dev(f), dev(fhat), xi)
    assert [st[k] for k in STAT_KEYS] == [st_ref[k] for k in STAT_KEYS]
    assert same_bits(host(g), g_ref)
    f = synth.grf3d((40, 48, 72), 1024).numpy()
    fhat = synth.quantise_proxy(f, 1e-5, 1024)
    g_ref, st_ref = oracle.correct(f, fhat, 1e-5)
    g, st = pmsz.correct(dev(f), dev(fhat), 1e-5)
    assert [st[k] for k in STAT_KEYS] == [st_ref[k] for k in STAT_KEYS]
    assert same_bits(host(g), g_ref)


@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_round_limit_gives_the_same_iterate(k):
    f, fhat, xi = random_case((20, 30, 40), np.float32, 5)
    g_ref, st_ref = oracle.correct(f, fhat, xi, max_iters=k)
    g, st = pmsz.correct(dev(f), dev(fhat), xi, max_iters=k)
    assert st_ref["status"] == "NOT_CONVERGED"
    assert [st[k2] for k2 in STAT_KEYS] == [st_ref[k2] for k2 in STAT_KEYS]
    assert same_bits(host(g), g_ref)


@pytest.mark.parametrize("k", [1, 3])
def test_resume_from_an_iterate_gives_the_same_result(k):
    """The iteration depends on (f, g^k) only: stopping after k rounds and
    correcting g^k as a new fhat ends at the same field, with the rounds of
    the two runs adding up to those of one run."""
    f, fhat, xi = random_case((24, 31, 45), np.float32, 21)
    g_all, st_all = pmsz.correct(dev(f), dev(fhat), xi)
    g_k, st_k = pmsz.correct(dev(f), dev(fhat), xi, max_iters=k)
    assert st_k["status"] == "NOT_CONVERGED"
    g_end, st_end = pmsz.correct(dev(f), g_k, xi)
    assert st_end["status"] == st_all["status"] == "OK"
    assert st_k["iterations"] + st_end["iterations"] == st_all["iterations"]
    assert st_k["steps_applied"] + st_end["steps_applied"] == st_all["steps_applied"]
    assert same_bits(host(g_end), host(g_all))


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_crafted_stall_case_on_gpu(dtype):
    """Two distinct values whose lower bounds merge (reading A9): the run
    ends STALLED at the merged bound, as in the oracle."""
    a = dtype(1e-20)
    f = np.array([[np.nextafter(a, dtype(1)), a]], dtype=dtype)
    lb, _ = oracle.bounds(f, 1.0)
    fhat = np.array([[lb[0, 0], 0.0]], dtype=dtype)
    g_ref, st_ref = oracle.correct(f, fhat, 1.0)
    g, st = pmsz.correct(dev(f), dev(fhat), 1.0)
    assert st_ref["status"] == "STALLED"
    assert [st[k] for k in STAT_KEYS] == [st_ref[k] for k in STAT_KEYS]
    assert same_bits(host(g), g_ref)


def _hand_cases():
    with open(os.path.join(GOLDEN, "hand_examples.json")) as fh:
        return json.load(fh)["cases"]


@pytest.mark.parametrize("case", _hand_cases(), ids=lambda c: c["name"])
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_hand_examples_on_gpu(case, dtype):
    if case.get("dtype") and np.dtype(case["dtype"]) != np.dtype(dtype):
        pytest.skip("case is specific to " + case["dtype"])
    shape = (case["ny"], case["nx"])
    f = np.array(case["f"], dtype=dtype).reshape(shape)
    if case["fhat"] == "lower_bound":
        fhat, _ = oracle.bounds(f, case["xi"])
    else:
        fhat = np.array(case["fhat"], dtype=dtype).reshape(shape)
    g, st = pmsz.correct(dev(f), dev(fhat), case["xi"])
    assert st["status"] == case["status"] and st["iterations"] == case["iterations"]
    if "g_final" in case:
        assert host(g).reshape(-1).tolist() == case["g_final"]


def test_validation_failures_leave_g_untouched():
    f, fhat, xi = random_case((9, 10, 70), np.float32, 8)
    bad = fhat.copy()
    bad[3, 4, 5] = np.nan
    g, st = pmsz.correct(dev(f), dev(bad), xi)
    assert st["status"] == "NONFINITE" and same_bits(host(g), bad)
    out = fhat.copy()
    out[1, 2, 3] = f[1, 2, 3] + np.float32(2 * xi)
    g, st = pmsz.correct(dev(f), dev(out), xi)
    assert st["status"] == "INPUT_BOUND" and same_bits(host(g), out)
    g, st = pmsz.correct(dev(f), dev(f), 0.0)
    assert st["status"] == "OK" and st["iterations"] == 0


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_validation_at_the_exact_bounds(dtype):
    """fhat exactly at every vertex's lower (or upper) bound is valid, and one
    value past the bound at any single vertex is out of bound; the bounds are
    the oracle's exact roundings, over magnitudes from subnormal to large and
    bounds from sub-ulp to huge, and the GPU's status equals the oracle's."""
    rng = np.random.default_rng(31)
    shape = (3, 5, 70)
    n = int(np.prod(shape))
    lo_e, hi_e = (-140, 100) if dtype == np.float32 else (-1060, 1000)
    f = (rng.choice([-1.0, 1.0], n) * rng.uniform(0.5, 1.0, n) *
         np.exp2(rng.integers(lo_e, hi_e, n).astype(np.float64))).astype(dtype).reshape(shape)
    xis = (1e-42, 1e-3, 1e30) if dtype == np.float32 else (1e-320, 1e-3, 1e300)
    for xi in xis:
        lb, ub = oracle.bounds(f, xi)
        for edge, step in ((lb, -np.inf), (ub, np.inf)):
            assert oracle.validate(f, edge, xi) != "INPUT_BOUND"
            _, st = pmsz.correct(dev(f), dev(edge), xi, max_iters=0)
            assert st["status"] not in ("INPUT_BOUND", "NONFINITE"), (xi, st)
            for i in rng.choice(n, 12, replace=False):
                past = edge.copy().reshape(-1)
                past[i] = np.nextafter(past[i], dtype(step))
                if not np.isfinite(past[i]):
                    continue
                past = past.reshape(shape)
                want = oracle.validate(f, past, xi)
                assert want == "INPUT_BOUND", (xi, i, want)
                _, st = pmsz.correct(dev(f), dev(past), xi, max_iters=0)
                assert st["status"] == want, (xi, int(i), st)


def test_subnormal_values():
    """Bounds and edits in the binary32 subnormal range (no flush to zero)."""
    rng = np.random.default_rng(17)
    tiny = np.float32(1e-40)
    f = (rng.uniform(-1, 1, size=(6, 40, 70)) * tiny).astype(np.float32)
    xi = 3e-41
    lb, ub = oracle.bounds(f, xi)
    fhat = (f + rng.uniform(-1, 1, size=f.shape).astype(np.float32) * np.float32(xi)).astype(
        np.float32)
    fhat = np.minimum(np.maximum(fhat, lb), ub)
    g_ref, st_ref = oracle.correct(f, fhat, xi)
    g, st = pmsz.correct(dev(f), dev(fhat), xi)
    assert st_ref["steps_applied"] > 0
    assert [st[k] for k in STAT_KEYS] == [st_ref[k] for k in STAT_KEYS]
    assert same_bits(host(g), g_ref)


@pytest.mark.parametrize("shape", [(64, 64, 64), (3, 130, 67), (300, 517), (1000, 1)],
                         ids=lambda s: "x".join(map(str, s)))
def test_labels_match_oracle(shape):
    f, fhat, xi = random_case(shape, np.float32, 21)
    for h in (f, fhat):
        d = pmsz.directions(dev(h))
        mx, mn = pmsz.labels(d)
        rmx, rmn = oracle.labels(oracle.directions(h))
        assert np.array_equal(host(mx), rmx) and np.array_equal(host(mn), rmn)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_verify_matches_oracle(dtype):
    f, fhat, xi = random_case((17, 40, 70), dtype, 31)
    rep = pmsz.verify(dev(f), dev(fhat), None, xi)
    assert rep == oracle.verify(f, fhat, None, xi)
    assert rep["asc_mismatch"] > 0
    g, _ = pmsz.correct(dev(f), dev(fhat), xi)
    rep = pmsz.verify(dev(f), g, dev(fhat), xi)
    ref = oracle.verify(f, host(g), fhat, xi)
    assert rep == ref
    assert rep["wrong_label"] == 0 and rep["vertices_edited"] > 0


def test_batched_matches_alone():
    cases = [synth.make_2d_case(nx, ny, rel, seed) for nx, ny, rel, seed in
             [(300, 257, 1e-2, 1), (129, 700, 1e-3, 2), (256, 256, 1e-4, 3), (70, 90, 1e-3, 4)]]
    alone = []
    for f, fhat, xi in cases:
        g, st = pmsz.correct(dev(f.numpy()), dev(fhat.numpy()), xi)
        alone.append((host(g), st))
    fields = [(dev(f.numpy()), dev(fhat.numpy()), xi) for f, fhat, xi in cases]
    stats = pmsz.correct_batched(fields)
    for (g_a, st_a), (_, g_b, _), st_b in zip(alone, fields, stats):
        assert st_a == st_b
        assert same_bits(g_a, host(g_b))


def test_mixed_dimension_batch_with_sweep_kernels_matches_alone():
    """A batch of 2^23 vertices or more runs its first two rounds' tile
    detection as sweep kernels, one per dimension; with 2D and 3D fields both
    in tile rounds (round 1 here), each kernel must take only its own
    dimension's tiles and their activity marks.  Every field ends as it does
    alone (where the two big fields take the one-launch path)."""
    cases = [synth.perlin_case(160, 4, 4, 1e-3, 21), synth.make_2d_case(2100, 2100, 1e-3, 22),
             synth.perlin_case(24, 3, 3, 1e-3, 1), synth.make_2d_case(300, 190, 1e-2, 3)]
    assert sum(f.numel() for f, _, _ in cases) >= 1 << 23
    alone = []
    for f, fhat, xi in cases:
        g, st = pmsz.correct(f.to(DEV), fhat.to(DEV), xi)
        alone.append((g, st))
    fields = [(f.to(DEV), fhat.to(DEV), xi) for f, fhat, xi in cases]
    stats = pmsz.correct_batched(fields)
    assert pmsz.last_timing()["sweeps"] > 0
    for i, ((g_a, st_a), (_, g_b, _), st_b) in enumerate(zip(alone, fields, stats)):
        assert st_a == st_b, i
        assert torch.equal(g_a, g_b), i


def test_later_tile_rounds_as_sweep_kernels_match_alone():
    """In a batch of 2^23 vertices or more, an engine launch ends before any
    later round in which a field of 2^23 vertices or more sweeps tiles, and
    that round's tile detection runs as a sweep kernel between launches.
    Here the 4096^2 field at 1e-2 keeps tile rounds past round 1 (more than
    two sweep launches); every field ends as it does alone."""
    cases = [synth.make_2d_case(4096, 4096, 1e-2, 31), synth.make_2d_case(1500, 900, 1e-3, 32),
             synth.perlin_case(40, 3, 3, 1e-3, 2), synth.make_2d_case(70, 90, 1e-3, 4)]
    alone = []
    for f, fhat, xi in cases:
        g, st = pmsz.correct(f.to(DEV), fhat.to(DEV), xi)
        alone.append((g, st))
    fields = [(f.to(DEV), fhat.to(DEV), xi) for f, fhat, xi in cases]
    stats = pmsz.correct_batched(fields)
    tm = pmsz.last_timing()
    assert tm["sweeps"] > 2, tm
    for i, ((g_a, st_a), (_, g_b, _), st_b) in enumerate(zip(alone, fields, stats)):
        assert st_a == st_b, i
        assert torch.equal(g_a, g_b), i
    # the per-round record spans every launch: its edits add up to the fields'
    rounds = pmsz.last_rounds()
    assert len(rounds) == tm["rounds"]
    assert sum(r["edits"] for r in rounds) == sum(st["steps_applied"] for st in stats)


def noise_case(n, xi, seed):
    """White noise on [0, 1] in an n^3 binary32 grid, fhat within xi of f: a
    loop whose edits shrink slowly, round after round."""
    rng = np.random.default_rng(seed)
    f = rng.uniform(0, 1, size=(n, n, n)).astype(np.float32)
    lb, ub = oracle.bounds(f, xi)
    fhat = (f.astype(np.float64) + rng.uniform(-xi, xi, size=f.shape)).astype(np.float32)
    return f, np.minimum(np.maximum(fhat, lb), ub), xi


@pytest.mark.parametrize("n", [24, 40])
def test_tail_rounds_and_handback_match_oracle(n):
    """Once a round edits few vertices the loop goes on in the tail kernel on
    one XCD; a tail round whose target list overflowed (a field of n^3
    vertices lists n^3 / 256 + 1024 targets) sweeps tiles, so the tail stops
    before it and the engine takes that round.  Either way the result is the
    oracle's, bit for bit."""
    f, fhat, xi = noise_case(n, 0.2, 7 + n)
    g_ref, st_ref = oracle.correct(f, fhat, xi)
    g, st = pmsz.correct(dev(f), dev(fhat), xi)
    tm = pmsz.last_timing()
    assert tm["tail_rounds"] > 0, tm
    assert tm["handbacks"] > 0, tm
    for k in STAT_KEYS:
        assert st[k] == st_ref[k], (k, st, st_ref)
    assert same_bits(host(g), g_ref)
    rounds = pmsz.last_rounds()
    assert len(rounds) == tm["rounds"]
    assert sum(r["edits"] for r in rounds) == st["steps_applied"]


def test_small_perlin_tail():
    """The 64^3 workload hands its rounds after the first few to the tail
    kernel and ends there."""
    f, fhat, xi = synth.small_perlin_case()
    g, st = pmsz.correct(f.to(DEV), fhat.to(DEV), xi)
    tm = pmsz.last_timing()
    assert tm["tail_rounds"] > 0 and tm["handbacks"] == 0, tm
    assert tm["tail_rounds"] < tm["rounds"]


def test_full_size_perlin_512():
    """512^3 binary32 Perlin (one GPU's weak-scaling share): the corrected field
    and the directions are compared through hashes the oracle wrote, and the
    labels at sampled vertices through the oracle's walked labels."""
    import hashlib
    path = os.path.join(GOLDEN, "perlin512_f32.json")
    gold = json.load(open(path))
    f, fhat, xi = synth.large_perlin_case(device=DEV)
    sha = lambda t: hashlib.sha256(host(t).view(np.uint8)).hexdigest()  # noqa: E731
    assert sha(f) == gold["sha256_f"], "input generator differs on this host"
    assert sha(fhat) == gold["sha256_fhat"]
    d = pmsz.directions(f)
    assert sha(d) == gold["sha256_dirs_f"]
    g, st = pmsz.correct(f, fhat, xi, dirs_f=d)
    for k in STAT_KEYS:
        assert st[k] == gold["stats"][k], (k, st, gold["stats"])
    assert sha(g) == gold["sha256_g"]
    # the benchmarked call: directions computed inside the correction
    g2, st2 = pmsz.correct(f, fhat, xi)
    for k in STAT_KEYS:
        assert st2[k] == gold["stats"][k], (k, st2, gold["stats"])
    assert sha(g2) == gold["sha256_g"]
    del g2
    mx, mn = pmsz.labels(d)
    idx = torch.tensor(gold["label_sample_idx"], device=DEV)
    assert host(mx.reshape(-1)[idx]).tolist() == gold["label_sample_max"]
    assert host(mn.reshape(-1)[idx]).tolist() == gold["label_sample_min"]
    rep = pmsz.verify(f, g, fhat, xi)
    assert rep["wrong_label"] == 0 and rep["bound_violations"] == 0
    assert rep["asc_mismatch"] == 0 and rep["desc_mismatch"] == 0


def _bad_dirs_cases():
    """Direction bytes no direction pass makes, each at one vertex of a valid
    array: code 8, a z-bit code in 2D, and codes stepping out of the grid at a
    boundary vertex (both nibbles)."""
    out = []
    for shape, i, byte in (((5, 6, 70), 123, 0x08), ((5, 6, 70), 123, 0x80),
                           ((40, 70), 77, 0x05), ((40, 70), 77, 0x40),
                           ((5, 6, 70), 0, 0x09), ((5, 6, 70), 0, 0xA0),
                           ((5, 6, 70), 5 * 6 * 70 - 1, 0x07), ((40, 70), 69, 0x01),
                           ((40, 70), 40 * 70 - 70, 0x20)):
        out.append((shape, i, byte))
    return out


@pytest.mark.parametrize("shape,i,byte", _bad_dirs_cases())
def test_invalid_direction_bytes_are_rejected(shape, i, byte):
    """Caller-supplied direction bytes become neighbour offsets: a byte that
    does not name a neighbour inside the grid is reported as INVALID_ARG by
    pmsz_correct (g untouched) and by pmsz_labels, before any offset is used."""
    f, fhat, xi = random_case(shape, np.float32, 5)
    d = pmsz.directions(dev(f))
    bad = d.clone().reshape(-1)
    bad[i] = byte
    bad = bad.reshape(d.shape)
    g = dev(fhat)
    with pytest.raises(pmsz.PmszError) as e:
        pmsz.correct(dev(f), g, xi, dirs_f=bad, inplace=True)
    assert e.value.status == 1
    assert same_bits(host(g), fhat)
    with pytest.raises(pmsz.PmszError) as e:
        pmsz.labels(bad)
    assert e.value.status == 1
    # the valid bytes still work
    g, st = pmsz.correct(dev(f), dev(fhat), xi, dirs_f=d)
    assert st["status"] == "OK"


@pytest.mark.parametrize("cycle", [2, 3])
def test_labels_reject_pointer_cycles(cycle):
    """Valid codes that do not form a forest are INVALID_ARG: two vertices
    pointing at each other (the chase comes back to its start), or three in a
    ring (it never settles within the pass limit)."""
    f, _, _ = random_case((4, 6, 66), np.float32, 6)
    d = pmsz.directions(dev(f)).reshape(-1)
    nx = 66
    if cycle == 2:
        ring = ((10, 0x01), (11, 0x09))           # 10 -> 11 -> 10
    else:
        ring = ((10, 0x01), (11, 0x02), (11 + nx, 0x0B))  # 10 -> 11 -> 11+nx -> 10
    for v, code in ring:
        d[v] = (d[v] & 0xF0) | code
    with pytest.raises(pmsz.PmszError) as e:
        pmsz.labels(d.reshape(4, 6, 66))
    assert e.value.status == 1


def test_labels_pass_counts():
    """Pointer jumping stops at the first pass that changes nothing: at most
    the passes a doubling chase needs over the longest integral line."""
    f, _, _ = random_case((16, 40, 70), np.float32, 7)
    d = pmsz.directions(dev(f))
    mx, mn = pmsz.labels(d)
    info = pmsz.last_labels()
    assert info["vertices"] == f.size
    assert 1 <= info["passes_max"] <= 12 and 1 <= info["passes_min"] <= 12
    rmx, rmn = oracle.labels(oracle.directions(f))
    assert np.array_equal(host(mx), rmx) and np.array_equal(host(mn), rmn)
