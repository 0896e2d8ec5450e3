"""Pins of the decomposed-domain correction of the oracle (Sec. IV-B):
an independent explicit-vertex-list implementation on tiny grids, the
single-block special case, the minimum rule of the ghost exchange, the
restriction of comparisons to a block's core, and the invariants of
Sec. IV-C."""
import numpy as np
import pytest

import brute
import oracle
from oracle import multiblock as mb


def _case(seed, shape, dtype, ties=False):
    rng = np.random.default_rng(seed)
    if ties:
        f = (rng.integers(0, 6, size=shape) * 0.125).astype(dtype)
    else:
        f = rng.uniform(0, 1, size=shape).astype(dtype)
    xi = float(rng.choice([0.05, 0.1, 0.3]))
    lb, ub = oracle.bounds(f, xi)
    t = rng.uniform(0, 1, size=shape)
    fhat = (lb.astype(np.float64) + t * (ub.astype(np.float64) - lb)).astype(dtype)
    fhat = np.minimum(np.maximum(fhat, lb), ub)
    return f, fhat, xi


CASES = [((7, 9), (3, 2)), ((6, 5), (2, 2)), ((8, 4), (2, 3)),
         ((4, 5, 6), (2, 2, 2)), ((5, 4, 6), (3, 1, 2)), ((3, 6, 5), (1, 2, 1))]


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("shape,blocks", CASES)
@pytest.mark.parametrize("per_round", [False, True])
def test_blocks_match_explicit_vertex_lists(seed, shape, blocks, per_round):
    dtype = np.float32 if seed % 2 == 0 else np.float64
    f, fhat, xi = _case(seed, shape, dtype, ties=seed % 3 == 0)
    g, st = mb.correct_blocks(f, fhat, xi, blocks, per_round=per_round)
    g_b, phases, lowered, critical, status = brute.slow_blocks(
        f, fhat, oracle.xi_t(dtype, xi), blocks, per_round=per_round)
    assert st["status"] == status
    assert st["phases"] == phases
    assert st["lowered"] == lowered
    assert st["critical_rounds"] == critical
    assert np.array_equal(g.view(np.uint8), g_b.view(np.uint8))


@pytest.mark.parametrize("ndim", [2, 3])
@pytest.mark.parametrize("seed", range(3))
def test_one_block_is_the_plain_correction(ndim, seed):
    shape = (9, 11) if ndim == 2 else (5, 6, 7)
    f, fhat, xi = _case(seed, shape, np.float32)
    g1, s1 = oracle.correct(f, fhat, xi)
    g, st = mb.correct_blocks(f, fhat, xi, (1, 1, 1))
    assert np.array_equal(g.view(np.uint8), g1.view(np.uint8))
    assert st["phases"] == 1 and st["lowered"] == 0
    assert st["local_rounds"] == s1["iterations"]
    assert st["steps_applied"] == s1["steps_applied"]


def test_exchange_takes_the_smallest_copy():
    # a boundary vertex held by three blocks with values 0, 1 and 2 (the
    # situation of the paper's ghost-layer figure) ends at 0 in every copy
    sl = (slice(0, 1), slice(0, 1))
    copies = [(sl, np.array([[1.0]])), (sl, np.array([[2.0]])), (sl, np.array([[0.0]]))]
    m, lowered = mb.merge((1, 1), np.float64, copies)
    assert m[0, 0] == 0.0 and lowered == 2
    assert all(a[0, 0] == 0.0 for _, a in copies)


def test_blocks_and_cores_tile_the_grid():
    for shape, blocks in CASES + [((64, 64, 64), (2, 2, 2)), ((17, 33), (4, 5))]:
        owned = np.zeros(shape, dtype=np.int32)
        for sl, core in mb.boxes(shape, blocks):
            sub = owned[sl]
            if len(shape) == 2:
                sub[core[2]:core[3], core[0]:core[1]] += 1
            else:
                sub[core[4]:core[5], core[2]:core[3], core[0]:core[1]] += 1
            # the copy reaches one vertex beyond the core wherever the grid does
            lo = [s.start for s in sl]
            hi = [s.stop for s in sl]
            cz = [(core[4], core[5]), (core[2], core[3]), (core[0], core[1])][-len(shape):]
            for a in range(len(shape)):
                assert cz[a][0] == (1 if lo[a] > 0 else 0)
                assert hi[a] - lo[a] - cz[a][1] == (1 if hi[a] < shape[a] else 0)
        assert (owned == 1).all()


def test_only_core_vertices_are_compared():
    # a mismatch seen only from outside the core causes no edit
    f = np.array([[0.0, 0.5, 1.0, 0.25]], dtype=np.float64).reshape(1, 4)
    fhat = f.copy()
    fhat[0, 3] = 0.9   # vertex 3 now beats vertex 2 as n_max of vertex 2 and 3
    lb, ub = oracle.bounds(f, 0.7)
    assert lb[0, 3] <= fhat[0, 3] <= ub[0, 3]
    g = fhat.copy()
    st = oracle.correct_core(f, g, 0.7, (0, 2, 0, 1, 0, 1))
    assert st["status"] == "OK" and st["iterations"] == 0
    g2 = fhat.copy()
    st2 = oracle.correct_core(f, g2, 0.7, (0, 4, 0, 1, 0, 1))
    assert st2["iterations"] > 0 and (g2 < fhat).any()


@pytest.mark.parametrize("blocks", [(2, 2, 2), (4, 2, 1), (3, 3, 3)])
def test_invariants_and_relaxed_needs_fewer_exchanges(blocks):
    rng = np.random.default_rng(7)
    shape = (18, 20, 22)
    f = rng.uniform(0, 1, size=shape)
    for ax in range(3):
        f = (f + np.roll(f, 1, axis=ax)) * 0.5
    f = f.astype(np.float32)
    xi = 0.02
    lb, ub = oracle.bounds(f, xi)
    fhat = (f.astype(np.float64) + rng.uniform(-xi, xi, size=shape)).astype(np.float32)
    fhat = np.minimum(np.maximum(fhat, lb), ub)
    out = {}
    for per_round in (False, True):
        g, st = mb.correct_blocks(f, fhat, xi, blocks, per_round=per_round)
        assert st["status"] == "OK"
        assert np.array_equal(oracle.directions(g), oracle.directions(f))
        assert (g <= fhat).all() and (g >= lb).all()
        out[per_round] = st
    assert out[False]["phases"] <= out[True]["phases"]
    assert out[False]["phases"] >= 2   # the exchange mattered
