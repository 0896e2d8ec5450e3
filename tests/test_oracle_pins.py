"""Pins of the CPU oracle against things other than itself.

Each test checks the oracle against what the paper and the mathematics fix:
explicit-simplex adjacency with closed-form edge counts, brute-force directions
and path-walking labels on every ordering of a 3x3 grid, exact rational
bounds, hand examples with dyadic values (tests/golden), an independent slow
correction, a library (scipy) extremum filter, and the invariants of
Sec. III-B / IV-A / IV-C on every iterate.
"""
import json
import os
from fractions import Fraction
from itertools import permutations

import numpy as np
import pytest

import brute
import oracle

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def code_to_offset(ndim, code):
    """Interface convention of the direction byte (documented in pmsz.h)."""
    if code == 0:
        return (0, 0, 0)
    m, s = code & 7, (-1 if code & 8 else 1)
    return (s * (m & 1), s * ((m >> 1) & 1), s * ((m >> 2) & 1))


def target(shape, i, code):
    if len(shape) == 2:
        ny, nx = shape
        nz = 1
    else:
        nz, ny, nx = shape
    x, y, z = i % nx, (i // nx) % ny, i // (nx * ny)
    dx, dy, dz = code_to_offset(3, code)
    return brute.vid(x + dx, y + dy, z + dz, nx, ny)


def grid_args(shape):
    if len(shape) == 2:
        return 2, shape[1], shape[0], 1
    return 3, shape[2], shape[1], shape[0]


# ---------------------------------------------------------------- mesh -------

@pytest.mark.parametrize("dims", [(2, 5, 4, 1), (2, 1, 6, 1), (2, 7, 1, 1), (3, 2, 2, 2),
                                  (3, 3, 4, 5), (3, 1, 3, 3), (3, 4, 1, 2), (3, 3, 3, 1)])
def test_simplex_edges_match_closed_form(dims):
    ndim, nx, ny, nz = dims
    adj = brute.adjacency(ndim, nx, ny, nz)
    edges = sum(len(a) for a in adj) // 2
    assert edges == brute.edge_count_closed_form(ndim, nx, ny, nz)


def test_single_cube_has_19_edges():
    adj = brute.adjacency(3, 2, 2, 2)
    assert sum(len(a) for a in adj) // 2 == 19
    assert adj[0] == set(range(1, 8))             # (0,0,0) touches every corner
    assert adj[1] == {0, 3, 5, 7}                 # (1,0,0)
    assert adj[7] == set(range(0, 7))             # (1,1,1)


@pytest.mark.parametrize("dims", [(2, 4, 3, 1), (3, 3, 3, 3), (3, 2, 3, 4), (3, 4, 2, 1)])
def test_oracle_neighbourhood_is_the_simplicial_one(dims):
    """Spike fields expose the oracle's neighbour relation: with a single 1 at j
    and 0 elsewhere, n_max(i) == j iff j is a neighbour of i (or i itself)."""
    ndim, nx, ny, nz = dims
    shape = (ny, nx) if ndim == 2 else (nz, ny, nx)
    n = nx * ny * nz
    adj = brute.adjacency(ndim, nx, ny, nz)
    for j in range(n):
        h = np.zeros(n, dtype=np.float64)
        h[j] = 1.0
        d = oracle.directions(h.reshape(shape))
        for i in range(n):
            reaches = target(shape, i, int(d.reshape(-1)[i]) & 15) == j
            assert reaches == (j == i or j in adj[i]), (i, j)


@pytest.mark.parametrize("dims", [(2, 4, 3, 1), (3, 3, 3, 3), (3, 3, 2, 4)])
def test_tie_break_by_vertex_index(dims):
    """A constant field is all ties: the larger index wins n_max, the smaller
    wins n_min."""
    ndim, nx, ny, nz = dims
    shape = (ny, nx) if ndim == 2 else (nz, ny, nx)
    n = nx * ny * nz
    adj = brute.adjacency(ndim, nx, ny, nz)
    d = oracle.directions(np.full(shape, 0.25, dtype=np.float32)).reshape(-1)
    for i in range(n):
        cand = {i} | adj[i]
        assert target(shape, i, int(d[i]) & 15) == max(cand)
        assert target(shape, i, int(d[i]) >> 4) == min(cand)


# ------------------------------------------------ directions and labels -------

def _brute_dirs_all_orderings(adj, perms):
    n = perms.shape[1]
    up = np.empty_like(perms)
    dn = np.empty_like(perms)
    for i in range(n):
        cand = np.array([i] + sorted(adj[i]))
        vals = perms[:, cand]
        up[:, i] = cand[np.argmax(vals, axis=1)]
        dn[:, i] = cand[np.argmin(vals, axis=1)]
    return up, dn


def test_every_ordering_of_3x3_grid():
    """All 9! orderings: directions against the simplicial neighbourhood and
    labels against step-by-step walks (Sec. III-A)."""
    adj = brute.adjacency(2, 3, 3)
    perms = np.array(list(permutations(range(9))), dtype=np.int64)
    up, dn = _brute_dirs_all_orderings(adj, perms)
    # labels by repeated walking, vectorised over orderings
    lab_up, lab_dn = up.copy(), dn.copy()
    rows = np.arange(len(perms))[:, None]
    for _ in range(9):
        lab_up = up[rows, lab_up]
        lab_dn = dn[rows, lab_dn]
    # the oracle, on a tall grid that stacks orderings with a separating row
    # would couple neighbours; call it per ordering in batches instead
    stride = 1
    for p in range(0, len(perms), stride):
        f = perms[p].astype(np.float32).reshape(3, 3)
        d = oracle.directions(f).reshape(-1)
        mx, mn = oracle.labels(d.reshape(3, 3))
        for i in range(9):
            assert target((3, 3), i, int(d[i]) & 15) == up[p, i]
            assert target((3, 3), i, int(d[i]) >> 4) == dn[p, i]
        assert np.array_equal(mx.reshape(-1), lab_up[p])
        assert np.array_equal(mn.reshape(-1), lab_dn[p])


@pytest.mark.parametrize("seed", range(6))
def test_random_tiny_3d_with_ties(seed):
    rng = np.random.default_rng(seed)
    nz, ny, nx = rng.integers(1, 5, size=3)
    nz = max(nz, 2)
    shape = (nz, ny, nx)
    h = rng.integers(0, 4, size=shape).astype(np.float64) * 0.5   # many ties
    adj = brute.adjacency(3, nx, ny, nz)
    d = oracle.directions(h).reshape(-1)
    mx, mn = oracle.labels(d.reshape(shape))
    flat = h.reshape(-1)
    for i in range(h.size):
        up, down = brute.steepest(flat, adj, i)
        assert target(shape, i, int(d[i]) & 15) == up
        assert target(shape, i, int(d[i]) >> 4) == down
        assert mx.reshape(-1)[i] == brute.walk(flat, adj, i, True)
        assert mn.reshape(-1)[i] == brute.walk(flat, adj, i, False)
    # labels computed on the fly from the field agree with the array labels
    idx = np.arange(h.size)
    amx, amn = oracle.labels_at(h, idx)
    assert np.array_equal(amx, mx.reshape(-1)) and np.array_equal(amn, mn.reshape(-1))


def test_extrema_match_scipy_filter():
    """Library cross-check on tie-free data: a vertex is a maximum iff it equals
    the maximum filter over the Freudenthal stencil footprint."""
    from scipy import ndimage
    rng = np.random.default_rng(7)
    h = rng.permutation(12 * 11 * 10).astype(np.float64).reshape(10, 11, 12)
    fp = np.zeros((3, 3, 3), dtype=bool)
    fp[1, 1, 1] = True
    for m in range(1, 8):
        dx, dy, dz = m & 1, (m >> 1) & 1, (m >> 2) & 1
        fp[1 + dz, 1 + dy, 1 + dx] = True
        fp[1 - dz, 1 - dy, 1 - dx] = True
    mx = ndimage.maximum_filter(h, footprint=fp, mode="constant", cval=-np.inf)
    mn = ndimage.minimum_filter(h, footprint=fp, mode="constant", cval=np.inf)
    d = oracle.directions(h)
    assert np.array_equal((d & 15) == 0, h == mx)
    assert np.array_equal((d >> 4) == 0, h == mn)


# ---------------------------------------------------------------- bounds ------

def _adversarial(dtype, rng, n):
    info = np.finfo(dtype)
    vals = list(rng.uniform(-2, 2, n).astype(dtype))
    vals += [dtype(0.0), dtype(-0.0), info.tiny, -info.tiny, info.smallest_subnormal,
             -info.smallest_subnormal, dtype(1.0), dtype(-1.0), dtype(1e-30), dtype(3.0)]
    vals += list((rng.uniform(-1, 1, n) * 10.0 ** rng.integers(-30, 10, n)).astype(dtype))
    return np.array(vals, dtype=dtype)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_bounds_are_exact_roundings(dtype):
    """lb = smallest value >= f - xi_T and ub = largest value <= f + xi_T,
    checked with exact rationals (Eq. 1 lower bound; the |f - g| <= xi bound of
    the problem statement)."""
    rng = np.random.default_rng(11)
    for xi in [0.0, 1e-4, 1e-3, 0.1, 1.0, 3e-7, 1e-20, 0.7]:
        f = _adversarial(dtype, rng, 40)
        lb, ub = oracle.bounds(f, xi)
        xt = oracle.xi_t(dtype, xi)
        for a, l, u in zip(f, lb, ub):
            assert l == brute.exact_lower(a, xt, dtype), (a, xi)
            assert u == brute.exact_upper(a, xt, dtype), (a, xi)


def test_xi_in_binary32_is_the_largest_float_not_above_xi():
    for xi in [1e-4, 1e-3, 0.1, 1.0 / 3.0, 2.0 ** -30, 1e-5 * 0.987654321, 0.0]:
        xt = oracle.xi_t(np.float32, xi)
        assert Fraction(xt) <= Fraction(xi)
        nxt = np.nextafter(np.float32(xt), np.float32(np.inf))
        assert Fraction(float(nxt)) > Fraction(xi)
        assert np.float32(xt) == xt
    assert oracle.xi_t(np.float64, 0.1) == 0.1


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_edit_halves_the_gap(dtype):
    """Eq. 1 with delta = half the remaining gap: the result never goes below
    the lower bound, strictly decreases a value above it, leaves a value at it
    unchanged, and sits within one unit in the last place of the midpoint."""
    rng = np.random.default_rng(3)
    f = _adversarial(dtype, rng, 200)
    lb, _ = oracle.bounds(f, 1e-3)
    gap = (rng.uniform(0, 1, f.size) * 2e-3).astype(dtype)
    g = np.maximum(lb, lb + gap).astype(dtype)
    g[::7] = lb[::7]
    g[1::11] = np.nextafter(lb[1::11], dtype(np.inf))
    e = oracle.edit(g, lb)
    for gi, li, ei in zip(g, lb, e):
        assert ei >= li
        if gi > li:
            assert ei < gi
            mid = (Fraction(float(gi)) + Fraction(float(li))) / 2
            ulp = Fraction(float(np.spacing(np.abs(ei)))) if ei != 0 else Fraction(
                float(np.finfo(dtype).smallest_subnormal))
            assert abs(Fraction(float(ei)) - mid) <= ulp
        else:
            assert ei == li


# ------------------------------------------------------- hand examples -------

def _cases():
    with open(os.path.join(GOLDEN, "hand_examples.json")) as fh:
        return json.load(fh)["cases"]


@pytest.mark.parametrize("case", _cases(), ids=lambda c: c["name"])
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_hand_examples(case, dtype):
    if case.get("dtype") and np.dtype(case["dtype"]) != np.dtype(dtype):
        pytest.skip("case is specific to " + case["dtype"])
    shape = (case["ny"], case["nx"])
    f = np.array(case["f"], dtype=dtype).reshape(shape)
    if case["fhat"] == "lower_bound":
        fhat, _ = oracle.bounds(f, case["xi"])
    else:
        fhat = np.array(case["fhat"], dtype=dtype).reshape(shape)
    flags, _ = oracle.flags(fhat, oracle.directions(f))
    assert sorted(np.flatnonzero(flags).tolist()) == case["flags_at_k0"]
    g, st = oracle.correct(f, fhat, case["xi"])
    assert st["status"] == case["status"]
    assert st["iterations"] == case["iterations"]
    if "g_final" in case:
        assert g.reshape(-1).tolist() == case["g_final"]
        mx, mn = oracle.labels(oracle.directions(g))
        assert mx.reshape(-1).tolist() == case["max_label"]
        assert mn.reshape(-1).tolist() == case["min_label"]


# ------------------------------------- independent slow correction ----------

def _tiny_case(seed, ndim, dtype, ties):
    rng = np.random.default_rng(seed)
    if ndim == 2:
        shape = (int(rng.integers(2, 6)), int(rng.integers(2, 7)))
    else:
        shape = tuple(int(v) for v in rng.integers(2, 5, size=3))
    if ties:
        f = (rng.integers(0, 6, size=shape) * 0.125).astype(dtype)
    else:
        f = rng.uniform(0, 1, size=shape).astype(dtype)
    xi = float(rng.choice([0.05, 0.1, 0.3]))
    lb, ub = oracle.bounds(f, xi)
    t = rng.uniform(0, 1, size=shape)
    fhat = (lb.astype(np.float64) + t * (ub.astype(np.float64) - lb)).astype(dtype)
    fhat = np.minimum(np.maximum(fhat, lb), ub)
    if ties:
        fhat[rng.uniform(size=shape) < 0.3] = dtype(0.25)
        fhat = np.minimum(np.maximum(fhat, lb), ub)
    return f, fhat, xi


@pytest.mark.parametrize("seed", range(12))
@pytest.mark.parametrize("ndim", [2, 3])
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_oracle_matches_slow_correction(seed, ndim, dtype):
    f, fhat, xi = _tiny_case(seed, ndim, dtype, ties=seed % 2 == 0)
    args = grid_args(f.shape)
    adj = brute.adjacency(*args)
    g_slow, k_slow, st_slow = brute.slow_correct(f, fhat, oracle.xi_t(dtype, xi), adj)
    g, st = oracle.correct(f, fhat, xi)
    assert st["status"] == st_slow
    assert st["iterations"] == k_slow
    assert np.array_equal(g.view(np.uint8), g_slow.view(np.uint8))


# ------------------------------------------------------------ invariants -----

def _invariant_case(ndim, dtype, seed):
    rng = np.random.default_rng(seed)
    if ndim == 3:
        shape = (10, 11, 12)
    else:
        shape = (40, 37)
    f = rng.uniform(0, 1, size=shape).astype(dtype)
    f = (f + np.roll(f, 1, axis=-1)) * 0.5     # some smoothness
    f = f.astype(dtype)
    xi = 0.05
    lb, ub = oracle.bounds(f, xi)
    fhat = (f.astype(np.float64) + rng.uniform(-xi, xi, size=shape)).astype(dtype)
    fhat = np.minimum(np.maximum(fhat, lb), ub)
    return f, fhat, xi, lb, ub


@pytest.mark.parametrize("ndim", [2, 3])
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_invariants_on_every_iterate(ndim, dtype):
    """Sec. III-B / IV-C: values only decrease and stay within the bound; edits
    happen only at flagged vertices (flags recomputed by brute force); at
    convergence the directions, extrema and labels of f are restored; more
    iterations do not change a converged field; resuming from g^k gives the
    same result (the iterate depends only on f and g^k)."""
    f, fhat, xi, lb, ub = _invariant_case(ndim, dtype, 5)
    args = grid_args(f.shape)
    adj = brute.adjacency(*args)
    flat_f = f.reshape(-1)
    dirs_f = [brute.steepest(flat_f, adj, i) for i in range(f.size)]
    g_final, st = oracle.correct(f, fhat, xi)
    assert st["status"] == "OK" and st["iterations"] > 1
    prev = fhat
    for k in range(1, st["iterations"] + 1):
        gk, sk = oracle.correct(f, fhat, xi, max_iters=k)
        assert sk["iterations"] == k
        assert np.all(gk <= prev) and np.all(gk >= lb) and np.all(gk <= ub)
        # brute-force flag set of the previous iterate
        pf = prev.reshape(-1)
        targets = set()
        for i in range(f.size):
            up, down = brute.steepest(pf, adj, i)
            if up != dirs_f[i][0]:
                targets.add(up)
            if down != dirs_f[i][1]:
                targets.add(dirs_f[i][1])
        changed = set(np.flatnonzero(gk.reshape(-1) != pf).tolist())
        assert changed <= targets
        # resume from g^k
        g_res, st_res = oracle.correct(f, gk, xi)
        assert np.array_equal(g_res, g_final)
        assert st_res["iterations"] == st["iterations"] - k
        prev = gk
    rep = oracle.verify(f, g_final, fhat, xi)
    for key in ("bound_violations", "asc_mismatch", "desc_mismatch", "false_max", "false_min",
                "missed_max", "missed_min", "wrong_max_label", "wrong_min_label", "wrong_label"):
        assert rep[key] == 0, key
    g2, st2 = oracle.correct(f, g_final, xi)
    assert st2["iterations"] == 0 and np.array_equal(g2, g_final)
    # labels by explicit walks
    mx, mn = oracle.labels(oracle.directions(g_final))
    for i in range(0, f.size, 7):
        assert mx.reshape(-1)[i] == brute.walk(flat_f, adj, i, True)
        assert mn.reshape(-1)[i] == brute.walk(flat_f, adj, i, False)


def test_verify_counts_against_brute_force():
    f, fhat, xi, lb, ub = _invariant_case(3, np.float32, 9)
    adj = brute.adjacency(*grid_args(f.shape))
    rep = oracle.verify(f, fhat, None, xi)
    ff, gg = f.reshape(-1), fhat.reshape(-1)
    cnt = dict(asc=0, desc=0, fmax=0, fmin=0, mmax=0, mmin=0, wl=0)
    for i in range(f.size):
        uf, df = brute.steepest(ff, adj, i)
        ug, dg = brute.steepest(gg, adj, i)
        cnt["asc"] += uf != ug
        cnt["desc"] += df != dg
        cnt["fmax"] += (ug == i and uf != i)
        cnt["mmax"] += (uf == i and ug != i)
        cnt["fmin"] += (dg == i and df != i)
        cnt["mmin"] += (df == i and dg != i)
        if i % 5 == 0:
            cnt["wl"] += (brute.walk(ff, adj, i, True) != brute.walk(gg, adj, i, True)
                          or brute.walk(ff, adj, i, False) != brute.walk(gg, adj, i, False))
    assert rep["asc_mismatch"] == cnt["asc"] and rep["desc_mismatch"] == cnt["desc"]
    assert rep["false_max"] == cnt["fmax"] and rep["missed_max"] == cnt["mmax"]
    assert rep["false_min"] == cnt["fmin"] and rep["missed_min"] == cnt["mmin"]
    assert rep["asc_mismatch"] > 0
    mxf, mnf = oracle.labels(oracle.directions(f))
    mxg, mng = oracle.labels(oracle.directions(fhat))
    wrong = (mxf != mxg) | (mnf != mng)
    assert rep["wrong_label"] == int(wrong.sum())
    assert int(wrong.reshape(-1)[::5].sum()) == cnt["wl"]
    assert rep["vertices_edited"] == -1
    assert rep["max_abs_err"] == float(np.max(np.abs(fhat.astype(np.float64) - f)))


# ----------------------------------------------------------- special cases ---

def test_special_cases():
    rng = np.random.default_rng(2)
    f = rng.uniform(0, 1, size=(6, 7, 8)).astype(np.float32)
    # fhat == f: nothing to do
    g, st = oracle.correct(f, f, 1e-3)
    assert st["status"] == "OK" and st["iterations"] == 0 and st["mismatch_initial"] == 0
    # xi == 0 forces fhat == f
    assert oracle.validate(f, f, 0.0) == "OK"
    bumped = f.copy()
    bumped[0, 0, 0] = np.nextafter(bumped[0, 0, 0], np.float32(2))
    assert oracle.validate(f, bumped, 0.0) == "INPUT_BOUND"
    # non-finite input
    bad = f.copy()
    bad[1, 2, 3] = np.nan
    assert oracle.validate(f, bad, 1e-3) == "NONFINITE"
    _, st = oracle.correct(f, bad, 1e-3)
    assert st["status"] == "NONFINITE"
    # a ramp has one maximum (last vertex) and one minimum (vertex 0)
    ramp = np.arange(5 * 6 * 7, dtype=np.float64).reshape(5, 6, 7)
    mx, mn = oracle.labels(oracle.directions(ramp))
    assert np.all(mx == ramp.size - 1) and np.all(mn == 0)
    # a single radial bump labels everything with its peak
    z, y, x = np.meshgrid(np.arange(9), np.arange(9), np.arange(9), indexing="ij")
    bump = -((x - 4.3) ** 2 + (y - 3.9) ** 2 + (z - 4.1) ** 2)
    mx, _ = oracle.labels(oracle.directions(bump))
    assert np.all(mx == brute.vid(4, 4, 4, 9, 9))
    # max_iters = 0 reports NOT_CONVERGED without editing
    f2, fhat2, xi2, _, _ = _invariant_case(2, np.float64, 1)
    g0, st0 = oracle.correct(f2, fhat2, xi2, max_iters=0)
    assert st0["status"] == "NOT_CONVERGED" and np.array_equal(g0, fhat2)
    # a negative error bound is invalid
    assert oracle.validate(f, f, -1.0) == "INVALID_ARG"


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_crafted_stall_case(dtype):
    """Reading A9: rounding can merge the lower bounds of two distinct values.
    f = (b, a) with b the next value above a (the maximum at the smaller
    index), xi = 1: both lower bounds are the smallest value at or above
    a - 1 (a is tiny), so once the spurious maximum (vertex 1) reaches it, the
    index tie-break still makes vertex 1 the maximum and vertex 0 the minimum,
    both rules keep flagging vertex 1, which sits at its bound: STALLED, with
    g at the merged bound on both vertices."""
    a = dtype(1e-20)
    f = np.array([[np.nextafter(a, dtype(1)), a]], dtype=dtype)
    lb, _ = oracle.bounds(f, 1.0)
    assert lb[0, 0] == lb[0, 1] and lb[0, 0] > dtype(-1)
    fhat = np.array([[lb[0, 0], 0.0]], dtype=dtype)
    g, st = oracle.correct(f, fhat, 1.0)
    assert st["status"] == "STALLED"
    assert st["flagged_final"] == 1 and st["stalled_flags"] == 1
    assert g[0, 0] == lb[0, 0] and g[0, 1] == lb[0, 1]
    # the independent loop agrees, value for value
    adj = brute.adjacency(2, 2, 1)
    g_slow, k_slow, st_slow = brute.slow_correct(f, fhat, oracle.xi_t(dtype, 1.0), adj)
    assert st_slow == "STALLED" and k_slow == st["iterations"]
    assert np.array_equal(g_slow.view(np.uint8), g.view(np.uint8))


# ---------------------------------------------- targeted-edit variant --------
# Each flagged vertex is lowered to the highest value at which it no longer
# beats its rival (the worked examples of Sec. IV-A lower a spurious maximum to
# its rival's value "or slightly below"), the smallest such value over its
# flaggers, never below its bound.

@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_targeted_ascending_example(dtype):
    """f = [0, 1, 0.5], fhat = [0, 0.75, 1.0], xi = 0.5: vertex 2 is a spurious
    maximum; it drops to the value just below its rival's 0.75 (index 2 > 1,
    so an equal value would still win) in one iteration."""
    f = np.array([[0, 1, 0.5]], dtype)
    fh = np.array([[0, 0.75, 1.0]], dtype)
    g, st = oracle.correct(f, fh, 0.5, mode="targeted")
    assert st["status"] == "OK" and st["iterations"] == 1 and st["steps_applied"] == 1
    assert g[0, 2] == np.nextafter(dtype(0.75), dtype(-np.inf))
    assert g[0, 0] == 0 and g[0, 1] == dtype(0.75)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_targeted_tie_goes_to_the_rival(dtype):
    """f = [0, 0.25, 1], fhat = [0.375, 0.125, 1], xi = 0.5: vertex 0 is both a
    false maximum (rival 1) and the original minimum pushed above vertex 1;
    index 0 < 1, so the rival's own value 0.125 already settles both ties."""
    f = np.array([[0, 0.25, 1]], dtype)
    fh = np.array([[0.375, 0.125, 1]], dtype)
    flags, prop, m = oracle.flags_targeted(fh, oracle.directions(f))
    assert np.flatnonzero(flags).tolist() == [0] and prop[0, 0] == 0.125
    g, st = oracle.correct(f, fh, 0.5, mode="targeted")
    assert st["status"] == "OK" and st["iterations"] == 1
    assert g.reshape(-1).tolist() == [0.125, 0.125, 1.0]
    assert np.array_equal(oracle.directions(g), oracle.directions(f))


@pytest.mark.parametrize("seed", range(10))
@pytest.mark.parametrize("ndim", [2, 3])
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_targeted_oracle_matches_slow_correction(seed, ndim, dtype):
    f, fhat, xi = _tiny_case(100 + seed, ndim, dtype, ties=seed % 2 == 0)
    adj = brute.adjacency(*grid_args(f.shape))
    g_slow, k_slow, st_slow = brute.slow_correct(f, fhat, oracle.xi_t(dtype, xi), adj,
                                                 mode="targeted")
    g, st = oracle.correct(f, fhat, xi, mode="targeted")
    assert st["status"] == st_slow
    assert st["iterations"] == k_slow
    assert np.array_equal(g.view(np.uint8), g_slow.view(np.uint8))


@pytest.mark.parametrize("ndim", [2, 3])
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_targeted_invariants(ndim, dtype):
    """Monotone, within bounds, edits only at flagged vertices, directions of f
    restored at convergence; and on this input no more iterations than the
    halving edit needs."""
    f, fhat, xi, lb, ub = _invariant_case(ndim, dtype, 9)
    g_final, st = oracle.correct(f, fhat, xi, mode="targeted")
    assert st["status"] == "OK"
    prev = fhat
    dirs_f = oracle.directions(f)
    for k in range(1, st["iterations"] + 1):
        gk, _ = oracle.correct(f, fhat, xi, max_iters=k, mode="targeted")
        assert np.all(gk <= prev) and np.all(gk >= lb) and np.all(gk <= ub)
        flags, _ = oracle.flags(prev, dirs_f)
        assert np.all(flags.astype(bool) | (gk == prev))
        prev = gk
    assert np.array_equal(oracle.directions(g_final), dirs_f)
    _, st_half = oracle.correct(f, fhat, xi)
    assert st["iterations"] <= st_half["iterations"]


# -------------------------------------------------- sampled-checker pins -----

def _boundary_and_random(shape, rng, extra):
    """Every vertex on a face, edge or corner of the box, plus `extra` random
    interior ones."""
    idx = np.arange(int(np.prod(shape))).reshape(shape)
    on = np.zeros(shape, dtype=bool)
    for ax in range(len(shape)):
        sl = [slice(None)] * len(shape)
        sl[ax] = 0
        on[tuple(sl)] = True
        sl[ax] = -1
        on[tuple(sl)] = True
    pick = idx[on].tolist() + rng.integers(0, idx.size, size=extra).tolist()
    return np.array(pick, dtype=np.int64)


@pytest.mark.parametrize("shape", [(7, 13), (1, 9), (5, 1), (4, 5, 6), (3, 1, 7), (2, 9, 1),
                                   (6, 5, 11)])
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_directions_at_matches_the_whole_field(shape, dtype):
    """orc_directions_at (the sampled checker of the large fields) at every
    face, edge and corner vertex and at random interior ones: equal to the
    direction bytes of the whole field and to the brute-force argmax / argmin
    over the simplicial neighbourhood (Sec. IV-A n_max / n_min)."""
    rng = np.random.default_rng(sum(shape) * 7 + (dtype == np.float64))
    f = rng.integers(0, 6, size=shape).astype(dtype)  # tie-heavy
    idx = _boundary_and_random(shape, rng, 40)
    at = oracle.directions_at(f, idx)
    full = oracle.directions(f).reshape(-1)
    assert np.array_equal(at, full[idx])
    adj = brute.adjacency(*grid_args(shape))
    flat = f.reshape(-1)
    for k, i in enumerate(idx.tolist()):
        up, down = brute.steepest(flat, adj, i)
        assert target(shape, i, int(at[k]) & 15) == up
        assert target(shape, i, int(at[k]) >> 4) == down


def _label_case(seed):
    """A tiny 3D field f and a perturbed copy g whose ascending and descending
    label errors differ in number."""
    rng = np.random.default_rng(seed)
    shape = (4, 5, 6)
    f = rng.uniform(0.0, 1.0, size=shape)
    g = f.copy()
    flat = g.reshape(-1)
    k = rng.integers(1, 4)
    where = rng.choice(flat.size, size=k, replace=False)
    flat[where] += rng.choice([-1.0, 1.0], size=k) * rng.uniform(0.2, 0.6, size=k)
    return f, g


def test_verify_label_split_and_edited_count_against_walks():
    """Sec. III-A segmentations, Sec. V-D counts: wrong_max_label counts the
    vertices whose ascending integral line ends at another maximum,
    wrong_min_label those whose descending line ends at another minimum,
    found here by explicit walks; vertices_edited counts the vertices where g
    differs from fhat, first and last vertex included."""
    found = 0
    for seed in range(200):
        f, g = _label_case(seed)
        adj = brute.adjacency(*grid_args(f.shape))
        ff, gg = f.reshape(-1), g.reshape(-1)
        up = sum(brute.walk(ff, adj, i, True) != brute.walk(gg, adj, i, True)
                 for i in range(ff.size))
        dn = sum(brute.walk(ff, adj, i, False) != brute.walk(gg, adj, i, False)
                 for i in range(ff.size))
        if up == dn or min(up, dn) == 0:
            continue
        # fhat: g with a known set of vertices moved, both ends of the array
        # among them; the others keep g's bits
        fhat = g.copy()
        moved = np.array([0, 7, 33, ff.size - 1])
        fhat.reshape(-1)[moved] += 1e-3
        rep = oracle.verify(f, g, fhat, 10.0)
        assert rep["wrong_max_label"] == up
        assert rep["wrong_min_label"] == dn
        assert rep["vertices_edited"] == moved.size
        rep2 = oracle.verify(f, g, g, 10.0)
        assert rep2["vertices_edited"] == 0
        found += 1
        if found == 3:
            break
    assert found == 3, "no case with differing ascending / descending label errors"
