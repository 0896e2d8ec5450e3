"""Slow, independent checks for tiny grids -- used only to pin the oracle.

Nothing here is shared with the oracle or the GPU library.  Adjacency is derived
from explicit simplices (the Kuhn split of each cube into six tetrahedra, one
per ordering of the axes, and of each square into two triangles), not from an
offset table; labels are found by walking integral lines one step at a time;
bounds are checked with exact rationals.
"""
from fractions import Fraction
from itertools import permutations

import numpy as np


def vid(x, y, z, nx, ny):
    return x + nx * (y + ny * z)


def adjacency(ndim, nx, ny, nz=1):
    """Vertex -> set of mesh neighbours, from the edges of every top simplex of
    the Freudenthal triangulation.  A simplex walks from a cell's lowest corner
    to its highest corner adding one unit vector at a time, in the order given
    by a permutation of the axes (Sec. III-A: PL function on a triangular /
    tetrahedral mesh).  A grid one vertex thick along an axis has no cells
    along it; its edges come from the same split of the remaining axes."""
    n = nx * ny * nz
    adj = [set() for _ in range(n)]
    dims = [nx, ny, nz] if ndim == 3 else [nx, ny]
    live = [a for a, d in enumerate(dims) if d > 1]
    # cells span the live axes only
    ranges = [range(d - 1) if d > 1 else range(1) for d in dims]
    for cell in np.ndindex(*[len(r) for r in ranges]):
        base = list(cell) + ([0] if ndim == 2 else [])
        for perm in permutations(live):
            p = list(base) if ndim == 3 else base[:2] + [0]
            verts = [vid(p[0], p[1], p[2], nx, ny)]
            for a in perm:
                p[a] += 1
                verts.append(vid(p[0], p[1], p[2], nx, ny))
            for u in verts:
                for v in verts:
                    if u != v:
                        adj[u].add(v)
    return adj


def edge_count_closed_form(ndim, nx, ny, nz=1):
    if ndim == 2:
        return (nx - 1) * ny + nx * (ny - 1) + (nx - 1) * (ny - 1)
    return ((nx - 1) * ny * nz + nx * (ny - 1) * nz + nx * ny * (nz - 1)
            + (nx - 1) * (ny - 1) * nz + (nx - 1) * ny * (nz - 1) + nx * (ny - 1) * (nz - 1)
            + (nx - 1) * (ny - 1) * (nz - 1))


def steepest(vals, adj, i):
    """(n_max(i), n_min(i)) over {i} + neighbours; ties by vertex index."""
    cand = [i] + sorted(adj[i])
    up = max(cand, key=lambda j: (vals[j], j))
    down = min(cand, key=lambda j: (vals[j], j))
    return up, down


def walk(vals, adj, i, ascending=True):
    while True:
        up, down = steepest(vals, adj, i)
        nxt = up if ascending else down
        if nxt == i:
            return i
        i = nxt


def rational(x):
    return Fraction(float(x)) if not isinstance(x, Fraction) else x


def exact_lower(f, xi_t, dtype):
    """Smallest value of dtype that is >= f - xi_t, found by exact rationals."""
    target = rational(f) - rational(xi_t)
    t = dtype(float(target))  # nearest, then fix up
    while rational(t) < target:
        t = np.nextafter(t, dtype(np.inf))
    while True:
        p = np.nextafter(t, dtype(-np.inf))
        if rational(p) >= target:
            t = p
        else:
            return t


def exact_upper(f, xi_t, dtype):
    target = rational(f) + rational(xi_t)
    t = dtype(float(target))
    while rational(t) > target:
        t = np.nextafter(t, dtype(-np.inf))
    while True:
        p = np.nextafter(t, dtype(np.inf))
        if rational(p) <= target:
            t = p
        else:
            return t


def beats(vals, a, b):
    """(value, index) order: a above b."""
    return vals[a] > vals[b] or (vals[a] == vals[b] and a > b)


def slow_correct(f, fhat, xi_t, adj, max_iters=10 ** 6, mode="halving", core=None):
    """Reference correction loop written from the rules of Sec. IV-A, in the
    field's own numpy scalar type.  Returns (g, iterations, status).
    core: the set of vertex ids that are compared (all when None); the
    vertices they flag may lie outside it.
    mode "targeted": each target is lowered to the highest value at which it
    no longer beats its rival (found here by stepping down value by value from
    the rival's value), the smallest such value over its flaggers, never below
    its bound."""
    dt = f.dtype.type
    fl = f.reshape(-1)
    g = fhat.reshape(-1).copy()
    n = fl.size
    lb = [exact_lower(fl[i], xi_t, dt) for i in range(n)]
    dir_f = [steepest(fl, adj, i) for i in range(n)]
    k = 0
    while True:
        targets = set()
        for i in range(n):
            if core is not None and i not in core:
                continue
            up, down = steepest(g, adj, i)
            if up != dir_f[i][0]:
                targets.add(up)          # spurious maximum / false maximum
            if down != dir_f[i][1]:
                targets.add(dir_f[i][1])  # original minimum must be lowered
        if not targets:
            return g.reshape(f.shape), k, "OK"
        if all(g[t] == lb[t] for t in targets):
            return g.reshape(f.shape), k, "STALLED"
        if k == max_iters:
            return g.reshape(f.shape), k, "NOT_CONVERGED"
        new = g.copy()
        if mode == "targeted":
            best = {}
            for i in range(n):
                if core is not None and i not in core:
                    continue
                up, down = steepest(g, adj, i)
                pairs = []
                if up != dir_f[i][0]:
                    pairs.append((up, dir_f[i][0]))
                if down != dir_f[i][1]:
                    pairs.append((dir_f[i][1], down))
                for t, rival in pairs:
                    # highest candidate value v with (v, t) below (g[rival], rival)
                    v = g[rival]
                    trial = g.copy()
                    trial[t] = v
                    while beats(trial, t, rival):
                        v = np.nextafter(v, dt(-np.inf))
                        trial[t] = v
                    if v == 0:
                        v = dt(0.0)
                    if t not in best or v < best[t]:
                        best[t] = v
            for t in targets:
                new[t] = best[t] if best[t] > lb[t] else lb[t]
        else:
            for t in targets:
                half = dt(0.5) * (g[t] - lb[t])
                m = lb[t] + half
                new[t] = m if m < g[t] else lb[t]
        g = new
        k += 1


def slow_blocks(f, fhat, xi_t, blocks, per_round=False, max_phases=1000):
    """The decomposed correction of Sec. IV-B on a tiny grid, written out with
    explicit vertex lists: every block copies its core plus the vertices one
    step outside it (its ghost layer), corrects the copy comparing core
    vertices only, then every vertex takes the smallest value among its
    copies.  Block k of an axis of n vertices cut b ways owns
    [k n // b, (k+1) n // b).  Returns (g, phases, lowered, critical rounds,
    status)."""
    ndim = f.ndim
    dims = list(reversed(f.shape))  # nx, ny[, nz]
    nb = list(blocks[:ndim])
    owned = []
    for n, b in zip(dims, nb):
        owned.append([list(range(k * n // b, (k + 1) * n // b)) for k in range(b)])
    flat_f = f.reshape(-1)
    g = fhat.reshape(-1).copy()
    nx, ny = dims[0], dims[1]
    blocks_list = []
    for combo in np.ndindex(*reversed(nb)):
        ks = list(reversed(combo))  # kx, ky[, kz]
        ranges = []
        core_ranges = []
        for a in range(ndim):
            own = owned[a][ks[a]]
            lo, hi = max(own[0] - 1, 0), min(own[-1] + 2, dims[a])
            ranges.append(list(range(lo, hi)))
            core_ranges.append(set(own))
        local = []   # global ids of the copy, in local id order (x fastest)
        core = set()
        zr = ranges[2] if ndim == 3 else [0]
        for z in zr:
            for y in ranges[1]:
                for x in ranges[0]:
                    lid = len(local)
                    local.append(vid(x, y, z, nx, ny))
                    if x in core_ranges[0] and y in core_ranges[1] and \
                            (ndim == 2 or z in core_ranges[2]):
                        core.add(lid)
        shape = (len(zr), len(ranges[1]), len(ranges[0]))
        adj = adjacency(ndim, shape[2], shape[1], shape[0])
        blocks_list.append((local, core, shape, adj))
    copies = [np.array([g[i] for i in local], dtype=f.dtype) for local, _, _, _ in blocks_list]
    lfs = [np.array([flat_f[i] for i in local], dtype=f.dtype) for local, _, _, _ in blocks_list]
    phases = lowered_total = critical = 0
    while phases < max_phases:
        results = []
        changed = False
        for b, (local, core, shape, adj) in enumerate(blocks_list):
            before = copies[b].copy()
            gb, k, status = slow_correct(lfs[b], copies[b], xi_t, adj,
                                         max_iters=1 if per_round else 10 ** 6, core=core)
            copies[b] = gb.reshape(-1).copy()
            changed |= bool((copies[b] != before).any())
            results.append((k, status))
        # exchange: smallest copy of every vertex, everywhere
        best = {}
        for b, (local, _, _, _) in enumerate(blocks_list):
            for lid, gid in enumerate(local):
                v = copies[b][lid]
                if gid not in best or v < best[gid]:
                    best[gid] = v
        lowered = 0
        for b, (local, _, _, _) in enumerate(blocks_list):
            for lid, gid in enumerate(local):
                if copies[b][lid] > best[gid]:
                    lowered += 1
                    copies[b][lid] = best[gid]
        for gid, v in best.items():
            g[gid] = v
        phases += 1
        lowered_total += lowered
        critical += max(k for k, _ in results)
        if all(st == "OK" for _, st in results) and lowered == 0:
            return g.reshape(f.shape), phases, lowered_total, critical, "OK"
        if not changed and lowered == 0:
            st = "STALLED" if any(st == "STALLED" for _, st in results) else "NOT_CONVERGED"
            return g.reshape(f.shape), phases, lowered_total, critical, st
    return g.reshape(f.shape), phases, lowered_total, critical, "NOT_CONVERGED"
