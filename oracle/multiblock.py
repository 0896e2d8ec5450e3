"""Decomposed-domain correction (Sec. IV-B) -- TEST INFRASTRUCTURE ONLY.

The domain is cut into non-overlapping blocks; each block holds its core plus
a one-vertex ghost layer copied from its neighbours (Sec. IV-B, domain
decomposition).  A phase runs the local correction of every block on its own
copy (only core vertices are compared; a flag may lower a ghost copy), then
synchronises: every vertex held by several blocks takes the minimum of its
copies, in all of them (Sec. IV-B, ghost layer synchronisation; values only
ever decrease, so the process converges, Sec. IV-C).

Two schedules (Sec. IV-B, relaxed synchronisation):
  relaxed  -- each block runs to local convergence before the exchange (pMSz);
  per-round -- one edit round per block between exchanges (sync-pMSz).

Readings (the paper gives no more detail): along an axis of n vertices cut
into b blocks, block k owns [floor(k n / b), floor((k+1) n / b)); its copy
spans one more vertex on each side that has a neighbour block.  The loop ends
with OK when every block's last check found no mismatch and the exchange
lowered no copy; with STALLED (or NOT_CONVERGED, when a block stopped at its
round limit) when a phase changed no value at all; with NOT_CONVERGED after
max_phases phases.
"""
import numpy as np

from . import correct_core, directions


def cuts(n, b):
    """Block starts along one axis: [floor(k n / b) for k = 0..b]."""
    return [k * n // b for k in range(b + 1)]


def boxes(shape, blocks):
    """Blocks of a field shaped (ny, nx) or (nz, ny, nx), numbered
    kx + bx (ky + by kz).  Each entry: (slices of the copied box in the
    field, core box (x0, x1, y0, y1, z0, z1) in the copy's coordinates)."""
    dims = tuple(reversed(shape))  # (nx, ny[, nz])
    bl = tuple(blocks[:len(dims)])
    per_axis = []
    for n, b in zip(dims, bl):
        c = cuts(n, b)
        axis = []
        for k in range(b):
            lo, hi = max(c[k] - 1, 0), min(c[k + 1] + 1, n)
            axis.append((lo, hi, c[k] - lo, c[k + 1] - lo))
        per_axis.append(axis)
    out = []
    if len(dims) == 2:
        for ky in range(bl[1]):
            for kx in range(bl[0]):
                X, Y = per_axis[0][kx], per_axis[1][ky]
                out.append(((slice(Y[0], Y[1]), slice(X[0], X[1])),
                            (X[2], X[3], Y[2], Y[3], 0, 1)))
    else:
        for kz in range(bl[2]):
            for ky in range(bl[1]):
                for kx in range(bl[0]):
                    X, Y, Z = per_axis[0][kx], per_axis[1][ky], per_axis[2][kz]
                    out.append(((slice(Z[0], Z[1]), slice(Y[0], Y[1]), slice(X[0], X[1])),
                                (X[2], X[3], Y[2], Y[3], Z[2], Z[3])))
    return out


def merge(shape, dtype, copies):
    """Ghost layer synchronisation: every vertex takes the minimum over the
    blocks that hold a copy of it, and every copy is set to that minimum.
    copies: list of (slices, array).  Returns (merged field, copies lowered)."""
    m = np.full(shape, np.inf, dtype=dtype)
    for sl, a in copies:
        m[sl] = np.minimum(m[sl], a)
    lowered = 0
    for sl, a in copies:
        lowered += int(np.count_nonzero(a > m[sl]))
        a[...] = m[sl]
    return m, lowered


def correct_blocks(f, fhat, xi, blocks, per_round=False, max_phases=1 << 20,
                   max_iters=1 << 40):
    """Run the decomposed correction; returns (g, stats).  blocks = (bx, by)
    or (bx, by, bz).  stats: status, phases (exchanges), local_rounds (edit
    rounds summed over blocks and phases), critical_rounds (per phase the
    most rounds of any block, summed: the schedule's length when every block
    has a GPU of its own), lowered (copies lowered by the exchanges),
    steps_applied (value changes by the local corrections)."""
    f = np.ascontiguousarray(f)
    bx = boxes(f.shape, blocks)
    lf = [np.array(f[sl], copy=True, order="C") for sl, _ in bx]
    lg = [np.array(fhat[sl], dtype=f.dtype, copy=True, order="C") for sl, _ in bx]
    ld = [directions(a) for a in lf]
    st = {"status": "OK", "phases": 0, "local_rounds": 0, "critical_rounds": 0,
          "lowered": 0, "steps_applied": 0}
    cap = 1 if per_round else max_iters
    g = np.array(fhat, dtype=f.dtype, copy=True)
    while True:
        if st["phases"] == max_phases:
            st["status"] = "NOT_CONVERGED"
            break
        res = [correct_core(lf[b], lg[b], xi, bx[b][1], max_iters=cap, dirs_f=ld[b])
               for b in range(len(bx))]
        for r in res:
            if r["status"] in ("NONFINITE", "INPUT_BOUND", "INVALID_ARG", "OOM"):
                st["status"] = r["status"]
                return np.array(fhat, dtype=f.dtype, copy=True), st
        g, lowered = merge(f.shape, f.dtype, [(bx[b][0], lg[b]) for b in range(len(bx))])
        steps = sum(r["steps_applied"] for r in res)
        st["phases"] += 1
        st["local_rounds"] += sum(r["iterations"] for r in res)
        st["critical_rounds"] += max(r["iterations"] for r in res)
        st["lowered"] += lowered
        st["steps_applied"] += steps
        if all(r["status"] == "OK" for r in res) and lowered == 0:
            break
        if steps == 0 and lowered == 0:
            st["status"] = ("STALLED" if any(r["status"] == "STALLED" for r in res)
                            else "NOT_CONVERGED")
            break
    return g, st
