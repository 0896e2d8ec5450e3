"""Benchmark of the pMSz correction on one MI355X.

A step is one full correction (pmsz_correct: directions of f, validation of
fhat, every detect/apply round until convergence) of the 512^3 binary32
Perlin workload (6 octaves, 8 lattice cells, eps = 1e-4 of the unit range,
seed 512): one GPU's share of the paper's weak-scaling study.  Inputs are
resident in HBM before timing starts; every timed step corrects its own copy
of fhat.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Gvoxels/s corrected at 512^3 fp32 ε=1e-4; batched vs plain; serve p50/p99 ms"
HBM_PEAK_GBS = 8000.0
ENGINE_SOURCES = ["engine.hip", "engine.hpp", "tiles.hpp", "common.hpp"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "engine_perlin512_f32_traffic.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_hash():
    h = hashlib.sha256()
    for name in ENGINE_SOURCES:
        with open(os.path.join(ROOT, "paper_2601_01787_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def algorithmic_bytes(voxels, swept, edits, s):
    """Bytes the method must move (per-unit figures): once per vertex f and fhat
    read and its direction byte written (2s+1); per vertex examined by a later
    detect pass g and the direction byte read and a flag bit written
    (s + 1 + 1/8); per edit f and g read and g written (3s)."""
    return voxels * (2 * s + 1) + max(swept - voxels, 0) * (s + 1.125) + edits * 3 * s


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    runs, if they were taken on the current source."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as fh:
        t = json.load(fh)
    if t.get("source_hash") != source_hash():
        return None
    return t.get("bytes_per_launch", {}).get(kernel)


def kernel_split(tm, rounds, s):
    """Per kernel of one correction: (total ms, launches, algorithmic bytes).
    The directions kernel reads f and writes the direction bytes (s + 1 per
    vertex).  Round 0's detection reads fhat, f and the direction bytes
    (2s + 1 per vertex); a later round's reads g and the direction bytes and
    writes flag bits (s + 1.125) per vertex examined, in tiles or by sparse
    examination; an edit reads f and g and writes g (3s).  With split sweeps
    the tile detection of rounds 0 and 1 is the sweep kernel's (two launches)
    and the rest the engine's: round 0's apply kernel and the engine launch
    from round 1 (two launches; the tail kernel's rounds, timed with the
    engine, are counted in it)."""
    det = [r["swept"] * ((2 * s + 1) if i == 0 else (s + 1.125)) for i, r in enumerate(rounds)]
    tiles = [(r["swept"] - r["sparse"]) * ((2 * s + 1) if i == 0 else (s + 1.125))
             for i, r in enumerate(rounds)]
    edits = tm["edits"] * 3 * s
    out = {"k_dirs_fields": (tm["dirs_ms"], 1, tm["voxels"] * (s + 1))}
    if tm.get("sweeps"):
        swept_b = sum(tiles[:2])
        out["k_sweep"] = (tm["sweep_ms"], tm["sweeps"], swept_b)
        out["k_engine"] = (tm["engine_ms"], 2, sum(det) - swept_b + edits)
    else:
        out["k_engine"] = (tm["engine_ms"], 1, sum(det) + edits)
    return out


GOLDEN_512 = os.path.join(ROOT, "tests", "golden", "perlin512_f32.json")
GOLDEN_GRF = os.path.join(ROOT, "tests", "golden", "grf1024x1024x768_f64.json")
GOLDEN_BATCH = os.path.join(ROOT, "tests", "golden", "batch256_f32.json")


def check_against_golden(f, fhat, g, st, path=GOLDEN_512):
    """The timed result against the oracle's: sha256 of the input, of the
    corrected field and every statistic, as written by the oracle-only script
    beside the golden file."""
    import numpy as np
    gold = json.load(open(path))

    def sha(t):
        return hashlib.sha256(t.cpu().numpy().view(np.uint8)).hexdigest()

    same_in = sha(f) == gold["sha256_f"] and sha(fhat) == gold["sha256_fhat"]
    same_g = sha(g) == gold["sha256_g"]
    same_st = all(st[k] == gold["stats"][k] for k in gold["stats"])
    return {"identical": bool(same_in and same_g and same_st), "inputs": same_in,
            "sha256_g": same_g, "stats": same_st,
            "oracle": os.path.relpath(path, ROOT)}


def cpu_baseline(f, fhat, xi, planes):
    """The oracle (untuned) on a bounded sample: the first `planes` z-planes of
    the same field, corrected as a field of their own."""
    import oracle
    fs = f[:planes].cpu().numpy().copy()
    hs = fhat[:planes].cpu().numpy().copy()
    t0 = time.perf_counter()
    _, st = oracle.correct(fs, hs, xi)
    dt = time.perf_counter() - t0
    return {"value": fs.size / dt / 1e9, "unit": "Gvoxels/s", "cores": oracle.threads(),
            "kind": "oracle",
            "sample": "first %d z-planes (%dx%dx%d, %d vertices) of the same field, corrected "
                      "as their own field: %d rounds, %.1f s" % (
                          planes, planes, fs.shape[1], fs.shape[2], fs.size,
                          st["iterations"], dt),
            "small_64": cpu_small()}


def cpu_small():
    """The oracle on the whole 64^3 binary32 Perlin field (the latency
    workload), on every host thread and on one, per correction."""
    import oracle
    import synth
    f, fhat, xi = synth.small_perlin_case(device="cpu")
    f, fhat = f.numpy(), fhat.numpy()
    all_threads = oracle.threads()
    out = {"threads": all_threads}
    try:
        for key, n in (("ms_all_threads", all_threads), ("ms_one_thread", 1)):
            oracle.set_threads(n)
            oracle.correct(f, fhat.copy(), xi)  # warm-up
            reps = 3
            t0 = time.perf_counter()
            for _ in range(reps):
                _, st = oracle.correct(f, fhat.copy(), xi)
            out[key] = round((time.perf_counter() - t0) * 1e3 / reps, 2)
        out["status"] = st["status"]
        out["iterations"] = st["iterations"]
    finally:
        oracle.set_threads(all_threads)
    return out


def bench_batched(dev, n_fields, seed):
    """Uneven 2D batch: n_fields Gaussian-peak fields, sizes log-uniform in
    [256, 4096] per axis, relative bound from {1e-2, 1e-3, 1e-4}.  Plain =
    one pmsz_correct per field in sequence; batched = one
    pmsz_correct_batched with the tile height autotuned for the batch (the
    default policy's time is reported beside it).  Results must be
    bit-identical."""
    import torch

    import paper_2601_01787_amd as pmsz
    import synth
    cases = synth.batch_cases(n_fields, seed, device=dev)
    vox = sum(f.numel() for f, _, _ in cases)
    torch.cuda.synchronize()
    # warm both paths on one field
    pmsz.correct(cases[0][0], cases[0][1], cases[0][2])
    pmsz.correct_batched([(cases[0][0], cases[0][1].clone(), cases[0][2])])
    g_plain = [fh.clone() for _, fh, _ in cases]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st_plain = [pmsz.correct(f, g, xi, inplace=True)[1] for (f, _, xi), g in zip(cases, g_plain)]
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    def batched():
        g_batch = [fh.clone() for _, fh, _ in cases]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st_batch = pmsz.correct_batched([(f, g, xi) for (f, _, xi), g in zip(cases, g_batch)])
        torch.cuda.synchronize()
        return time.perf_counter() - t0, g_batch, st_batch

    t_batch, g_batch, st_batch = batched()
    same = all(torch.equal(a, b) for a, b in zip(g_plain, g_batch)) and st_plain == st_batch
    # autotuned tile height for this batch (tuning runs are outside the timing)
    target0 = pmsz.get_tiles_target(2, torch.float32)
    best, tune_ms = pmsz.tune_tiles(cases, reps=2)
    t_tuned, g_tuned, st_tuned = batched()
    tm = pmsz.last_timing()
    same = same and all(torch.equal(a, b) for a, b in zip(g_plain, g_tuned)) and \
        st_tuned == st_plain
    # the engine launch of the tuned batch against the HBM roofline
    alg = algorithmic_bytes(tm["voxels"], tm["swept"], tm["edits"], 4)
    loop_ms = tm["engine_ms"] + tm["sweep_ms"]
    roof = {"kernels": "k_sweep<float> + k_engine<float>" if tm["sweeps"] else "k_engine<float>",
            "engine_ms": round(tm["engine_ms"], 4), "sweep_ms": round(tm["sweep_ms"], 4),
            "dirs_ms": round(tm["dirs_ms"], 4), "algorithmic_bytes": alg,
            "achieved_gbs": round(alg / (loop_ms * 1e-3) / 1e9, 1),
            "frac": round(alg / (loop_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "swept_vertices": tm["swept"], "edits": tm["edits"], "rounds": tm["rounds"]}
    # every field against the oracle's golden result (the recorded batch)
    oracle_same = None
    if n_fields == 256 and seed == 256 and os.path.exists(GOLDEN_BATCH):
        import numpy as np
        gold = json.load(open(GOLDEN_BATCH))["fields"]
        oracle_same = all(
            hashlib.sha256(g.cpu().numpy().view(np.uint8)).hexdigest() == ref["sha256_g"] and
            all(st[k] == ref["stats"][k] for k in ref["stats"])
            for g, st, ref in zip(g_tuned, st_tuned, gold))
    return {"fields": n_fields, "voxels": vox, "roofline": roof, "oracle_identical": oracle_same,
            "plain_gvox_s": round(vox / t_plain / 1e9, 3),
            "batched_gvox_s": round(vox / t_tuned / 1e9, 3),
            "plain_ms": round(t_plain * 1e3, 2), "batched_ms": round(t_tuned * 1e3, 2),
            "speedup": round(t_plain / t_tuned, 2), "identical": bool(same),
            "max_iterations": max(s["iterations"] for s in st_batch),
            "tiles_target": {"default": target0 or "2048/fields in [32, 256]", "tuned": best,
                             "device_ms_by_target": {k: round(v, 3) for k, v in tune_ms.items()},
                             "batched_ms_default": round(t_batch * 1e3, 2)}}


def bench_small(dev, calls):
    """The 64^3 binary32 Perlin field (4 octaves, eps 1e-3, L2-resident):
    latency of one whole correction call (host planning, descriptor upload,
    directions pass and the one-launch loop, synchronised) and the device time
    per round."""
    import torch

    import paper_2601_01787_amd as pmsz
    import synth
    f, fhat, xi = synth.small_perlin_case(device=dev)
    ws = pmsz.workspace(pmsz.grid_of(f), pmsz.WS_CORRECT, dev)
    gs = [fhat.clone() for _ in range(calls + 2)]
    for g in gs[:2]:
        pmsz.correct(f, g, xi, inplace=True, ws=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for g in gs[2:]:
        _, st = pmsz.correct(f, g, xi, inplace=True, ws=ws)
    torch.cuda.synchronize()
    us = (time.perf_counter() - t0) * 1e6 / calls
    tm = pmsz.last_timing()
    rr = pmsz.last_rounds()
    dev_us = (tm["dirs_ms"] + tm["sweep_ms"] + tm["engine_ms"]) * 1e3
    return {"workload": "perlin 64^3 f32, 4 octaves, 4 cells, eps 1e-3, seed 1234",
            "us_per_call": round(us, 1), "device_us": round(dev_us, 1),
            "rounds": tm["rounds"], "device_us_per_round": round(tm["engine_ms"] * 1e3 / max(tm["rounds"], 1), 1),
            "iterations": st["iterations"], "status": st["status"],
            "per_round": {"detect_us": [round(r["detect_ms"] * 1e3, 1) for r in rr],
                          "apply_us": [round(r["apply_ms"] * 1e3, 1) for r in rr],
                          "swept": [r["swept"] for r in rr], "sparse": [r["sparse"] for r in rr],
                          "edits": [r["edits"] for r in rr]}}


def bench_large(dev, steps):
    """1024 x 1024 x 768 binary64 Gaussian random field (k^-3), relative bound
    1e-5: one pmsz_correct per step on resident inputs, each step on its own
    copy of fhat."""
    import torch

    import paper_2601_01787_amd as pmsz
    import synth
    f, fhat, xi = synth.grf_case(device=dev)
    grid = pmsz.grid_of(f)
    ws = pmsz.workspace(grid, pmsz.WS_CORRECT, dev)
    g = fhat.clone()
    _, st = pmsz.correct(f, g, xi, inplace=True, ws=ws)  # warm-up
    ms, tm = [], None
    for _ in range(steps):
        g.copy_(fhat)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, st = pmsz.correct(f, g, xi, inplace=True, ws=ws)
        torch.cuda.synchronize()
        ms.append((time.perf_counter() - t0) * 1e3)
        tm = pmsz.last_timing()
    ms_step = sum(ms) / len(ms)
    alg = algorithmic_bytes(tm["voxels"], tm["swept"], tm["edits"], 8)
    dev_ms = tm["dirs_ms"] + tm["sweep_ms"] + tm["engine_ms"]
    return {"workload": "grf k^-3 1024x1024x768 f64, rel eps 1e-5, seed 1024",
            "voxels": f.numel(), "steps": steps, "ms_per_step": round(ms_step, 3),
            "gvox_s": round(f.numel() / ms_step / 1e6, 3),
            "device_ms": round(dev_ms, 3), "dirs_ms": round(tm["dirs_ms"], 3),
            "engine_ms": round(tm["engine_ms"], 3), "sweep_ms": round(tm["sweep_ms"], 3),
            "hbm_frac": round(alg / (dev_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "iterations": st["iterations"], "edits": st["steps_applied"],
            "mismatch_initial": st["mismatch_initial"], "rounds": tm["rounds"],
            "swept_vertices": tm["swept"], "status": st["status"],
            "parity": check_against_golden(f, fhat, g, st, GOLDEN_GRF)}


def bench_targeted(f, fhat, xi, steps, g_halving):
    """The targeted-edit variant on the same resident workload: time, rounds,
    edits and the edit ratio (vertices whose value changed / all vertices,
    the paper's edit-ratio measure), beside the halving edit's."""
    import torch

    import paper_2601_01787_amd as pmsz
    ws = pmsz.workspace(pmsz.grid_of(f), pmsz.WS_CORRECT_TARGETED, f.device)
    g = fhat.clone()
    _, st = pmsz.correct(f, g, xi, inplace=True, ws=ws, mode="targeted")  # warm-up
    ms = []
    for _ in range(steps):
        g.copy_(fhat)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, st = pmsz.correct(f, g, xi, inplace=True, ws=ws, mode="targeted")
        torch.cuda.synchronize()
        ms.append((time.perf_counter() - t0) * 1e3)
    rep_t = pmsz.verify(f, g, fhat, xi)
    rep_h = pmsz.verify(f, g_halving, fhat, xi)
    n = f.numel()
    ms_step = sum(ms) / len(ms)
    # storage of the corrections: the edit stream of each result
    raw = n * f.element_size()
    storage = {}
    for name, gg in (("halving", g_halving), ("targeted", g)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stream, ne = pmsz.encode_edits(fhat, gg)
        torch.cuda.synchronize()
        t_enc = (time.perf_counter() - t0) * 1e3
        back = pmsz.decode_edits(fhat, stream)
        storage[name] = {"edits": ne, "bytes": stream.numel(),
                         "bits_per_edit": round(8 * stream.numel() / max(ne, 1), 2),
                         "fraction_of_raw_field": round(stream.numel() / raw, 6),
                         "encode_ms": round(t_enc, 3), "lossless": bool(torch.equal(back, gg))}
    return {"ms_per_step": round(ms_step, 4), "gvox_s": round(n / ms_step / 1e6, 3),
            "status": st["status"], "iterations": st["iterations"],
            "edits": st["steps_applied"], "vertices_edited": rep_t["vertices_edited"],
            "edit_ratio": round(rep_t["vertices_edited"] / n, 6),
            "max_abs_err": rep_t["max_abs_err"],
            "halving_vertices_edited": rep_h["vertices_edited"],
            "halving_edit_ratio": round(rep_h["vertices_edited"] / n, 6),
            "halving_max_abs_err": rep_h["max_abs_err"],
            "directions_restored": rep_t["asc_mismatch"] == 0 and rep_t["desc_mismatch"] == 0,
            "edit_storage": storage}


def bench_labels_verify(f, fhat, g, xi, reps):
    """Segmentation labels (pmsz_labels) of f's and of the corrected field's
    directions, and the evaluation counts (pmsz_verify), on the resident 512^3
    workload.  Labels: device time from the library's events; algorithmic
    bytes = per vertex 1 (direction byte) + 8 (two labels written) once, then
    per pointer-jumping pass 12 (own label and the label it points at read,
    own label written; 8 on the last pass, which writes nothing)."""
    import torch

    import paper_2601_01787_amd as pmsz
    out = {}
    n = f.numel()
    for name, h in (("labels_f", f), ("labels_g", g)):
        d = pmsz.directions(h)
        pmsz.labels(d)  # warm-up
        ms, info = [], None
        for _ in range(reps):
            pmsz.labels(d)
            info = pmsz.last_labels()
            ms.append(info["ms"])
        passes = info["passes_max"] + info["passes_min"]
        alg = n * 9 + n * 12 * max(passes - 2, 0) + n * 8 * min(passes, 2)
        dev_ms = sorted(ms)[len(ms) // 2]
        out[name] = {"ms": round(dev_ms, 4), "passes_max": info["passes_max"],
                     "passes_min": info["passes_min"], "algorithmic_bytes": alg,
                     "achieved_gbs": round(alg / (dev_ms * 1e-3) / 1e9, 1),
                     "frac": round(alg / (dev_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        del d
    pmsz.verify(f, g, fhat, xi)  # warm-up
    ms = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rep = pmsz.verify(f, g, fhat, xi)
        ms.append((time.perf_counter() - t0) * 1e3)
    wall = sorted(ms)[len(ms) // 2]
    out["verify"] = {"ms_per_call": round(wall, 3), "gvox_s": round(n / wall / 1e6, 3),
                     "report": rep}
    return out


def bench_blocks(f, fhat, xi, configs):
    """The decomposed-domain correction (Sec. IV-B) emulated on one GPU: for
    each block grid, relaxed exchanges (each block converges locally first)
    against per-round exchanges.  Reports exchanges (phases), the schedule's
    length in rounds with one GPU per block (critical_rounds), all rounds,
    lowered copies, device time of the local corrections and of the
    exchanges, and that every direction is restored."""
    import torch

    import paper_2601_01787_amd as pmsz
    out = {}
    for bl in configs:
        key = "x".join(map(str, bl))
        out[key] = {}
        for name, per_round in (("relaxed", False), ("per_round", True)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            g, st = pmsz.correct_blocks(f, fhat, xi, bl, per_round=per_round)
            torch.cuda.synchronize()
            wall = (time.perf_counter() - t0) * 1e3
            rep = pmsz.verify(f, g, fhat, xi)
            out[key][name] = {
                "status": st["status"], "phases": st["phases"],
                "critical_rounds": st["critical_rounds"], "local_rounds": st["local_rounds"],
                "lowered": st["lowered"], "edits": st["steps_applied"],
                "compute_ms": round(st["compute_ms"], 3),
                "exchange_ms": round(st["exchange_ms"], 3), "wall_ms": round(wall, 3),
                "vertices_edited": rep["vertices_edited"],
                "directions_restored": rep["asc_mismatch"] == 0 and rep["desc_mismatch"] == 0,
                "bound_violations": rep["bound_violations"]}
            del g
    return out


def bench_serving(dev, rates, n_requests, pool_per_class, seed, max_seconds=None):
    """Open-loop serving: Poisson arrivals at each rate; requests drawn from a
    pre-generated pool (generation stays out of the loop) over five classes
    (128^3, 256^3, 512^3 Perlin; 1024^2, 4096^2 Gaussian peaks; binary32) with
    relative bounds from {1e-2, 1e-3, 1e-4}.  The continuous-batching server
    and a FIFO server of plain per-request launches replay the same arrival
    sequence; every served result is compared with the request's alone result.
    The batching server admits by HBM footprint and caps the vertices in
    flight (its default work budget)."""
    import numpy as np
    import torch

    import paper_2601_01787_amd as pmsz
    import synth
    from paper_2601_01787_amd import serve
    rng = np.random.default_rng(seed)
    pool = []
    for cls in ("perlin128", "perlin256", "perlin512", "peaks1024", "peaks4096"):
        for j in range(pool_per_class):
            rel = float(rng.choice([1e-2, 1e-3, 1e-4]))
            s = int(rng.integers(1 << 30))
            if cls.startswith("perlin"):
                n = int(cls[6:])
                f, fhat, xi = synth.perlin_case(n, 6, 8, rel, s, device=dev)
            else:
                n = int(cls[5:])
                f, fhat, xi = synth.make_2d_case(n, n, rel, s, device=dev)
            g, _ = pmsz.correct(f, fhat, xi)
            pool.append({"cls": cls, "f": f, "fhat": fhat, "xi": xi, "g": g})
    torch.cuda.synchronize()
    out = []
    for rate in rates:
        # n_requests, or as many as arrive in max_seconds
        n_req = n_requests if max_seconds is None else min(n_requests, int(rate * max_seconds))
        arr = np.cumsum(rng.exponential(1.0 / rate, size=n_req))
        pick = rng.integers(len(pool), size=n_req)
        row = {"rate_req_s": rate, "requests": n_req}
        log("serving at %g req/s: %d requests" % (rate, n_req))
        for kind in ("batched", "fifo"):
            reqs = []
            for i, (t, k) in enumerate(zip(arr, pick)):
                p = pool[int(k)]
                r = serve.Request(i, p["f"], p["fhat"], p["xi"], float(t))
                reqs.append(r)
            bad = []
            which = {i: int(k) for i, k in enumerate(pick)}

            def check(r):
                if not torch.equal(r.g, pool[which[r.rid]]["g"]):
                    bad.append(r.rid)

            done = serve.run_open_loop(kind, reqs, dev, hbm_budget=96 << 30, max_fields=64,
                                       rounds_per_step=0, check=check)
            s = serve.latency_summary(done)
            s["identical"] = not bad and len(done) == n_req
            row[kind] = s
        out.append(row)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-planes", type=int, default=512)
    ap.add_argument("--batch-fields", type=int, default=256,
                    help="fields of the uneven 2D batch (0 skips the batched comparison)")
    ap.add_argument("--targeted-steps", type=int, default=3,
                    help="timed steps of the targeted-edit variant on the same workload (0 skips)")
    ap.add_argument("--large-steps", type=int, default=3,
                    help="timed steps of the 1024x1024x768 binary64 workload (0 skips it)")
    ap.add_argument("--serve-rates", default="50,200,500",
                    help="Poisson arrival rates (req/s) of the serving comparison ('' skips it)")
    ap.add_argument("--serve-requests", type=int, default=200)
    ap.add_argument("--serve-seconds", type=float, default=None,
                    help="cap each rate's arrivals at this many seconds (with --serve-requests)")
    ap.add_argument("--serve-pool", type=int, default=4,
                    help="pre-generated fields per request class")
    ap.add_argument("--small-calls", type=int, default=50,
                    help="calls of the 64^3 latency leg (0 to skip)")
    ap.add_argument("--blocks", default="2x2x2,4x4x4",
                    help="block grids of the decomposed-domain leg ('' to skip)")
    ap.add_argument("--labels-reps", type=int, default=3,
                    help="timed repetitions of the labels and verify leg (0 skips it)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run one plain device copy of this size (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2601_01787_amd as pmsz
    import synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    log("generating 512^3 Perlin workload on", torch.cuda.get_device_name(dev))
    f, fhat, xi = synth.large_perlin_case(device=dev)
    n_vox = f.numel()
    grid = pmsz.grid_of(f)
    ws = pmsz.workspace(grid, pmsz.WS_CORRECT, dev)
    K, W = args.steps, args.warmup
    gs = [fhat.clone() for _ in range(W + K)]
    torch.cuda.synchronize()

    if args.copy_probe_mib:
        src = torch.empty(args.copy_probe_mib << 18, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)  # a device-to-device copy: HIP's copy kernel reads and writes the size once
        torch.cuda.synchronize()
        # read-only probes in the marches' load shapes: dword rows, byte rows
        pmsz.probe_read(src, 0)
        pmsz.probe_read(src, 1)
        log("copy probe: %d MiB read, %d MiB written; read probes: %d MiB as dword rows, "
            "%d MiB as byte rows" % ((args.copy_probe_mib,) * 4))
        del src, dst

    log("warmup", W)
    for i in range(W):
        _, st = pmsz.correct(f, gs[i], xi, inplace=True, ws=ws)
        assert st["status"] == "OK", st
    torch.cuda.synchronize()

    log("timing", K, "steps")
    tims, stats, rounds_all = [], [], []
    t0 = time.perf_counter()
    for i in range(K):
        _, st = pmsz.correct(f, gs[W + i], xi, inplace=True, ws=ws)
        tims.append(pmsz.last_timing())
        rounds_all.append(pmsz.last_rounds())
        stats.append(st)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / K
    value = n_vox / (ms_per_step * 1e-3) / 1e9
    for st in stats:
        assert st["status"] == "OK" and st["iterations"] == stats[0]["iterations"], st
    parity = check_against_golden(f, fhat, gs[W + K - 1], stats[-1])
    if not parity["identical"]:
        log("the corrected 512^3 field differs from the oracle's:", parity)
        sys.exit(1)

    tm = tims[-1]
    per_round = rounds_all[-1]
    s = f.element_size()
    # the dominant kernel: the largest share of the correction's device time
    split = {}
    for t, rr in zip(tims, rounds_all):
        for k, (ms, n, b) in kernel_split(t, rr, s).items():
            acc = split.setdefault(k, [0.0, 0, 0.0])
            acc[0] += ms
            acc[1] += n
            acc[2] += b
    dom = max(split, key=lambda k: split[k][0])
    ms_tot, launches, bytes_tot = split[dom]
    avg_ms = ms_tot / launches
    per_launch = bytes_tot / launches
    achieved = per_launch / (avg_ms * 1e-3) / 1e9
    name = dom + "<float>"
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic(name), "kernel": name,
                "kernel_avg_ms": round(avg_ms, 4), "algorithmic_bytes": int(per_launch),
                "launches_per_step": launches // len(tims)}
    kernels = {k + "<float>": {"ms_per_step": round(v[0] / len(tims), 4),
                               "launches_per_step": v[1] // len(tims),
                               "algorithmic_gbs": round(v[2] / (v[0] * 1e-3) / 1e9, 1)
                               if v[0] > 0 else None}
               for k, v in split.items()}
    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "Gvoxels/s", "n_gpus": 1,
        "steps": K, "warmup": W, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "perlin 512^3 f32, 6 octaves, 8 cells, eps 1e-4, seed 512; "
                               "one field per launch", "voxels": n_vox,
                   "parallelism": "1 GPU"},
        "roofline": roofline,
        "parity": parity,
        "detail": {"iterations": stats[0]["iterations"], "edits": stats[0]["steps_applied"],
                   "mismatch_initial": stats[0]["mismatch_initial"], "rounds": tm["rounds"],
                   "swept_vertices": tm["swept"], "tiles": tm["tiles"], "grid": tm["grid"],
                   "kernels": kernels,
                   "first_round_ms": round(tm["first_round_ms"], 4),
                   "later_detect_ms": round(tm["detect_ms"], 4),
                   "later_apply_ms": round(tm["apply_ms"], 4),
                   "per_round": {"detect_ms": [round(r["detect_ms"], 4) for r in per_round],
                                 "sparse": [r["sparse"] for r in per_round],
                                 "apply_ms": [round(r["apply_ms"], 4) for r in per_round],
                                 "swept": [r["swept"] for r in per_round],
                                 "flagged": [r["flagged"] for r in per_round],
                                 "edits": [r["edits"] for r in per_round]}},
    }
    if args.targeted_steps:
        log("targeted-edit variant:", args.targeted_steps, "steps")
        out["targeted"] = bench_targeted(f, fhat, xi, args.targeted_steps, gs[-1])
    if args.labels_reps:
        log("labels and verify:", args.labels_reps, "reps")
        out["labels_verify"] = bench_labels_verify(f, fhat, gs[-1], xi, args.labels_reps)
    del gs
    torch.cuda.empty_cache()
    if args.blocks:
        configs = [tuple(int(v) for v in c.split("x")) for c in args.blocks.split(",") if c]
        log("decomposed domain:", configs)
        out["blocks"] = bench_blocks(f, fhat, xi, configs)
        torch.cuda.empty_cache()
    if args.batch_fields:
        log("batched vs plain on", args.batch_fields, "2D fields")
        out["batched"] = bench_batched(dev, args.batch_fields, 256)
        torch.cuda.empty_cache()
    if args.small_calls:
        log("small field latency")
        out["small_64"] = bench_small(dev, args.small_calls)
    if args.large_steps:
        log("large binary64 workload:", args.large_steps, "steps")
        out["large_f64"] = bench_large(dev, args.large_steps)
        torch.cuda.empty_cache()
    if args.serve_rates:
        rates = [float(x) for x in args.serve_rates.split(",") if x]
        log("serving: rates", rates, "x", args.serve_requests, "requests")
        out["serving"] = bench_serving(dev, rates, args.serve_requests, args.serve_pool, 7,
                                       args.serve_seconds)
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) on", args.cpu_planes, "planes")
        out["cpu_baseline"] = cpu_baseline(f, fhat, xi, args.cpu_planes)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
