"""Serving-session parity on the GPU: a field's result and statistics are the
same whether it is corrected alone (pmsz_correct) or inside a session that
admits and retires other fields between steps (continuous batching)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2601_01787_amd as pmsz
import synth
from paper_2601_01787_amd import serve

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
KEYS = ("iterations", "steps_applied", "flagged_final", "stalled_flags", "mismatch_initial",
        "status")


def _cases():
    out = []
    for n, seed in ((24, 1), (40, 2)):
        f, fhat, xi = synth.perlin_case(n, 3, 3, 1e-3, seed)
        out.append((f, fhat, xi))
    for nx, ny, rel, seed in ((300, 190, 1e-2, 3), (129, 257, 1e-3, 4), (70, 64, 1e-4, 5)):
        out.append(synth.make_2d_case(nx, ny, rel, seed))
    return [(f.to(DEV), fh.to(DEV), xi) for f, fh, xi in out]


def _alone(cases):
    res = []
    for f, fh, xi in cases:
        g, st = pmsz.correct(f, fh, xi)
        res.append((g, st))
    return res


def test_session_mix_matches_alone():
    cases = _cases()
    alone = _alone(cases)
    ses = pmsz.Session(torch.float32, 8, torch.device(DEV))
    live = {}
    # admit two, step once, admit the rest while those are in flight
    order = [0, 1, None, 2, 3, None, 4]
    for item in order:
        if item is None:
            ses.step(1)
            ses.sync()
            continue
        f, fh, xi = cases[item]
        g = fh.clone()
        n = pmsz.field_workspace_size(pmsz.grid_of(f))
        buf = torch.empty(n + 256, dtype=torch.uint8, device=DEV)
        off = (-buf.data_ptr()) % 256
        ws = buf[off:off + n]
        live[ses.add(f, g, xi, ws)] = (item, g)
    finished = {}
    for _ in range(10000):
        if len(finished) == len(cases):
            break
        ses.step(2)
        ses.sync()
        for h, (item, g) in list(live.items()):
            st, done = ses.result(h)
            if done:
                finished[item] = (g, st)
                ses.remove(h)
                del live[h]
    ses.close()
    assert len(finished) == len(cases)
    for i, (g_a, st_a) in enumerate(alone):
        g_b, st_b = finished[i]
        assert torch.equal(g_a, g_b), i
        assert [st_a[k] for k in KEYS] == [st_b[k] for k in KEYS], (i, st_a, st_b)


def test_session_matches_oracle_on_small_field():
    f, fh, xi = synth.small_perlin_case()
    g_ref, st_ref = oracle.correct(f.numpy(), fh.numpy(), xi)
    f, fh = f.to(DEV), fh.to(DEV)
    ses = pmsz.Session(torch.float32, 2, torch.device(DEV))
    g = fh.clone()
    n = pmsz.field_workspace_size(pmsz.grid_of(f))
    ws = torch.empty(n, dtype=torch.uint8, device=DEV)
    h = ses.add(f, g, xi, ws)
    done = False
    while not done:
        ses.step(1)
        ses.sync()
        st, done = ses.result(h)
    ses.close()
    assert [st[k] for k in KEYS] == [st_ref[k] for k in KEYS]
    torch.cuda.synchronize()
    assert np.array_equal(g.cpu().numpy().view(np.uint32), g_ref.view(np.uint32))


@pytest.mark.parametrize("rounds_per_step", [2, 0], ids=["fixed2", "preemptive"])
def test_open_loop_server_results_match_alone(rounds_per_step):
    """Poisson arrivals into the batching server (fixed two-round steps, and
    preemptible steps that end when a field finishes or a request waits):
    every served result equals the alone result of the same input."""
    cases = _cases()
    alone = _alone(cases)
    rng = np.random.default_rng(7)
    t = np.cumsum(rng.exponential(1.0 / 400.0, size=12))
    reqs = []
    for i, ti in enumerate(t):
        k = int(rng.integers(len(cases)))
        f, fh, xi = cases[k]
        r = serve.Request(i, f, fh, xi, float(ti))
        r.stats = k
        reqs.append(r)
    which = {r.rid: r.stats for r in reqs}
    bad = []

    def check(r):
        k = which[r.rid]
        if not torch.equal(r.g, alone[k][0]):
            bad.append(r.rid)

    done = serve.run_open_loop("batched", reqs, DEV, hbm_budget=1 << 30, max_fields=4,
                               rounds_per_step=rounds_per_step, check=check)
    assert len(done) == len(reqs) and not bad
    summary = serve.latency_summary(done)
    assert summary["requests"] == len(reqs) and summary["p50_ms"] > 0


def test_cancelled_field_leaves_the_others_unchanged():
    """A field removed before it finishes (a cancelled request) stops at a
    valid iterate (within its bounds, never above fhat), and the fields that
    shared its steps end exactly as they do alone."""
    import oracle
    cases = _cases()
    alone = _alone(cases)
    ses = pmsz.Session(torch.float32, 8, torch.device(DEV))
    live, bufs = {}, []
    for i, (f, fh, xi) in enumerate(cases):
        g = fh.clone()
        n = pmsz.field_workspace_size(pmsz.grid_of(f))
        buf = torch.empty(n + 256, dtype=torch.uint8, device=DEV)
        off = (-buf.data_ptr()) % 256
        bufs.append(buf)
        live[ses.add(f, g, xi, buf[off:off + n])] = (i, g)
    victim = max(range(len(cases)), key=lambda i: alone[i][1]["iterations"])
    ses.step(1)
    ses.sync()
    for h, (i, g) in list(live.items()):
        if i == victim:
            st, done = ses.result(h)
            assert not done
            ses.remove(h)
            del live[h]
            f, fh, xi = cases[i]
            lb, _ = oracle.bounds(f.cpu().numpy(), xi)
            gh = g.cpu().numpy()
            assert bool(np.all(gh >= lb)) and bool(np.all(gh <= fh.cpu().numpy()))
    finished = {}
    for _ in range(10000):
        if not live:
            break
        ses.step(2)
        ses.sync()
        for h, (i, g) in list(live.items()):
            st, done = ses.result(h)
            if done:
                finished[i] = (g, st)
                ses.remove(h)
                del live[h]
    ses.close()
    assert victim not in finished and len(finished) == len(cases) - 1
    for i, (g_b, st_b) in finished.items():
        g_a, st_a = alone[i]
        assert torch.equal(g_a, g_b), i
        assert [st_a[k] for k in KEYS] == [st_b[k] for k in KEYS], (i, st_a, st_b)


def test_preemptible_steps_match_alone():
    """Steps that end when a field finishes (stop_on_done) and steps ended by
    a stop request after their first round: each field ends bit-identical to
    its alone result, and the fields a step reports finished are exactly the
    ones that are done."""
    cases = _cases()
    alone = _alone(cases)
    ses = pmsz.Session(torch.float32, 8, torch.device(DEV))
    live, bufs = {}, []
    for i, (f, fh, xi) in enumerate(cases):
        g = fh.clone()
        n = pmsz.field_workspace_size(pmsz.grid_of(f))
        buf = torch.empty(n + 256, dtype=torch.uint8, device=DEV)
        off = (-buf.data_ptr()) % 256
        bufs.append(buf)
        live[ses.add(f, g, xi, buf[off:off + n])] = (i, g)
    finished, steps = {}, 0
    while live and steps < 10000:
        ses.step(0, stop_on_done=True)
        if steps % 2:
            ses.request_stop()  # ends the step after at most two rounds
        ses.sync()
        steps += 1
        fin = dict(ses.finished())
        for h, (i, g) in list(live.items()):
            st, done = ses.result(h)
            assert done == (h in fin)
            if done:
                finished[i] = (g, st)
                ses.remove(h)
                del live[h]
    ses.close()
    assert not live and steps > 1
    for i, (g_b, st_b) in finished.items():
        g_a, st_a = alone[i]
        assert torch.equal(g_a, g_b), i
        assert [st_a[k] for k in KEYS] == [st_b[k] for k in KEYS], (i, st_a, st_b)


def _add(ses, case, bufs):
    f, fh, xi = case
    g = fh.clone()
    n = pmsz.field_workspace_size(pmsz.grid_of(f))
    buf = torch.empty(n + 256, dtype=torch.uint8, device=DEV)
    off = (-buf.data_ptr()) % 256
    bufs.append(buf)
    return ses.add(f, g, xi, buf[off:off + n]), g


def test_split_steps_match_alone():
    """Steps whose starting fields hold 2^23 vertices or more run the tile
    detection of their first two rounds as kernels of their own between
    engine launches.  Fields that start in such steps, and fields already
    running in them (tile and sparse rounds), end bit-identical to their
    alone results, with fixed-round, stop-on-done and stopped steps."""
    big = [synth.perlin_case(208, 4, 4, 1e-3, 11), synth.make_2d_case(3000, 3000, 1e-3, 12)]
    cases = [(f.to(DEV), fh.to(DEV), xi) for f, fh, xi in big] + _cases()[:3]
    alone = _alone(cases)
    ses = pmsz.Session(torch.float32, 8, torch.device(DEV))
    live, bufs, finished = {}, [], {}

    def collect():
        fin = dict(ses.finished())
        for h, (i, g) in list(live.items()):
            st, done = ses.result(h)
            assert done == (h in fin), (i, done)
            if done:
                finished[i] = (g, st)
                ses.remove(h)
                del live[h]

    def add(i):
        h, g = _add(ses, cases[i], bufs)
        live[h] = (i, g)

    add(0)
    ses.step(1)  # split, first launch only
    ses.sync()
    collect()
    add(2)
    add(3)
    ses.step(3)  # nothing fresh at 2^23: one launch
    ses.sync()
    collect()
    add(1)  # a fresh 9M-vertex field next to running ones: split
    ses.step(0, stop_on_done=True)
    ses.sync()
    collect()
    add(4)
    steps = 0
    while live and steps < 10000:
        ses.step(0, stop_on_done=True)
        if steps % 3 == 1:
            ses.request_stop()
        ses.sync()
        collect()
        steps += 1
    ses.close()
    assert len(finished) == len(cases)
    for i, (g_a, st_a) in enumerate(alone):
        g_b, st_b = finished[i]
        assert torch.equal(g_a, g_b), i
        assert [st_a[k] for k in KEYS] == [st_b[k] for k in KEYS], (i, st_a, st_b)


def test_stop_when_done_steps_match_alone():
    """Steps asked to end once a field is done (pmsz_session_request_stop_when_done)
    end with at least one field finished, report exactly the fields that are
    done, and every field ends bit-identical to its alone result."""
    cases = _cases()
    alone = _alone(cases)
    ses = pmsz.Session(torch.float32, 8, torch.device(DEV))
    live, bufs, finished = {}, [], {}
    for i in range(len(cases)):
        h, g = _add(ses, cases[i], bufs)
        live[h] = (i, g)
    steps = 0
    while live and steps < 10000:
        ses.step(0)
        ses.request_stop(when_done=True)
        if steps == 1:
            ses.request_stop()  # a plain stop request overrides it
        ses.sync()
        fin = dict(ses.finished())
        assert fin or steps == 1
        for h, (i, g) in list(live.items()):
            st, done = ses.result(h)
            assert done == (h in fin), (i, done)
            if done:
                finished[i] = (g, st)
                ses.remove(h)
                del live[h]
        steps += 1
    ses.close()
    assert len(finished) == len(cases) and steps < len(cases) + 2
    for i, (g_a, st_a) in enumerate(alone):
        g_b, st_b = finished[i]
        assert torch.equal(g_a, g_b), i
        assert [st_a[k] for k in KEYS] == [st_b[k] for k in KEYS], (i, st_a, st_b)


def test_burst_of_requests_matches_alone():
    """A burst of requests arriving together (a backlog from the start): the
    server runs bulk steps, admits without the vertex cap while 16 or more
    wait, collects fields on stop-when-done requests; every result equals
    the alone result and every request is served."""
    cases = _cases()
    alone = _alone(cases)
    rng = np.random.default_rng(11)
    reqs = []
    for i in range(40):
        k = int(rng.integers(len(cases)))
        f, fh, xi = cases[k]
        r = serve.Request(i, f, fh, xi, 0.0001 * i)
        r.stats = k
        reqs.append(r)
    which = {r.rid: r.stats for r in reqs}
    bad = []

    def check(r):
        if not torch.equal(r.g, alone[which[r.rid]][0]):
            bad.append(r.rid)

    done = serve.run_open_loop("batched", reqs, DEV, hbm_budget=1 << 30, max_fields=6,
                               rounds_per_step=0, check=check, work_budget=1 << 14)
    assert len(done) == len(reqs) and not bad
