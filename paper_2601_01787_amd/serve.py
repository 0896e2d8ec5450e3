"""Continuous-batching correction server on one GPU.

Requests (f, fhat, xi) arrive over time.  The server keeps a serving session
of the C library (pmsz_session_*): requests are admitted while their HBM
footprint fits the budget and a slot is free, each step runs a few rounds of
the persistent correction kernel over every admitted request, finished
requests leave at once and the next ones are admitted in their place, so
requests that arrive while others are on the GPU share the device with them.
A request's result is the same as correcting it alone (the per-field
iteration does not depend on what else is in the step).

``FifoServer`` is the baseline: one plain pmsz_correct per request, in
arrival order.
"""
import collections
import itertools
import time

import torch

from . import Session, correct, field_workspace_size, grid_of


class Request:
    __slots__ = ("rid", "f", "fhat", "xi", "arrival", "admitted", "done_at", "g", "ws",
                 "handle", "stats", "footprint")

    def __init__(self, rid, f, fhat, xi, arrival):
        self.rid = rid
        self.f, self.fhat, self.xi = f, fhat, xi
        self.arrival = arrival
        self.admitted = None
        self.done_at = None
        self.g = None
        self.ws = None
        self.handle = None
        self.stats = None
        self.footprint = None


# Vertices admitted at once: one 512^3 field plus a few small ones.
DEFAULT_WORK_BUDGET = 160 << 20


def footprint(f):
    """Device bytes a request holds while admitted: its f, fhat and g, and its
    field workspace (flag bitmap, direction bytes, tile flags, state)."""
    return 3 * f.numel() * f.element_size() + field_workspace_size(grid_of(f)) + 256


class BatchingServer:
    """Admits requests by HBM footprint into a serving session and keeps the
    persistent correction kernel running over every admitted request.

    Steps are preemptible.  With no backlog (nothing waiting when the step
    is launched) a step ends after the round in which a field finishes (its
    result is collected at once) and after the current round when a new
    request arrives that can be admitted (it joins the next step).  Under a
    backlog, ending a step at every arrival and every finished field would
    relaunch the kernel about twice per request; such steps instead run for
    `bulk_step` seconds and then end after the current round when a waiting
    request can be admitted, else after the first round that begins with a
    field done, collecting every field finished by then.  With
    `rounds_per_step` > 0 steps are instead fixed at that many rounds.

    Every field of a step advances in the same rounds, so a round lasts as
    long as the largest field's round; `work_budget` (vertices) caps the
    vertices admitted at once so that large fields do not hold every small
    one back for their whole run (a request larger than the budget is
    admitted when the session is empty).  None disables the cap.  With
    `backlog_len` or more requests waiting the cap is `backlog_work_budget`
    instead (None: none): under a backlog, fields that share steps overlap
    their latency-bound rounds, and waiting costs more than sharing.  Requests
    are admitted in arrival order, a request that does not fit being passed
    by later ones that do, until it has waited `max_wait` seconds."""

    def __init__(self, device, hbm_budget, max_fields=64, rounds_per_step=0,
                 dtype=torch.float32, max_iters=1 << 40, work_budget=DEFAULT_WORK_BUDGET,
                 max_wait=0.02, bulk_step=0.002, backlog_len=16, backlog_work_budget=None):
        self.device = torch.device(device)
        self.budget = int(hbm_budget)
        self.work_budget = work_budget
        self.backlog_len = backlog_len
        self.backlog_work_budget = backlog_work_budget
        self.cap = work_budget
        self.work = 0
        self.rounds = int(rounds_per_step)
        self.max_iters = max_iters
        self.max_wait = max_wait
        self.session = Session(dtype, max_fields, self.device)
        self.max_fields = max_fields
        self.in_use = 0
        self.active = {}
        self.steps = 0
        self.in_flight = False
        self.stop_sent = False
        self.bulk_step = bulk_step
        self.bulk = False
        self.launched_at = 0.0
        self.deliver_sent = False

    def set_queue(self, waiting):
        """The vertex cap for `waiting` requests in the queue."""
        self.cap = self.backlog_work_budget if waiting >= self.backlog_len else self.work_budget

    def can_admit(self, req):
        if len(self.active) >= self.max_fields or self.in_use + req.footprint > self.budget:
            return False
        return (self.cap is None or not self.active
                or self.work + req.f.numel() <= self.cap)

    def admit(self, req, now):
        req.g = req.fhat.clone()
        n = field_workspace_size(grid_of(req.f))
        buf = torch.empty(n + 256, dtype=torch.uint8, device=self.device)
        off = (-buf.data_ptr()) % 256
        req.ws = buf[off:off + n]
        req.handle = self.session.add(req.f, req.g, req.xi, req.ws, max_iters=self.max_iters)
        req.admitted = now
        self.in_use += req.footprint
        self.work += req.f.numel()
        self.active[req.handle] = req

    def admit_from(self, pending, now, max_scan=64):
        """Admit waiting requests (a deque in arrival order) that fit,
        looking at no more than the `max_scan` oldest (a long queue is not
        rescanned at every step)."""
        self.set_queue(len(pending))
        kept = []
        scanned = 0
        while pending and scanned < max_scan and len(self.active) < self.max_fields:
            r = pending.popleft()
            scanned += 1
            if self.can_admit(r):
                self.admit(r, now)
                continue
            kept.append(r)
            # the oldest request that waited too long is not passed again
            if now - r.arrival > self.max_wait:
                break
        pending.extendleft(reversed(kept))

    def launch(self, now=0.0, backlog=False):
        """Launch a step over every admitted request (none in flight).  now:
        the caller's clock; backlog: requests are waiting."""
        if self.active and not self.in_flight:
            if self.rounds > 0:
                self.session.step(self.rounds)
            else:
                self.session.step(0, stop_on_done=not backlog)
            self.in_flight = True
            self.stop_sent = False
            self.deliver_sent = False
            self.bulk = backlog and self.rounds <= 0
            self.launched_at = now
            self.steps += 1

    def preempt(self):
        """End the step in flight after its current round."""
        if self.in_flight and not self.stop_sent and self.rounds <= 0:
            self.session.request_stop()
            self.stop_sent = True

    def tick(self, now, admissible):
        """Stop requests for the step in flight.  admissible: a waiting
        request can be admitted."""
        if not self.in_flight or self.stop_sent or self.rounds > 0:
            return
        if not self.bulk:
            if admissible:
                self.preempt()
        elif now - self.launched_at >= self.bulk_step:
            if admissible:
                self.preempt()
            elif not self.deliver_sent:
                self.session.request_stop(when_done=True)
                self.deliver_sent = True

    def poll(self, wait=False):
        """None while the step runs (unless wait); else the finished
        requests of the step that ended."""
        if not self.in_flight:
            return []
        if not wait and self.session.running():
            return None
        self.session.sync()
        self.in_flight = False
        finished = []
        for h, st in self.session.finished():
            req = self.active.pop(h)
            req.stats = st
            self.session.remove(h)
            self.in_use -= req.footprint
            self.work -= req.f.numel()
            req.ws = None
            finished.append(req)
        return finished

    def step(self):
        """One blocking step over every admitted request; returns the
        finished ones."""
        self.launch()
        return self.poll(wait=True)

    def close(self):
        if self.in_flight:
            self.poll(wait=True)
        self.session.close()


def run_open_loop(server_kind, requests, device, hbm_budget, max_fields=64, rounds_per_step=0,
                  check=None, work_budget=DEFAULT_WORK_BUDGET):
    """Replay `requests` (sorted by arrival time, seconds from start) against
    a server in real time.  Returns the served requests.  `check(req)` (if
    given) is called on every finished request."""
    dev = torch.device(device)
    pending = collections.deque()
    arrivals = collections.deque(sorted(requests, key=lambda r: r.arrival))
    done = []
    for r in arrivals:
        r.footprint = footprint(r.f)
    srv = None
    if server_kind == "batched":
        srv = BatchingServer(dev, hbm_budget, max_fields, rounds_per_step,
                             work_budget=work_budget)
    try:
        return _replay(server_kind, srv, arrivals, pending, done, dev, check)
    finally:
        if srv is not None:
            srv.close()


def _replay(server_kind, srv, arrivals, pending, done, dev, check):
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    while arrivals or pending or (server_kind == "batched" and srv.active):
        now = time.perf_counter() - t0
        while arrivals and arrivals[0].arrival <= now:
            pending.append(arrivals.popleft())
        if server_kind == "batched":
            if srv.in_flight:
                srv.set_queue(len(pending))
                srv.tick(now, bool(pending) and
                         any(srv.can_admit(r) for r in itertools.islice(pending, 64)))
                finished = srv.poll()
                if finished is None:
                    continue  # the step runs on; keep watching arrivals
            else:
                finished = []
                srv.admit_from(pending, now)
                if pending and not srv.active:
                    raise RuntimeError("request %d does not fit the HBM budget" % pending[0].rid)
                srv.launch(now, backlog=bool(pending))
            t = time.perf_counter() - t0
            for r in finished:
                r.done_at = t
                if check:
                    check(r)
                r.g = None
            done.extend(finished)
        else:
            if pending:
                r = pending.popleft()
                r.admitted = now
                g, st = correct(r.f, r.fhat, r.xi)
                torch.cuda.synchronize(dev)
                r.done_at = time.perf_counter() - t0
                r.g, r.stats = g, st
                if check:
                    check(r)
                r.g = None
                done.append(r)
        if not pending and arrivals and (server_kind != "batched" or not srv.active):
            wait = arrivals[0].arrival - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(min(wait, 0.01))
    return done


def latency_summary(done, duration=None):
    lat = sorted((r.done_at - r.arrival) * 1e3 for r in done)
    if not lat:
        return {}
    pick = lambda q: lat[min(len(lat) - 1, int(q * (len(lat) - 1) + 0.5))]  # noqa: E731
    span = max(r.done_at for r in done) - min(r.arrival for r in done)
    vox = sum(r.f.numel() for r in done)
    return {"requests": len(lat), "p50_ms": round(pick(0.50), 3), "p99_ms": round(pick(0.99), 3),
            "mean_ms": round(sum(lat) / len(lat), 3), "req_per_s": round(len(lat) / span, 2),
            "gvox_per_s": round(vox / span / 1e9, 3)}
