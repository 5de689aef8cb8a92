"""Serving loop logic on the CPU: admission by footprint, the logical schedule and latency
bookkeeping, with stand-in plans that record what the server asks of them (no GPU)."""
import contextlib

import pytest

from paper_2402_05283_amd import serve


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class Done:
    def query(self):
        return True


class FakePlan:
    def __init__(self, scan, log):
        self.scan, self.log, self.k = scan, log, 0
        self.stream = None

    def submit(self, n, I, S, asynchronous=False):
        self.log.append((self.scan.sid, "submit", n, self.k))

    def iterate(self, n):
        self.k += n
        self.log.append((self.scan.sid, "iterate", n, self.k))

    def assemble_volume(self):
        self.log.append((self.scan.sid, "volume", self.k))
        return ("volume", self.scan.sid, self.k)

    def record_event(self):
        return Done()


def make_server(budget, log, clock, **kw):
    def batch(plans, n):
        for p in plans:
            p.iterate(n)
    return serve.Server(budget, clock=clock, plan_factory=lambda s: FakePlan(s, log), batch_fn=batch,
                        stream_ctx=lambda p: contextlib.nullcontext(), **kw)


def run(server, clock, jobs, order_seed=0):
    """Push frames per the jobs' schedules with a fake clock, stepping the server between."""
    import random
    rng = random.Random(order_seed)
    scans = {}
    events = []
    for ji, (t0, N, Np, fps) in enumerate(jobs):
        events.append((t0, "open", ji, None))
        for n in range(Np):
            events.append((t0 + n / fps, "frame", ji, n))
    events.sort(key=lambda e: (e[0], e[1] != "open"))
    for t, kind, ji, n in events:
        clock.t = t
        if kind == "open":
            scans[ji] = server.open_scan(jobs[ji][1], jobs[ji][2], seed=ji)
        else:
            server.push_frame(scans[ji], n, None, None, t=t)
        for _ in range(rng.randrange(0, 4)):      # a random amount of scheduling between arrivals
            clock.t += 1e-3
            server.step()
    while server.busy():
        clock.t += 1e-3
        server.step()
    return [scans[i] for i in range(len(jobs))]


def ops_of(log, sid):
    return [e[1:] for e in log if e[0] == sid]


def test_schedule_is_logical_and_independent_of_the_mix():
    clock = FakeClock()
    alone_logs = []
    jobs = [(0.0, 64, 5, 20.0), (0.01, 128, 3, 50.0), (0.02, 64, 4, 10.0)]
    for ji, job in enumerate(jobs):
        log = []
        srv = make_server(1 << 40, log, clock, n_ei=5, r_frame=10, r_final=20)
        clock.t = 0.0
        run(srv, clock, [job], order_seed=ji)
        alone_logs.append([e[1:] for e in log])
    for seed in range(3):
        log = []
        srv = make_server(1 << 40, log, clock, n_ei=5, r_frame=10, r_final=20)
        clock.t = 0.0
        scans = run(srv, clock, jobs, order_seed=100 + seed)
        for sid, sc in enumerate(scans):
            assert ops_of(log, sc.sid) == alone_logs[sid]
    # the schedule itself: frame j submitted at k = j * r_frame; r_final after the last frame
    ops = alone_logs[0]
    submits = [o for o in ops if o[0] == "submit"]
    assert [o[2] for o in submits] == [0, 10, 20, 30, 40]
    assert ops[-1] == ("volume", 5 * 10 + 20)
    assert all(o[1] == 5 for o in ops if o[0] == "iterate")


def test_admission_by_footprint_and_latency():
    clock = FakeClock()
    log = []
    fp = serve.Server.footprint(64, 4)
    srv = make_server(2 * fp + fp // 2, log, clock, n_ei=10, r_final=10)
    jobs = [(0.0, 64, 4, 100.0), (0.0, 64, 4, 100.0), (0.0, 64, 4, 100.0)]
    scans = run(srv, clock, jobs)
    first_ops = {}
    for i, e in enumerate(log):
        first_ops.setdefault(e[0], i)
    # the third scan only starts once one of the first two has finished and left
    finish = min(max(i for i, e in enumerate(log) if e[0] == s) for s in (0, 1))
    assert first_ops[2] > finish
    for s in scans:
        assert s.done and s.latency_s is not None and s.latency_s >= 0
        assert s.volume == ("volume", s.sid, 4 * 10 + 10)
    assert srv.used == 0


def test_rejects_bad_schedules_and_oversized_scans():
    with pytest.raises(ValueError):
        serve.Server(1 << 30, n_ei=10, r_frame=15)
    with pytest.raises(ValueError):
        serve.Server(1 << 30, n_ei=10, r_final=5)
    srv = serve.Server(1024)
    with pytest.raises(ValueError):
        srv.open_scan(64, 4)


def test_scans_on_the_clock_run_alone():
    """While a scan whose last frame has landed is unfinished, the other scans issue no episode
    (hold_others); without it they keep issuing.  Either way every scan's schedule is the same."""
    def trace(hold):
        clock = FakeClock()
        log = []
        # depth_final 1: the timed scan takes one episode per round, so it stays unfinished for
        # several rounds
        srv = make_server(1 << 40, log, clock, n_ei=5, r_frame=5, r_final=20, depth_final=1, hold_others=hold)
        a = srv.open_scan(64, 2, seed=0)
        b = srv.open_scan(64, 6, seed=1)
        for n in range(2):
            srv.push_frame(a, n, None, None, t=0.0)
        for n in range(5):
            srv.push_frame(b, n, None, None, t=0.0)
        iters_of_b = []
        while not a.done:
            clock.t += 1e-3
            srv.step()
            iters_of_b.append(b.iters_done)
        srv.push_frame(b, 5, None, None, t=clock.t)
        while srv.busy():
            clock.t += 1e-3
            srv.step()
        return log, iters_of_b, a, b
    log_h, b_held, a_h, b_h = trace(True)
    log_f, b_free, a_f, b_f = trace(False)
    assert max(b_held) == 0
    assert max(b_free) > 5
    for sid in (0, 1):
        assert ops_of(log_h, sid) == ops_of(log_f, sid)
    assert a_h.volume == ("volume", 0, 2 * 5 + 20) and b_h.volume == ("volume", 1, 6 * 5 + 20)


def test_scan_on_the_clock_queues_its_credit_at_once():
    """A timed scan drains its backlog in one round: every landed frame is submitted and its credit
    queued (up to depth_final episodes in flight), not one frame and one episode per round."""
    class Pending:
        def query(self):
            return False

    clock = FakeClock()
    log = []
    srv = make_server(1 << 40, log, clock, n_ei=5, r_frame=5, r_final=20, depth_final=8)
    a = srv.open_scan(64, 2, seed=0)
    for n in range(2):
        srv.push_frame(a, n, None, None, t=0.0)
    a.plan.record_event = lambda: Pending()          # nothing completes: in-flight work piles up
    srv.step()
    # one round submitted both frames and queued all their 2 * 5 + 20 iterations
    assert a.n_submitted == 2 and a.credit == 0 and a.iters_done == 2 * 5 + 20
    assert len(a.in_flight) == (2 * 5 + 20) // 5


def test_shortest_scan_on_the_clock_goes_first():
    """Two scans on the clock: with shortest_first the one with less remaining work (smaller N) is
    issued and finishes first, the other waits; without it both issue in the same rounds.  The
    schedules (what each plan is asked to do) are the same either way."""
    def trace(shortest):
        clock = FakeClock()
        log = []
        srv = make_server(1 << 40, log, clock, n_ei=5, r_frame=5, r_final=10, depth_final=1,
                          shortest_first=shortest)
        big = srv.open_scan(128, 2, seed=0)
        small = srv.open_scan(64, 2, seed=1)
        for sc in (big, small):
            for n in range(2):
                srv.push_frame(sc, n, None, None, t=0.0)
        order = []
        while srv.busy():
            clock.t += 1e-3
            srv.step()
            for sc in (big, small):
                if sc.done and sc.sid not in order:
                    order.append(sc.sid)
        return log, order
    log_s, order_s = trace(True)
    log_f, order_f = trace(False)
    assert order_s == [1, 0]
    for sid in (0, 1):
        assert ops_of(log_s, sid) == ops_of(log_f, sid)
    # with shortest_first the big scan issues nothing until the small one has issued all of its work
    first_small_done = max(i for i, e in enumerate(log_s) if e[0] == 1 and e[1] == "iterate")
    big_iters_before = [e for e in log_s[:first_small_done] if e[0] == 0 and e[1] == "iterate"]
    assert big_iters_before == []
