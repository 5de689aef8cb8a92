"""Serving loop: scans arrive as streams of diffraction frames and are reconstructed as they land.

Each scan gets a plan (workspace + stream) once it fits the HBM budget; scans that do not fit
wait in arrival order.  The carousel iteration starts on the partial angle set and is refined as
frames land (partial sets: absent neighbours drop out of Eq. 4 with renormalised weights; an angle
joins at the next episode boundary).  After the last frame, a final run of iterations and step D
(Fourier-slice insertion + 3D inverse FFT) give the volume; the time from the last frame's arrival
to the volume being ready is the scan's latency.

The schedule is logical, so a scan's result does not depend on wall-clock interleaving or on the
other scans in the mix: frame j (in landing order) is submitted only after the scan has run
exactly j * r_frame iterations; each landed frame adds r_frame iterations of credit and the last
one adds r_final more.  r_frame and r_final are multiples of n_ei, so every chunk of work is whole
episodes.  All scans with credit advance together, one episode per round, through
cpra_iterate_batch (scans of one size share launches, size classes overlap on their streams); frames
are submitted without waiting for the GPU (the data check completes in stream order); at most
`depth` episodes per scan are in flight, which bounds how long a frame submission can wait; a
scan whose last frame has landed (its latency clock is running) may queue up to `depth_final` and
is issued first (it drains its backlog of frames and credit at once, up to that many episodes), and
with `hold_others` the other scans issue no new episode while such a scan is
unfinished, so it does not share the GPU with work whose latency is not yet being measured (the
others fall behind their frames for that while and catch up afterwards; the logical schedule keeps
their results unchanged).  With `shortest_first`, of several scans on the clock the one with the
least remaining work issues first.
"""
from __future__ import annotations

import collections
import time

from . import _lib


class Scan:
    """One scan in the server: its frames, credit and result."""

    def __init__(self, sid, N, Np, theta, seed, plan_kw, t_open):
        self.sid, self.N, self.Np = sid, int(N), int(Np)
        self.theta, self.seed, self.plan_kw = theta, seed, dict(plan_kw)
        self.t_open = t_open
        self.plan = None
        self.arrived = collections.deque()     # (n, I, S, t_arrival) not yet submitted
        self.n_expected = self.Np
        self.n_submitted = 0
        self.credit = 0
        self.iters_done = 0
        self.in_flight = collections.deque()   # completion events of issued episodes
        self.t_last_frame = None
        # host clock at: the last frame's submit, the last episode's issue, step D's issue
        self.t_last_submit = self.t_last_issue = self.t_assemble = None
        self.volume = None
        self.volume_event = None
        self.t_done = None
        self.latency_s = None
        self.footprint = 0

    @property
    def done(self):
        return self.t_done is not None


class Server:
    """Request loop over the C ABI.

    hbm_budget: bytes of device memory the server may hand out as plan workspaces and volumes.
    n_ei: episode length (iterations between carousel couplings).
    r_frame, r_final: iterations per landed frame and after the last frame (multiples of n_ei).
    algo, beta: the iteration (HIO with feedback beta, or ER).
    """

    def __init__(self, hbm_budget, n_ei=10, r_frame=None, r_final=50, algo=_lib.HIO, beta=0.9, depth=1,
                 depth_final=8, hold_others=True, shortest_first=True, clock=time.perf_counter, plan_factory=None,
                 batch_fn=None, stream_ctx=None):
        r_frame = n_ei if r_frame is None else r_frame
        if r_frame % n_ei or r_final % n_ei or r_frame <= 0 or r_final < 0:
            raise ValueError("r_frame and r_final must be non-negative multiples of n_ei (r_frame > 0)")
        self.budget, self.used = int(hbm_budget), 0
        self.n_ei, self.r_frame, self.r_final = n_ei, r_frame, r_final
        self.algo, self.beta, self.depth, self.depth_final = algo, beta, depth, max(depth, depth_final)
        self.hold_others = hold_others
        self.shortest_first = shortest_first
        self.clock = clock
        self.plan_factory = plan_factory or self._make_plan
        self.batch_fn = batch_fn or (lambda plans, n: _lib.iterate_batch(plans, n, self.algo, self.beta))
        # plan calls run with the plan's stream current, so no scan's work waits on another's
        self.stream_ctx = stream_ctx or self._torch_stream
        self.waiting = collections.deque()    # scans not yet admitted, in arrival order
        self.active = []
        self.finished = []
        self._next_id = 0
        self.step_max_s = 0.0      # longest single scheduling round (host time)
        self.slow_steps = 0        # rounds that took more than 50 ms

    # ---------------------------------------------------------------- set-up
    @staticmethod
    def footprint(N, Np, **plan_kw):
        """Device bytes a scan holds while admitted: its workspace and its N^3 volume."""
        real = plan_kw.get("real", _lib.REAL_F32)
        p = _lib.make_params(N, Np, theta=plan_kw.get("theta"), n_ei=plan_kw.get("n_ei", 10),
                             real=real, amp=plan_kw.get("amp", _lib.AMP_F32))
        return _lib.workspace_size(p) + 256 + N ** 3 * (8 if real == _lib.REAL_F64 else 4)

    @staticmethod
    def _torch_stream(plan):
        import torch
        return torch.cuda.stream(plan.stream)

    def _make_plan(self, scan):
        import torch
        stream = torch.cuda.Stream()
        return _lib.Plan(scan.N, scan.Np, theta=scan.theta, n_ei=self.n_ei, seed=scan.seed, stream=stream,
                         **scan.plan_kw)

    def open_scan(self, N, Np, theta=None, seed=0, **plan_kw):
        """Announce a scan; it is admitted as soon as its footprint fits the budget."""
        s = Scan(self._next_id, N, Np, theta, seed, plan_kw, self.clock())
        self._next_id += 1
        s.footprint = self.footprint(N, Np, theta=theta, n_ei=self.n_ei, **plan_kw)
        if s.footprint > self.budget:
            raise ValueError(f"scan needs {s.footprint} bytes, more than the whole budget {self.budget}")
        self.waiting.append(s)
        self._admit()
        return s

    def push_frame(self, scan, n, intensity, support, t=None):
        """A frame (angle n: (1,N,N) float32 intensity and uint8 support, device tensors) landed."""
        t = self.clock() if t is None else t
        scan.arrived.append((int(n), intensity, support, t))
        if len(scan.arrived) + scan.n_submitted == scan.n_expected:
            scan.t_last_frame = t

    def _admit(self):
        while self.waiting and self.used + self.waiting[0].footprint <= self.budget:
            s = self.waiting.popleft()
            s.plan = self.plan_factory(s)
            self.used += s.footprint
            self.active.append(s)

    # ---------------------------------------------------------------- loop
    def _retire_events(self, s):
        while s.in_flight and s.in_flight[0].query():
            s.in_flight.popleft()

    def step(self):
        """One scheduling round.  Returns True if any work was issued or completed."""
        t_in = self.clock()
        progressed = self._step()
        dt = self.clock() - t_in
        self.step_max_s = max(self.step_max_s, dt)
        self.slow_steps += dt > 0.05
        return progressed

    def _step(self):
        progressed = False
        for s in self.active:
            self._retire_events(s)
            # submit the next frame only once the credit of the previous ones is spent
            if s.credit == 0 and s.arrived and s.n_submitted < s.n_expected:
                self._submit_next(s)
                progressed = True
        # a scan whose last frame has landed may queue more episodes (its latency is being
        # measured) and goes first in the batch; with hold_others the rest wait for it
        def timed(s):
            return s.t_last_frame is not None

        hold = self.hold_others and any(timed(s) for s in self.active)
        # shortest_first: of the scans on the clock with episodes still to issue, only the one with
        # the least remaining work issues new ones (the others' queued episodes still run)
        lead = None
        if self.shortest_first:
            ready = [s for s in self.active if timed(s) and (s.credit > 0 or s.arrived)]
            if ready:
                lead = min(ready, key=self._remaining)

        def room(s):
            if timed(s):
                if lead is not None and s is not lead:
                    return 0
                return self.depth_final - len(s.in_flight)
            return 0 if hold else self.depth - len(s.in_flight)
        batch = [s for s in self.active if s.credit > 0 and room(s) > 0]
        batch.sort(key=lambda s: not timed(s))
        if batch:
            self.batch_fn([s.plan for s in batch], self.n_ei)
            for s in batch:
                self._issued(s)
            progressed = True
        # a scan on the clock drains its backlog now, up to depth_final episodes in flight: the next
        # landed frame once its credit is spent, then that frame's episodes, and so on, instead of
        # one frame and one episode per round
        for s in self.active:
            if not timed(s):
                continue
            while room(s) > 0:
                if s.credit > 0:
                    self.batch_fn([s.plan], self.n_ei)
                    self._issued(s)
                elif s.arrived and s.n_submitted < s.n_expected:
                    self._submit_next(s)
                else:
                    break
                progressed = True
        for s in list(self.active):
            if s.volume_event is None and s.n_submitted == s.n_expected and s.credit == 0:
                with self.stream_ctx(s.plan):
                    s.volume = s.plan.assemble_volume()
                s.volume_event = self._record(s)
                s.t_assemble = self.clock()
                progressed = True
            if s.volume_event is not None and s.volume_event.query():
                s.t_done = self.clock()
                s.latency_s = s.t_done - s.t_last_frame
                self.active.remove(s)
                self.finished.append(s)
                self.used -= s.footprint
                s.plan = None                      # the workspace goes back to the allocator
                progressed = True
        if progressed:
            self._admit()
        return progressed

    def _remaining(self, s):
        """Iterations still to issue times the pattern size and angle count: the scan's remaining GPU
        work, up to a constant."""
        left = s.credit + self.r_frame * len(s.arrived) + (self.r_final if s.n_submitted < s.n_expected else 0)
        return left * s.N * s.N * s.n_expected

    def _submit_next(self, s):
        n, I, S, _ = s.arrived.popleft()
        with self.stream_ctx(s.plan):
            s.plan.submit(n, I, S, asynchronous=True)
        s.n_submitted += 1
        s.credit += self.r_frame + (self.r_final if s.n_submitted == s.n_expected else 0)
        if s.n_submitted == s.n_expected:
            s.t_last_submit = self.clock()

    def _issued(self, s):
        s.credit -= self.n_ei
        s.iters_done += self.n_ei
        s.in_flight.append(self._record(s))
        if s.credit == 0 and s.n_submitted == s.n_expected:
            s.t_last_issue = self.clock()

    @staticmethod
    def _record(s):
        ev = getattr(s.plan, "record_event", None)
        if ev is not None:
            return ev()
        import torch
        e = torch.cuda.Event()
        e.record(s.plan.stream)
        return e

    def busy(self):
        return bool(self.waiting or self.active)


class Job:
    """A scan as a client sends it: start time, shape, seed, frame rate and a frame source.

    frames(n) -> (intensity (1,N,N) float32, support (1,N,N) uint8) device tensors of angle n;
    angles arrive in order 0..Np-1, frame j at t_start + j / fps.
    """

    def __init__(self, t_start, N, Np, frames, fps, seed=0, theta=None, **plan_kw):
        self.t_start, self.N, self.Np, self.frames, self.fps = t_start, N, Np, frames, fps
        self.seed, self.theta, self.plan_kw = seed, theta, plan_kw
        self.scan = None
        self.next_frame = 0


def replay(server, jobs, t0=None, idle_sleep=2e-4, on_done=None):
    """Drive `server` with `jobs` in real time (frame arrival times relative to t0); returns the
    finished Scan objects in job order once every scan has its volume.  on_done(scan), if given,
    is called as each scan finishes."""
    t0 = server.clock() if t0 is None else t0
    pending = sorted(jobs, key=lambda j: j.t_start)
    while True:
        now = server.clock() - t0
        nxt = None
        for j in pending:
            if j.scan is None:
                if now >= j.t_start:
                    j.scan = server.open_scan(j.N, j.Np, theta=j.theta, seed=j.seed, **j.plan_kw)
                else:
                    nxt = j.t_start if nxt is None else min(nxt, j.t_start)
                    continue
            while j.next_frame < j.Np:
                t_arr = j.t_start + j.next_frame / j.fps
                if t_arr > now:
                    nxt = t_arr if nxt is None else min(nxt, t_arr)
                    break
                I, S = j.frames(j.next_frame)
                server.push_frame(j.scan, j.next_frame, I, S, t=t0 + t_arr)
                j.next_frame += 1
        n_before = len(server.finished)
        progressed = server.step()
        if on_done is not None:
            for sc in server.finished[n_before:]:
                on_done(sc)
        if all(j.scan is not None and j.scan.done for j in pending):
            return [j.scan for j in jobs]
        if not progressed:
            wait = idle_sleep if nxt is None else min(idle_sleep, max(0.0, nxt - (server.clock() - t0)))
            time.sleep(wait)
