"""Continuous-batching request loop for Brand updates and preconditionings.

Every layer's two K-factor states (input side A, output side Gamma) stay
resident in HBM.  Requests arrive as a backward pass would emit them:

* ``UpdateRequest(layer, side, M)``  one B-KFAC step of one factor (Algorithm 4);
* ``PrecondRequest(layer, G, S, lam_g, lam_a)``  the two-sided inverse
  application to one layer gradient (Section 2.1 / Algorithm 1).

Scheduling (host side; all arithmetic runs in the HIP library):

* admission in arrival order, per-state FIFO: a request is admitted only when
  every earlier request touching one of its states has been issued, and while
  the workspace bytes of the groups in flight stay within ``byte_budget``
  (requests that arrive while others run are admitted as budget frees up);
* same-phase admitted requests are fused by shape bucket into one grouped
  launch sequence (``kfb_brand_update_batched`` / ``kfb_precondition_batched``,
  whose per-problem results equal single calls bit for bit);
* at most ``max_inflight`` groups are on the device at once: while the slots
  are taken, arriving requests wait and are fused into larger groups when a
  slot frees (this is what lets throughput approach the grouped closed loop
  under load instead of flooding the device with groups of one);
* with ``pad_updates``, updates of every factor that keeps the same number of
  modes r_eff = min(k_valid, r) share a bucket, whatever its width d and the
  batch width: the group runs as ``kfb_brand_update_grouped``, which pads each
  problem on the device to the group's widest factor and batch (zero rows and
  columns; each problem weighted by its own batch width, so the result is the
  exact update by its real columns, and the padded modes are empty slots that
  add nothing to the inverse and that spectrum continuation skips).  This
  trades extra work per update for much larger groups when the layers'
  shapes vary: the core eigensolve, whose cost does not depend on d, then
  runs for many problems per launch.  Results are no longer bit-identical to
  a request run alone, only equal within rounding;
* groups go round-robin onto several default-priority HIP streams, each first
  waiting on the completion events of the last operations on its states, so
  work on different states overlaps on the device while per-state order holds;
* a request's inputs may still be in production on the submitter's stream
  (a backward pass enqueues M or G there and submits at once): ``submit``
  records an event on the current stream, and the group that carries the
  request waits on it before its first launch;
* completion is observed by polling the group's event; latency is completion
  minus arrival on the host clock.  Completed requests are handed to the
  caller through ``sink`` (a list the caller owns, e.g. for one measured run)
  and kept only in a bounded ``done_log`` otherwise, so a long-running server
  holds no references to the tensors of old requests.
"""
from __future__ import annotations

import collections
import ctypes
import time
from dataclasses import dataclass, field

from . import kfb


@dataclass
class UpdateRequest:
    layer: int
    side: str                 # 'A' (input factor, width d_in) or 'G' (output factor, width d_out)
    M: object                 # device tensor (n, d) in the state's batch dtype
    t_arrival: float = 0.0
    t_done: float = 0.0
    rid: int = -1
    error: str = ""
    ready: object = None      # event on the submitter's stream, recorded at submit


@dataclass
class PrecondRequest:
    layer: int
    G: object                 # device tensor (d_out, d_in), row-major
    S: object                 # output tensor, same shape
    lam_g: float = 0.01
    lam_a: float = 0.01
    flags: int = 0
    t_arrival: float = 0.0
    t_done: float = 0.0
    rid: int = -1
    error: str = ""
    ready: object = None      # event on the submitter's stream, recorded at submit


@dataclass
class _Group:
    kind: str
    reqs: list
    stream: object
    event: object
    ws: object
    nbytes: int
    t_issue: float = 0.0
    keep: object = None   # padded batches, alive until the group completes


@dataclass
class ServerStats:
    completed: int = 0
    updates: int = 0
    preconds: int = 0
    groups: int = 0
    grouped_problems: int = 0
    update_groups: int = 0
    update_problems: int = 0
    max_inflight_bytes: int = 0
    rejected: int = 0


class Server:
    def __init__(self, layers, n_max: int, rho: float = 0.95, prec: int = kfb.KFB_BF16_MIXED,
                 streams: int = 4, byte_budget: int = 8 << 30, max_group: int = 64, device="cuda",
                 max_inflight: int | None = None, pad_updates: bool = False, done_log_max: int = 1024):
        """layers: list of (d_in, d_out, r_A, r_G)."""
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.prec = prec
        self.n_max = n_max
        self.pad_updates = bool(pad_updates)
        self.fa, self.fg = [], []
        for (d_in, d_out, r_a, r_g) in layers:
            self.fa.append(kfb.Factor(d_in, r_a, n_max, rho, prec, device=self.device))
            self.fg.append(kfb.Factor(d_out, r_g, n_max, rho, prec, device=self.device))
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(streams)]
        self.byte_budget = int(byte_budget)
        self.max_group = int(max_group)
        self.max_inflight = int(max_inflight) if max_inflight else len(self.streams)
        self.pending = collections.deque()
        self.inflight: list[_Group] = []
        self.inflight_bytes = 0
        self.last_event = {}      # state handle value -> event of its last operation
        self.rr = 0
        self.stats = ServerStats()
        self.hooks_before_issue = None   # optional callback(kind, reqs, stream), enqueued before the group
        self.hooks_after_issue = None    # optional callback(kind, reqs, stream), enqueued before its event
        self.failed = collections.deque(maxlen=done_log_max)
        self.done_log = collections.deque(maxlen=done_log_max)   # the latest completions
        self.sink = None                 # optional caller-owned list receiving every completion
        self._next_rid = 0
        self._rest_prefix = 0
        self._lib = kfb.load()

    # ------------------------------------------------------------------ API
    def factor(self, layer: int, side: str):
        return self.fa[layer] if side == "A" else self.fg[layer]

    def submit(self, req, t_arrival: float | None = None):
        """Queue a request.  Its tensors may still be being written on the caller's
        current stream: the group that runs it waits for that work first."""
        req.t_arrival = time.perf_counter() if t_arrival is None else t_arrival
        ev = self.torch.cuda.Event()
        ev.record(self.torch.cuda.current_stream(self.device))
        req.ready = ev
        req.rid = self._next_rid
        self._next_rid += 1
        self.pending.append(req)
        return req.rid

    def busy(self) -> bool:
        return bool(self.pending or self.inflight)

    def poll(self) -> list:
        """Retire finished groups; returns the requests completed by this call."""
        done = []
        keep = []
        now = time.perf_counter()
        for g in self.inflight:
            if g.event.query():
                for r in g.reqs:
                    r.t_done = now
                    r.ready = None
                    done.append(r)
                    self.done_log.append(r)
                    if self.sink is not None:
                        self.sink.append(r)
                self.inflight_bytes -= g.nbytes
                self.stats.completed += len(g.reqs)
            else:
                keep.append(g)
        self.inflight = keep
        return done

    def step(self) -> int:
        """One scheduler tick: retire, admit, group, issue into the free slots.
        Returns the number of groups issued."""
        self.poll()
        free = self.max_inflight - len(self.inflight)
        if free <= 0 or not self.pending:
            return 0
        admitted = self._admit()
        issued = 0
        leftover = []
        for key, reqs in admitted.items():
            for i in range(0, len(reqs), self.max_group):
                chunk = reqs[i:i + self.max_group]
                if issued < free and self._issue(key, chunk):
                    issued += 1
                else:
                    leftover.extend(chunk)
        if leftover:
            # back into the queue in arrival order (keeps per-state FIFO): they are
            # older than every request the admission scan did not reach, so only the
            # scanned prefix of the queue needs merging
            head = [self.pending.popleft() for _ in range(min(self._rest_prefix, len(self.pending)))]
            merged = sorted(head + leftover, key=lambda r: r.rid)
            self.pending.extendleft(reversed(merged))
        return issued

    def drain(self, timeout_s: float = 120.0):
        t0 = time.perf_counter()
        while self.busy():
            if not self.step():
                time.sleep(0)
            if time.perf_counter() - t0 > timeout_s:
                raise TimeoutError("server did not drain")

    # ------------------------------------------------------------ internals
    def _states_of(self, r):
        if isinstance(r, UpdateRequest):
            return (self.factor(r.layer, r.side),)
        return (self.fg[r.layer], self.fa[r.layer])

    def _key(self, r):
        if isinstance(r, UpdateRequest):
            f = self.factor(r.layer, r.side)
            info = f.info()
            r_eff = min(info["k_valid"], f.r)
            if self.pad_updates:
                return ("U", r_eff)
            return ("U", f.d, f.r, r_eff, int(r.M.shape[0]), int(r.M.stride(0)))
        fg, fa = self.fg[r.layer], self.fa[r.layer]
        kg, ka = fg.info()["k_valid"], fa.info()["k_valid"]
        return ("P", fg.d, fa.d, kg, ka, r.flags, int(r.G.stride(0)), int(r.S.stride(0)))

    def _bytes_for(self, key, reqs) -> int:
        lib = self._lib
        if key[0] == "U":
            hs = (ctypes.c_void_p * len(reqs))(*[self.factor(r.layer, r.side).handle.value for r in reqs])
            if self.pad_updates:   # the padded copies live in the call's workspace
                wd = (ctypes.c_int32 * len(reqs))(*[int(r.M.shape[0]) for r in reqs])
                return int(lib.kfb_update_grouped_workspace_bytes(len(reqs), hs, wd))
            return int(lib.kfb_update_batched_workspace_bytes(len(reqs), hs, key[4]))
        hg = (ctypes.c_void_p * len(reqs))(*[self.fg[r.layer].handle.value for r in reqs])
        ha = (ctypes.c_void_p * len(reqs))(*[self.fa[r.layer].handle.value for r in reqs])
        return int(lib.kfb_precondition_batched_workspace_bytes(len(reqs), hg, ha))

    def _admit(self):
        """Arrival-order admission with per-state FIFO and the byte budget."""
        groups = collections.OrderedDict()
        blocked = set()      # states with an earlier request left pending
        used = set()         # states already taken by a request of this tick
        budget_left = self.byte_budget - self.inflight_bytes
        rest = collections.deque()
        est = {}
        # look at the oldest requests only: enough to fill every free slot with a
        # full group several times over (a long backlog is not rescanned each tick)
        scan = max(32, 4 * self.max_group * self.max_inflight)
        while self.pending and scan > 0:
            scan -= 1
            r = self.pending.popleft()
            sts = [f.handle.value for f in self._states_of(r)]
            if any(s in blocked or s in used for s in sts):
                rest.append(r)
                blocked.update(sts)
                continue
            key = self._key(r)
            if key not in est:
                est[key] = self._bytes_for(key, [r])
            need = est[key]
            if need > self.byte_budget:
                # can never be admitted: fail this request and keep serving the others
                r.error = f"needs {need} workspace bytes, above the budget {self.byte_budget}"
                r.t_done = time.perf_counter()
                self.failed.append(r)
                self.stats.rejected += 1
                continue
            if need > budget_left:
                rest.append(r)
                blocked.update(sts)
                continue
            budget_left -= need
            used.update(sts)
            groups.setdefault(key, []).append(r)
        self._rest_prefix = len(rest)
        rest.extend(self.pending)
        self.pending = rest
        return groups

    def _issue(self, key, reqs) -> bool:
        torch = self.torch
        stream = self.streams[self.rr % len(self.streams)]
        self.rr += 1
        nbytes = self._bytes_for(key, reqs)
        with torch.cuda.stream(stream):
            for r in reqs:
                if r.ready is not None:          # inputs produced on the submitter's stream
                    stream.wait_event(r.ready)
                for f in self._states_of(r):
                    ev = self.last_event.get(f.handle.value)
                    if ev is not None:
                        stream.wait_event(ev)
            if self.hooks_before_issue:
                self.hooks_before_issue(key[0], reqs, stream)
            ws = kfb.Workspace(self.device)
            keep = None
            if key[0] == "U":
                factors = [self.factor(r.layer, r.side) for r in reqs]
                if self.pad_updates:
                    kfb.update_grouped(factors, [r.M for r in reqs], ws)
                else:
                    kfb.update_batched(factors, [r.M for r in reqs], ws)
                self.stats.updates += len(reqs)
            else:
                kfb.precondition_batched([self.fg[r.layer] for r in reqs], [self.fa[r.layer] for r in reqs],
                                         [r.G for r in reqs], [r.S for r in reqs], [r.lam_g for r in reqs],
                                         [r.lam_a for r in reqs], reqs[0].flags, ws)
                self.stats.preconds += len(reqs)
            if self.hooks_after_issue:
                self.hooks_after_issue(key[0], reqs, stream)
            ev = torch.cuda.Event()
            ev.record(stream)
        for r in reqs:
            for f in self._states_of(r):
                self.last_event[f.handle.value] = ev
        self.inflight.append(_Group(key[0], reqs, stream, ev, ws, nbytes, time.perf_counter(), keep))
        self.inflight_bytes += nbytes
        self.stats.max_inflight_bytes = max(self.stats.max_inflight_bytes, self.inflight_bytes)
        self.stats.groups += 1
        self.stats.grouped_problems += len(reqs)
        if key[0] == "U":
            self.stats.update_groups += 1
            self.stats.update_problems += len(reqs)
        return True


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    i = min(len(xs) - 1, max(0, int(round(q / 100.0 * (len(xs) - 1)))))
    return xs[i]


def poisson_run(server: Server, make_request, rate: float, n_requests: int, seed: int = 0,
                timeout_s: float = 300.0, progress=None, progress_every: float = 30.0):
    """Open-loop Poisson arrivals at `rate` req/s; returns (wall seconds, completed requests).
    progress(submitted, completed, seconds) is called about every progress_every seconds."""
    import numpy as np
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=n_requests)
    done = []
    prev_sink, server.sink = server.sink, done
    try:
        t0 = time.perf_counter()
        arrivals = t0 + np.cumsum(gaps)
        i = 0
        t_report = t0 + progress_every
        while i < n_requests or server.busy():
            now = time.perf_counter()
            if progress is not None and now >= t_report:
                progress(i, len(done), now - t0)
                t_report = now + progress_every
            while i < n_requests and arrivals[i] <= now:
                server.submit(make_request(i, rng), t_arrival=float(arrivals[i]))
                i += 1
            server.step()
            if now - t0 > timeout_s:
                raise TimeoutError("poisson run did not finish")
        wall = time.perf_counter() - t0
    finally:
        server.sink = prev_sink
    return wall, done
