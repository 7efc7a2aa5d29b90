"""Step-request server with continuous batching over the fused kernel.

Cell state lives on the device in a slot pool sized by an HBM budget (x, v, F: 36 bytes
per vertex). A request asks for one time step of a session's cells; a session owns a
contiguous range of red-cell slots and one of platelet slots and keeps its state resident
between requests. The server loop admits arrived requests whenever their session is idle
and its cells have slots; every tick advances the union of all admitted requests' cells with
ONE fused launch (the library's active-cell work list), so requests that arrive while
earlier ticks run join the next tick and share its launch. Up to two ticks are in flight on
the stream; completion times come from events on that stream.

When a session needs slots that are taken, idle sessions (resident, no request in flight)
are moved out to pinned host memory, least recently stepped first, and moved back when their
next request is admitted: the copies (x and v, 24 bytes per vertex) run on the stream in
order with the steps, so a session's results do not depend on whether it was moved.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from . import npfem as N

RBC, PLT = 0, 1
BYTES_PER_VERTEX = 36          # x, v, F in FP32


class RangeAllocator:
    """First-fit allocator of contiguous slot ranges in [0, capacity)."""

    def __init__(self, capacity: int):
        self.free = [(0, capacity)]          # sorted (start, length)

    def alloc(self, n: int):
        if n == 0:
            return (0, 0)
        for i, (s, ln) in enumerate(self.free):
            if ln >= n:
                if ln == n:
                    self.free.pop(i)
                else:
                    self.free[i] = (s + n, ln - n)
                return (s, n)
        return None

    def release(self, rng):
        s, n = rng
        if n == 0:
            return
        self.free.append((s, n))
        self.free.sort()
        merged = []
        for a, ln in self.free:
            if merged and merged[-1][0] + merged[-1][1] == a:
                merged[-1] = (merged[-1][0], merged[-1][1] + ln)
            else:
                merged.append((a, ln))
        self.free = merged


@dataclass
class Session:
    sid: int
    n_rbc: int
    n_plt: int
    rbc: tuple = (0, 0)          # slot range
    plt: tuple = (0, 0)
    remaining: int = 10          # requests left before the session is freed
    busy: bool = False
    initialised: bool = False    # resident in slots
    saved: object = None         # (x, v) pinned host copies while moved out
    last_tick: int = -1          # last tick that stepped it (eviction order)
    moved: int = 0               # times moved out to host memory


@dataclass
class Request:
    rid: int
    arrival: float               # seconds from the start of the run
    session: int
    done: float = -1.0
    tick: int = -1


@dataclass
class Tick:
    index: int
    requests: list
    event: object = None


class SlotPool:
    """Device-resident slots for RBC and platelet cells (one library batch over all slots)."""

    def __init__(self, cell_types: dict, rest: dict, hbm_budget_bytes: int, rbc_fraction=0.8,
                 dt=0.1):
        import torch
        nv = {k: cell_types[k].info()["n_vertices"] for k in (RBC, PLT)}
        per_mix = rbc_fraction * nv[RBC] + (1 - rbc_fraction) * nv[PLT]
        n_cells = int(hbm_budget_bytes // (BYTES_PER_VERTEX * per_mix))
        self.cap = {RBC: int(rbc_fraction * n_cells), PLT: n_cells - int(rbc_fraction * n_cells)}
        types = [cell_types[RBC]] * self.cap[RBC] + [cell_types[PLT]] * self.cap[PLT]
        self.batch = N.Batch(types, precision=32, form="fused")
        self.nv = nv
        self.first = {RBC: 0, PLT: self.cap[RBC]}           # first cell id of each type
        V = self.batch.vertex_count
        self.x = torch.zeros((3, V), dtype=torch.float32, device="cuda")
        self.v = torch.zeros_like(self.x)
        self.f = torch.zeros_like(self.x)
        self.alloc = {RBC: RangeAllocator(self.cap[RBC]), PLT: RangeAllocator(self.cap[PLT])}
        self.rest = {k: torch.tensor(np.ascontiguousarray(rest[k].T), dtype=torch.float32,
                                     device="cuda") for k in (RBC, PLT)}
        self.dt = dt
        self.bytes = BYTES_PER_VERTEX * V

    def vertex_range(self, kind: int, rng) -> slice:
        c0 = self.first[kind] + rng[0]
        v0 = int(self.batch.offsets[c0])
        return slice(v0, v0 + rng[1] * self.nv[kind])

    def cell_ids(self, kind: int, rng) -> np.ndarray:
        return np.arange(self.first[kind] + rng[0], self.first[kind] + rng[0] + rng[1],
                         dtype=np.int32)


def request_forces(pool: SlotPool, sess: Session, rid: int, sigma: float):
    """Seeded N(0, sigma) forces of request `rid` into the session's force slots."""
    import torch
    g = torch.Generator(device="cuda")
    g.manual_seed(1_000_003 * rid + 17)
    for kind, rng in ((RBC, sess.rbc), (PLT, sess.plt)):
        if rng[1]:
            sl = pool.vertex_range(kind, rng)
            pool.f[:, sl] = sigma * torch.randn((3, sl.stop - sl.start), generator=g,
                                                device="cuda", dtype=torch.float32)


def init_session_state(pool: SlotPool, sess: Session, seed: int, spread: float = 200.0):
    """Place the session's cells at seeded positions (rest shapes translated), v = 0."""
    import torch
    g = torch.Generator(device="cuda")
    g.manual_seed(7_000_001 * sess.sid + 3)
    for kind, rng in ((RBC, sess.rbc), (PLT, sess.plt)):
        if rng[1]:
            sl = pool.vertex_range(kind, rng)
            shift = spread * torch.rand((3, rng[1], 1), generator=g, device="cuda")
            pool.x[:, sl] = (pool.rest[kind][:, None, :] + shift).reshape(3, -1)
            pool.v[:, sl] = 0.0


class StepServer:
    def __init__(self, pool: SlotPool, n_pd_iters: int = 10, sigma: float = 1.0,
                 max_in_flight: int = 2):
        self.pool = pool
        self.K = n_pd_iters
        self.sigma = sigma
        self.max_in_flight = max_in_flight
        self.sessions: dict[int, Session] = {}
        self.track: set = set()          # session ids whose final state is kept
        self.finals: dict = {}           # sid -> (x, v) host copies at release / end of run
        self.resident = 0                # cells of the admitted sessions
        self.peak_resident = 0
        self.evictions = 0               # sessions moved out to host memory
        self.restores = 0                # ... and back
        self.protect: set = set()        # sessions of the tick being built (never moved out)

    def _try_slots(self, sess: Session) -> bool:
        r = self.pool.alloc[RBC].alloc(sess.n_rbc)
        if r is None:
            return False
        p = self.pool.alloc[PLT].alloc(sess.n_plt)
        if p is None:
            self.pool.alloc[RBC].release(r)
            return False
        sess.rbc, sess.plt = r, p
        return True

    def _evict(self, sess: Session):
        """Move an idle resident session's x and v to pinned host memory and free its slots."""
        import torch
        saved = []
        for kind, rng in ((RBC, sess.rbc), (PLT, sess.plt)):
            if rng[1]:
                sl = self.pool.vertex_range(kind, rng)
                hx = torch.empty((2, 3, sl.stop - sl.start), dtype=torch.float32, pin_memory=True)
                hx[0].copy_(self.pool.x[:, sl], non_blocking=True)
                hx[1].copy_(self.pool.v[:, sl], non_blocking=True)
                saved.append(hx)
            else:
                saved.append(None)
        sess.saved = saved
        self.pool.alloc[RBC].release(sess.rbc)
        self.pool.alloc[PLT].release(sess.plt)
        sess.rbc = sess.plt = (0, 0)
        sess.initialised = False
        sess.moved += 1
        self.resident -= sess.n_rbc + sess.n_plt
        self.evictions += 1

    def _admit(self, sess: Session) -> bool:
        if sess.initialised:
            return True
        if not self._try_slots(sess):
            # move idle sessions out, least recently stepped first, until the slots fit
            idle = sorted((s for s in self.sessions.values()
                           if s.initialised and not s.busy and s.sid not in self.protect),
                          key=lambda s: s.last_tick)
            for s in idle:
                self._evict(s)
                if self._try_slots(sess):
                    break
            else:
                return False
        if sess.saved is not None:   # back from host memory, in stream order
            for (kind, rng), hx in zip(((RBC, sess.rbc), (PLT, sess.plt)), sess.saved):
                if rng[1]:
                    sl = self.pool.vertex_range(kind, rng)
                    self.pool.x[:, sl].copy_(hx[0], non_blocking=True)
                    self.pool.v[:, sl].copy_(hx[1], non_blocking=True)
            sess.saved = None
            self.restores += 1
        else:
            init_session_state(self.pool, sess, sess.sid)
        sess.initialised = True
        self.resident += sess.n_rbc + sess.n_plt
        self.peak_resident = max(self.peak_resident, self.resident)
        return True

    def _snapshot(self, sess: Session):
        import torch
        xs, vs = [], []
        if sess.saved is not None:   # moved out: the host copies (after their copies finish)
            torch.cuda.current_stream().synchronize()
            for hx in sess.saved:
                if hx is not None:
                    xs.append(hx[0].double().numpy())
                    vs.append(hx[1].double().numpy())
        else:
            for kind, rng in ((RBC, sess.rbc), (PLT, sess.plt)):
                if rng[1]:
                    sl = self.pool.vertex_range(kind, rng)
                    xs.append(self.pool.x[:, sl].double().cpu().numpy())
                    vs.append(self.pool.v[:, sl].double().cpu().numpy())
        self.finals[sess.sid] = (np.concatenate(xs, axis=1), np.concatenate(vs, axis=1))

    def _release(self, sess: Session):
        if sess.sid in self.track:
            self._snapshot(sess)
        sess.saved = None
        self.pool.alloc[RBC].release(sess.rbc)
        self.pool.alloc[PLT].release(sess.plt)
        sess.rbc = sess.plt = (0, 0)
        sess.initialised = False
        self.resident -= sess.n_rbc + sess.n_plt

    def warmup(self):
        """Run one tick of the whole request path (state set-up, seeded forces, active list,
        step, copy-out) on one slot of each cell type, outside any timing. The first use of
        these paths in a process loads GPU code and creates generators (~150 ms here), which
        would otherwise land on the first requests. Slot allocation is left as it was, and the
        slots' contents are rewritten when a session is admitted to them."""
        import torch
        tmp = Session(sid=-1, n_rbc=1 if self.pool.cap[RBC] else 0,
                      n_plt=1 if self.pool.cap[PLT] else 0, remaining=1)
        if not self._admit(tmp):
            return
        request_forces(self.pool, tmp, 0, self.sigma)
        ids = np.concatenate([self.pool.cell_ids(RBC, tmp.rbc), self.pool.cell_ids(PLT, tmp.plt)])
        self.pool.batch.set_active(ids)
        ev = torch.cuda.Event(enable_timing=True)
        self.pool.batch.step(self.pool.x, self.pool.v, self.pool.f, self.pool.dt, self.K)
        ev.record(torch.cuda.current_stream())
        while not ev.query():
            time.sleep(0.0002)
        self._snapshot(tmp)
        self.finals.pop(tmp.sid, None)
        self.pool.alloc[RBC].release(tmp.rbc)
        self.pool.alloc[PLT].release(tmp.plt)
        self.resident -= tmp.n_rbc + tmp.n_plt
        self.peak_resident = 0
        self.pool.batch.set_active(None)
        self.pool.batch.check()

    def run(self, requests: list, sessions: dict, on_tick=None):
        """Serve `requests` (sorted by arrival) in real time; returns per-request latencies.

        One warm-up tick runs first (see warmup). The Python garbage collector is paused for
        the duration of the loop (after one full collection): a collection pass over a large
        heap stalls the host for up to a few hundred milliseconds, and every request in flight
        would wait for it."""
        import gc
        self.warmup()
        was_enabled = gc.isenabled()
        gc.collect()
        gc.disable()
        try:
            return self._run(requests, sessions, on_tick)
        finally:
            if was_enabled:
                gc.enable()

    def _run(self, requests: list, sessions: dict, on_tick=None):
        import torch
        self.sessions = sessions
        stream = torch.cuda.current_stream()
        pending = deque(requests)
        waiting: list = []
        in_flight: deque = deque()
        ticks = []
        torch.cuda.synchronize()
        start_ev = torch.cuda.Event(enable_timing=True)
        start_ev.record(stream)
        t0 = time.perf_counter()
        busy_ms = 0.0
        n_cells_stepped = 0
        waited: set = set()              # requests held back at least once for want of slots
        while pending or waiting or in_flight:
            now = time.perf_counter() - t0
            while pending and pending[0].arrival <= now:
                waiting.append(pending.popleft())
            # retire finished ticks
            while in_flight and in_flight[0].event.query():
                tk = in_flight.popleft()
                t_done = start_ev.elapsed_time(tk.event) * 1e-3
                for rq in tk.requests:
                    rq.done = t_done
                    s = self.sessions[rq.session]
                    s.busy = False
                    s.remaining -= 1
                    if s.remaining <= 0:
                        self._release(s)
            # admit: one request per idle session, in arrival order
            batch_reqs = []
            if len(in_flight) < self.max_in_flight:
                still = []
                self.protect = set()
                for rq in waiting:
                    s = self.sessions[rq.session]
                    if not s.busy and self._admit(s):
                        s.busy = True
                        self.protect.add(s.sid)
                        batch_reqs.append(rq)
                    else:
                        if not s.busy:
                            waited.add(rq.rid)
                        still.append(rq)
                waiting = still
            # slots held by live sessions come free when their last requests (still to arrive
            # or waiting) are done; only with no session resident can a wait last forever
            if not batch_reqs and not in_flight and waiting and self.resident == 0:
                raise RuntimeError("slot pool too small: waiting requests can never be admitted")
            if batch_reqs:
                ids = []
                for rq in batch_reqs:
                    s = self.sessions[rq.session]
                    request_forces(self.pool, s, rq.rid, self.sigma)
                    ids.append(self.pool.cell_ids(RBC, s.rbc))
                    ids.append(self.pool.cell_ids(PLT, s.plt))
                cells = np.concatenate(ids)
                self.pool.batch.set_active(cells)
                e0 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                self.pool.batch.step(self.pool.x, self.pool.v, self.pool.f, self.pool.dt, self.K)
                ev = torch.cuda.Event(enable_timing=True)
                ev.record(stream)
                tk = Tick(len(ticks), batch_reqs, ev)
                tk.start = e0
                tk.n_cells = len(cells)
                for rq in batch_reqs:
                    rq.tick = tk.index
                    self.sessions[rq.session].last_tick = tk.index
                ticks.append(tk)
                in_flight.append(tk)
                n_cells_stepped += len(cells)
                if on_tick:
                    on_tick(tk)
            elif not in_flight:
                time.sleep(0.0002)
        torch.cuda.synchronize()
        total = time.perf_counter() - t0
        for sid in self.track:
            s = self.sessions[sid]
            if (s.initialised or s.saved is not None) and sid not in self.finals:
                self._snapshot(s)
        for tk in ticks:
            busy_ms += tk.start.elapsed_time(tk.event)
        self.pool.batch.set_active(None)
        return {"ticks": ticks, "wall_s": total, "busy_ms": busy_ms,
                "cells_stepped": n_cells_stepped, "admission_waits": len(waited),
                "peak_cells_resident": self.peak_resident, "evictions": self.evictions,
                "restores": self.restores}


def poisson_workload(duration_s: float, rate: float, seed: int, n_min=50, n_max=10_000,
                     rbc_fraction=0.8, continue_prob=0.8, per_session=10):
    """Seeded arrivals: (requests, sessions). Each request continues a live session with
    probability continue_prob (the oldest live session with requests left), else opens a
    new one with N = round(exp U[ln n_min, ln n_max]) cells split rbc_fraction/rest."""
    rng = np.random.default_rng(seed)
    t = 0.0
    reqs, sessions, live = [], {}, []
    used: dict = {}
    rid = 0
    while True:
        t += rng.exponential(1.0 / rate)
        if t > duration_s:
            break
        if live and rng.uniform() < continue_prob:
            sid = live[int(rng.integers(len(live)))]
        else:
            n = int(round(np.exp(rng.uniform(np.log(n_min), np.log(n_max)))))
            n_r = int(round(rbc_fraction * n))
            sid = len(sessions)
            sessions[sid] = Session(sid, n_r, n - n_r, remaining=per_session)
            live.append(sid)
        reqs.append(Request(rid, t, sid))
        rid += 1
        used[sid] = used.get(sid, 0) + 1
        if used[sid] >= per_session:
            live.remove(sid)
    # a session ends with its last request of the run (at most per_session of them)
    for sid, s in sessions.items():
        s.remaining = used.get(sid, 0)
    return reqs, sessions


def replay_alone(cell_types: dict, rest: dict, sess_def: Session, request_ids: list,
                 n_pd_iters: int, sigma: float, budget_bytes: int = 64 << 20):
    """Run one session's requests one after another in a pool of its own; returns (x, v)."""
    import torch
    pool = SlotPool(cell_types, rest, budget_bytes)
    srv = StepServer(pool, n_pd_iters, sigma)
    s = Session(sess_def.sid, sess_def.n_rbc, sess_def.n_plt, remaining=len(request_ids) + 1)
    srv.sessions = {s.sid: s}
    if not srv._admit(s):
        raise RuntimeError("session does not fit the replay pool")
    cells = np.concatenate([pool.cell_ids(RBC, s.rbc), pool.cell_ids(PLT, s.plt)])
    pool.batch.set_active(cells)
    for rid in request_ids:
        request_forces(pool, s, rid, sigma)
        pool.batch.step(pool.x, pool.v, pool.f, pool.dt, n_pd_iters)
    torch.cuda.synchronize()
    srv._snapshot(s)
    return srv.finals[s.sid]


def latency_summary(requests: list) -> dict:
    lat = np.array([r.done - r.arrival for r in requests if r.done >= 0]) * 1e3
    if lat.size == 0:
        return {"n": 0}
    return {"n": int(lat.size), "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)), "max_ms": float(lat.max()),
            "mean_ms": float(lat.mean())}
