"""Continuous-batching service of data-assimilation cycles on one GPU.

A *session* is one ensemble kept resident in device memory between cycles,
with its own plan (made with LETKF_FLAG_CYCLE) and observation arrays.  A
*request* asks for one cycle of a session: n lattice-BGK steps, then one
LETKF analysis (the DA cycle of Sec. II-B), all inside ``letkf_cycle``.

Scheduling:
* admission by device-memory budget: a session is materialised (plan
  workspace + ensemble) on its first request if the budget allows, otherwise
  idle resident sessions are evicted least-recently-used first; if nothing can
  be evicted the request waits;
* a session runs one cycle at a time (its cycles are sequential);
* every other ready request is dispatched at once to a free stream slot, so
  requests that arrive while others run overlap with them on the device;
* completion is observed through per-request events; latency = completion
  time - arrival time (host clock);
* once a cycle's event has fired, the session plan's device status is read
  (without waiting on anything else) and kept on the request: a cycle that
  found an invalid observation, a non-finite value or an unconverged
  eigensolve is counted as failed, not served.

Each session owns all of its device memory, so a session's results are the
same alone and in any mix (checked by a GPU test, bitwise).
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np

from . import letkf as L
from . import synth


@dataclasses.dataclass
class SessionSpec:
    name: str
    wl: synth.Workload
    n_steps: int = 50
    tau: float = 0.52
    force_amp: float = 1e-5
    force_kx: int = 4
    precision: int = L.LETKF_PREC_FP64


class Session:
    def __init__(self, sid: int, spec: SessionSpec):
        self.sid = sid
        self.spec = spec
        self.problem = synth.make_problem(spec.wl)   # host copy of the initial state + obs
        self.plan: Optional[int] = None
        self.x = None
        self.obs = None
        self.bytes = 0
        self.busy = False
        self.last_used = 0.0
        self.cycles_done = 0
        self.host_state: Optional[np.ndarray] = None   # state saved at eviction

    # device residency -------------------------------------------------------
    def materialise(self):
        import torch
        p, wl = self.problem, self.spec.wl
        self.plan = L.letkf_plan([L.make_problem(wl.nx, wl.ny, wl.k, len(p.obs_ix), wl.L, wl.infl,
                                                 precision=self.spec.precision)],
                                 flags=L.LETKF_FLAG_CYCLE)
        dev = torch.device("cuda:0")
        start = self.host_state if self.host_state is not None else p.xb
        self.x = torch.from_numpy(start).to(dev)
        f = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
        self.obs = (f(p.obs_ix), f(p.obs_iy), f(p.obs_kind), f(p.obs_val), f(p.obs_var))
        self.bytes = L.letkf_plan_workspace_bytes(self.plan) + self.x.numel() * 8 + sum(
            t.numel() * t.element_size() for t in self.obs)
        torch.cuda.current_stream().synchronize()   # uploads done before any slot stream reads

    def release(self, keep_state: bool = False):
        """Free the device memory; keep_state saves the ensemble to host memory
        first (eviction), so a later admission continues from it."""
        if keep_state and self.x is not None:
            self.host_state = self.x.cpu().numpy()
        if self.plan is not None:
            L.letkf_plan_destroy(self.plan)
        self.plan, self.x, self.obs, self.bytes = None, None, None, 0

    def state(self) -> np.ndarray:
        return self.x.cpu().numpy() if self.x is not None else self.host_state

    @property
    def resident(self) -> bool:
        return self.plan is not None

    def footprint(self) -> int:
        """Device bytes the session needs when resident (estimated before admission)."""
        wl = self.spec.wl
        n_obs = len(self.problem.obs_ix)
        state = wl.nx * wl.ny * 9 * wl.k * 8
        kp = max(16, 1 << (wl.k - 1).bit_length())
        nb = (kp // 16) * (kp // 16 + 1) // 2
        npts = wl.nx * wl.ny
        slab = min(npts, max(256, (1 << 30) // ((nb * 256 + kp) * 8)))
        return 3 * state + n_obs * (kp * 8 + 60) + slab * (nb * 256 + kp) * 8 + (1 << 20)

    def dispatch(self, stream):
        s = self.spec
        io = L.make_cycle_io(0, self.x, self.obs, s.n_steps, s.tau, s.force_amp, s.force_kx)
        L.letkf_cycle(self.plan, [io], stream)

    def status(self) -> int:
        """Device status of the session's cycles since the last read; the
        caller has seen the cycle's completion event, so nothing is waited on."""
        return L.letkf_status(self.plan, sync=False)


@dataclasses.dataclass
class Request:
    rid: int
    sid: int
    t_arrive: float
    t_dispatch: float = 0.0
    t_done: float = 0.0
    status: int = -1          # LETKF_* code of the cycle once done


class AssimilationServer:
    def __init__(self, specs: Sequence[SessionSpec], budget_bytes: int, n_slots: int = 8):
        import torch
        self.sessions = [Session(i, sp) for i, sp in enumerate(specs)]
        self.budget = int(budget_bytes)
        self.used = 0
        self.streams = [torch.cuda.Stream() for _ in range(n_slots)]   # default priority
        self.free_slots = list(range(n_slots))
        self.waiting: collections.deque = collections.deque()
        self.running: Dict[int, tuple] = {}     # slot -> (request, event, session)
        self.done: List[Request] = []
        self.admissions = 0
        self.evictions = 0

    # memory -----------------------------------------------------------------
    def _admit(self, sess: Session) -> bool:
        need = sess.footprint()
        if need > self.budget:
            raise ValueError(f"session {sess.sid} needs {need} bytes, over the whole budget")
        while self.used + need > self.budget:
            idle = [s for s in self.sessions if s.resident and not s.busy]
            if not idle:
                return False
            victim = min(idle, key=lambda s: s.last_used)
            self.used -= victim.bytes
            victim.release(keep_state=True)
            self.evictions += 1
        sess.materialise()
        self.used += sess.bytes
        self.admissions += 1
        return True

    # scheduling -------------------------------------------------------------
    def submit(self, req: Request):
        self.waiting.append(req)

    def _try_dispatch(self, now: float):
        if not self.free_slots:
            return
        still = collections.deque()
        while self.waiting:
            req = self.waiting.popleft()
            sess = self.sessions[req.sid]
            if not self.free_slots or sess.busy:
                still.append(req)
                continue
            if not sess.resident and not self._admit(sess):
                still.append(req)
                continue
            slot = self.free_slots.pop()
            stream = self.streams[slot]
            import torch
            with torch.cuda.stream(stream):
                sess.dispatch(stream)
                ev = torch.cuda.Event()
                ev.record(stream)
            sess.busy = True
            req.t_dispatch = now
            self.running[slot] = (req, ev, sess)
        self.waiting = still

    def _poll(self, now: float):
        for slot in list(self.running):
            req, ev, sess = self.running[slot]
            if ev.query():
                req.t_done = time.perf_counter()
                req.status = sess.status()
                sess.busy = False
                sess.last_used = req.t_done
                sess.cycles_done += 1
                self.done.append(req)
                del self.running[slot]
                self.free_slots.append(slot)

    def step(self):
        now = time.perf_counter()
        self._poll(now)
        self._try_dispatch(now)

    def drain(self):
        while self.waiting or self.running:
            self.step()

    def run_poisson(self, rate_hz: float, n_requests: int, seed: int = 4,
                    pick: Optional[Callable[[np.random.Generator], int]] = None) -> dict:
        """Arrivals with exponential gaps of mean 1/rate; returns latency stats."""
        rng = np.random.default_rng(seed)
        gaps = rng.exponential(1.0 / rate_hz, size=n_requests)
        sids = [pick(rng) if pick else int(rng.integers(len(self.sessions)))
                for _ in range(n_requests)]
        t0 = time.perf_counter()
        arrivals = t0 + np.cumsum(gaps)
        i = 0
        while i < n_requests or self.waiting or self.running:
            now = time.perf_counter()
            while i < n_requests and arrivals[i] <= now:
                self.submit(Request(i, sids[i], float(arrivals[i])))
                i += 1
            self.step()
        t1 = time.perf_counter()
        done = self.done[-n_requests:]
        ok = [r for r in done if r.status == L.LETKF_OK]
        lat = np.array([r.t_done - r.t_arrive for r in ok]) * 1e3
        points = sum(self.sessions[r.sid].spec.wl.nx * self.sessions[r.sid].spec.wl.ny
                     for r in ok)
        codes: Dict[str, int] = {}
        for r in done:
            if r.status != L.LETKF_OK:
                name = L.letkf_strerror(r.status) if r.status >= 0 else "no status"
                codes[name] = codes.get(name, 0) + 1
        pct = lambda q: round(float(np.percentile(lat, q)), 3) if len(lat) else None
        return {"requests": n_requests, "offered_rate_hz": rate_hz,
                "wall_s": round(t1 - t0, 3),
                "served": len(ok), "failed": len(done) - len(ok), "failures": codes,
                "throughput_cycles_per_s": round(len(ok) / (t1 - t0), 2),
                "throughput_analyses_per_s": round(points / (t1 - t0), 1),
                "p50_ms": pct(50), "p99_ms": pct(99),
                "mean_ms": round(float(lat.mean()), 3) if len(lat) else None,
                "admissions": self.admissions, "evictions": self.evictions,
                "slots": len(self.streams), "budget_bytes": self.budget}

    def close(self):
        import torch
        torch.cuda.synchronize()
        for s in self.sessions:
            s.release()
        self.used = 0


def default_specs(n_sessions: int = 12, seed: int = 4, with_large: bool = True) -> List[SessionSpec]:
    """Sessions mixing the shapes of the three analysis workloads: one of the
    1024^2, k = 64 precision workload (FP32 form), two of the 256^2, k = 32
    FP64 workload (stride 2, L = 8, each with its own seed), and the rest
    drawn by the mixed-batch recipe (lattices 64^2-512^2, k in {16, 32, 64},
    random masks with clustered gaps, L 4-16, sigma 0.002-0.01; FP32 form).
    with_large=False leaves out the 1024^2 session."""
    out = []
    if with_large:
        big = dataclasses.replace(synth.WORKLOADS["grid1024_k64"], name="s_grid1024_k64", seed=400)
        out.append(SessionSpec(big.name, big, precision=L.LETKF_PREC_FP32))
    for j in range(2):
        wl = dataclasses.replace(synth.WORKLOADS["grid256_k32"], name=f"s_grid256_k32_{j}",
                                 seed=410 + j)
        out.append(SessionSpec(wl.name, wl))
    for wl in synth.batching_workloads(max(n_sessions - len(out), 0), seed=seed):
        out.append(SessionSpec(f"s_{wl.name}", wl, precision=L.LETKF_PREC_FP32))
    return out[:n_sessions]
