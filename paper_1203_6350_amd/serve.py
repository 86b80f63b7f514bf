"""Continuous-batching server for sweep requests on one GPU.

Two request kinds:
* a domain job: one periodic lattice (size, steps, sponge strength and width,
  damping variant, Mach number) run from a centred Gaussian pulse; the result
  is its FP64 diagnostics vector (mass, momentum, energy sums, max deviation,
  non-finite count) after the requested number of steps;
* a Von Neumann job: the eigenvalues of the amplification matrix on an
  n_k x n_k wavenumber grid for one parameter set.

Scheduling. Requests enter a FIFO queue when they arrive, and the host
part of a domain job's set-up (its initial fields) starts on a worker
thread at once. A domain job is admitted when its device footprint fits
the free HBM budget and a slot is free; its lattice then stays resident
until it is done. The server runs ticks: each tick advances every resident
domain by up to ``tick`` steps in one batched launch per K steps (the
members that need fewer steps stop early). Ticks are pipelined: the next
tick is enqueued before the previous one has finished (two in flight), the
diagnostics of the domains that finish in a tick are enqueued behind it and
copied to pinned host memory, and a tick's finished domains are retired
when its completion event fires. Admission, retirement and the next tick's
launch therefore run on the host while the device works on the tick before.
Requests that arrive while others are on the GPU join at the next tick.
Von Neumann jobs run on a second stream and overlap the ticks. Latency is
measured from a request's arrival to its result being on the host. A domain
whose state holds non-finite values at the end (Type I with s + chi > 2
blows up, Sec. 2.2.1) is reported with ``unstable = True``.

The scheduler talks to an executor object; ``GpuExecutor`` drives liblbm.
"""
from __future__ import annotations

import collections
import math
import time
from dataclasses import dataclass, field

import numpy as np

from . import workloads as wl


@dataclass
class Request:
    rid: int
    kind: str                 # "domain" or "vn"
    arrival: float            # seconds after the start of the run
    spec: object = None       # DomainSpec for domain jobs
    steps: int = 0
    vn_params: dict = None
    nk: int = 0
    t_admit: float = None
    t_done: float = None
    result: object = None
    error: str = None


def make_requests(rate, count, seed=5, domain_fraction=0.5, n_range=(64, 1024),
                  step_range=(500, 5000), nk_range=(64, 256), storage="f32"):
    """Open-loop Poisson arrivals at ``rate`` requests/s with the parameter
    distributions of the serving workload (seeded)."""
    g = wl.rng(4, salt=seed)
    t = 0.0
    out = []
    for rid in range(count):
        t += g.exponential(1.0 / rate)
        if g.uniform() < domain_fraction:
            N = int(round(math.exp(g.uniform(math.log(n_range[0]), math.log(n_range[1])))))
            steps = int(g.integers(step_range[0], step_range[1] + 1))
            chi_max = float(g.uniform(0.01, 0.5))
            W = wl.clamp_width(int(g.integers(8, 65)), N)
            ma = float(g.uniform(0.0, 0.3))
            var = ("I", "II", "III")[int(g.integers(0, 3))]
            c = (N - 1) / 2
            spec = wl.DomainSpec(nx=N, ny=N, variant=var, storage=storage, chi_max=chi_max,
                                 width=W, u0=ma * wl.CS, pulses=[(c, c, 1e-3, N / 20.0)],
                                 steps=steps, seed=rid)
            out.append(Request(rid, "domain", t, spec=spec, steps=steps))
        else:
            nk = int(round(math.exp(g.uniform(math.log(nk_range[0]), math.log(nk_range[1])))))
            var = ("I", "II", "III")[int(g.integers(0, 3))]
            p = dict(s=wl.S_MRT_DEFAULT, chi=float(g.uniform(0.01, 0.5)),
                     qref=(1.0, float(g.uniform(0.0, 0.3)) * wl.CS, 0.0), variant=var, n=0.5, m=0.5)
            out.append(Request(rid, "vn", t, vn_params=p, nk=nk))
    return out


# ---------------------------------------------------------------- GPU executor

class GpuExecutor:
    """Runs admitted domains through one liblbm batch and Von Neumann jobs on a
    second stream. Device memory comes from torch's caching allocator; all of
    the batch's lattices live on the batch's stream, so member changes,
    ticks, diagnostics and frees are ordered by that stream alone."""

    def __init__(self, keep_state=False, blocks_per_cu=8, workers=8):
        import concurrent.futures
        import torch
        from . import lbm
        self.torch = torch
        self.lbm = lbm
        lbm.load()
        self.stream = torch.cuda.Stream()
        self.vn_stream = torch.cuda.Stream()
        self._sptr = int(self.stream.cuda_stream)
        self._vn_sptr = int(self.vn_stream.cuda_stream)
        self.batch = None
        self.blocks_per_cu = blocks_per_cu
        self.keep_state = keep_state
        self._members = []      # handles in the batch's current member list
        self._zombies = []      # finished states still in that list
        self._pool = concurrent.futures.ThreadPoolExecutor(max_workers=workers)

    def footprint(self, req):
        spec = req.spec
        cfg = self.lbm.make_config(spec.nx, spec.ny, storage=spec.storage, variant=spec.variant)
        return self.lbm.lbm_required_bytes(cfg) + 8 * (spec.nx + spec.ny) + 8 * spec.nx * spec.ny

    def _host_fields(self, spec):
        """rho [ny][nx], chi_x [nx], chi_y [ny] in one pinned FP64 buffer."""
        rho, _, _ = spec.fields()
        cx, cy = spec.chi_1d()
        buf = self.torch.empty(rho.size + cx.size + cy.size, dtype=self.torch.float64,
                               pin_memory=True)
        b = buf.numpy()
        b[:rho.size] = rho.ravel()
        b[rho.size:rho.size + cx.size] = cx
        b[rho.size + cx.size:] = cy
        return buf

    def prepare(self, req):
        """Start the host part of a domain job's set-up (its initial density
        field, into pinned memory) on a worker thread."""
        req._fields = self._pool.submit(self._host_fields, req.spec)

    def admit(self, req):
        torch, lbm = self.torch, self.lbm
        spec = req.spec
        fut = getattr(req, "_fields", None)
        rho_host = fut.result() if fut is not None else self._host_fields(spec)
        req._fields = None
        cfg = lbm.make_config(spec.nx, spec.ny, storage=spec.storage, variant=spec.variant, s=spec.s,
                              rho_base=spec.rho0, ux_base=spec.base_state[1], stream=self._sptr)
        nbytes = lbm.lbm_required_bytes(cfg) // 2
        with torch.cuda.stream(self.stream):
            bufs = [torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda") for _ in range(2)]
            dev = rho_host.to("cuda", non_blocking=True)
        a = [b[(-b.data_ptr()) % 256:] for b in bufs]  # 256-byte aligned views
        n = spec.nx * spec.ny
        # nothing below waits for the device: the set-up is enqueued on the
        # batch stream behind the ticks in flight
        h = lbm.lbm_create_ext(cfg, a[0], a[1])
        lbm.lbm_set_sponge_separable_dev(h, dev[n:n + spec.nx], dev[n + spec.nx:], "max", spec.qref)
        lbm.lbm_init_fields_dev(h, dev[:n])
        return {"h": h, "bufs": bufs, "rho": dev, "rho_host": rho_host}

    def launch(self, states, steps, tick, finishing):
        """Enqueue one tick (member i takes steps[i]) and, behind it, the
        diagnostics of the states in `finishing` into pinned host memory.
        Returns a ticket for done / wait / results."""
        torch, lbm = self.torch, self.lbm
        handles = [s["h"] for s in states]
        if self.batch is None:
            self.batch = lbm.lbm_batch_create(handles, self._sptr)
            lbm.lbm_batch_set_grid(self.batch, self.blocks_per_cu)
        elif handles != self._members:
            lbm.lbm_batch_set_members(self.batch, handles)
        self._members = handles
        self._reap()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(self.stream)
        lbm.lbm_batch_tick(self.batch, tick, steps)
        n = len(finishing)
        host = None
        if n:
            with torch.cuda.stream(self.stream):
                dev = torch.empty((n, 7), dtype=torch.float64, device="cuda")
                for i, s in enumerate(finishing):
                    lbm.lbm_diagnostics_dev(s["h"], dev[i])
                host = torch.empty((n, 7), dtype=torch.float64, pin_memory=True)
                host.copy_(dev, non_blocking=True)
            keep = dev
        else:
            keep = None
        ev1.record(self.stream)
        return {"ev0": ev0, "ev1": ev1, "host": host, "keep": keep, "finishing": finishing}

    def done(self, ticket):
        return ticket["ev1"].query()

    def wait(self, ticket):
        ticket["ev1"].synchronize()

    def gpu_seconds(self, ticket):
        return ticket["ev0"].elapsed_time(ticket["ev1"]) * 1e-3

    def results(self, ticket):
        """Results of the ticket's finishing states (after done); releases
        them."""
        out = []
        diag = ticket["host"].numpy() if ticket["host"] is not None else []
        for s, d in zip(ticket["finishing"], diag):
            d = d.copy()
            r = {"diagnostics": d, "unstable": bool(d[6] > 0)}
            if self.keep_state:
                r["state"] = self.lbm.lbm_save_state(s["h"])
            out.append(r)
            self._release(s)
        return out

    def _release(self, state):
        # a handle may be destroyed once it has left the batch's member list
        # (the tick that dropped it is enqueued behind the last one that
        # advanced it); until then it waits with the zombies
        if state["h"] in self._members:
            self._zombies.append(state)
            return
        self.lbm.lbm_destroy(state["h"])
        state["h"] = None
        state["bufs"] = None
        state["rho"] = None

    def _reap(self):
        keep = []
        for z in self._zombies:
            if z["h"] in self._members:
                keep.append(z)
            else:
                self.lbm.lbm_destroy(z["h"])
                z["h"] = None
                z["bufs"] = None
                z["rho"] = None
        self._zombies = keep

    def vn_submit(self, req):
        torch, lbm = self.torch, self.lbm
        kx, ky = wl.vn_grid(req.nk)
        with torch.cuda.stream(self.vn_stream):
            dkx = torch.from_numpy(kx).to("cuda", non_blocking=True)
            dky = torch.from_numpy(ky).to("cuda", non_blocking=True)
            eig = torch.empty((1, kx.size, 9, 2), dtype=torch.float64, device="cuda")
            lbm.vn_amplification_dev([req.vn_params], dkx, dky, eig, stream=self._vn_sptr)
            host = torch.empty(eig.shape, dtype=torch.float64, pin_memory=True)
            host.copy_(eig, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(self.vn_stream)
        return {"ev": ev, "host": host, "keep": (dkx, dky, eig)}

    def vn_poll(self, job):
        if not job["ev"].query():
            return None
        # (re, im) pairs viewed as complex in place; each spectrum is sorted
        # by decreasing |lambda|, so its first entry is its largest
        lam = job["host"].numpy()[0].view(np.complex128)[..., 0]
        return {"max_abs_lambda": float(np.abs(lam[:, 0]).max()), "eig": lam}

    def close(self):
        if self.batch is not None:
            self.lbm.lbm_batch_destroy(self.batch)
            self.batch = None
        self._members = []
        self._reap()
        self._pool.shutdown(wait=True)
        self.torch.cuda.synchronize()


# ---------------------------------------------------------------- scheduler

@dataclass
class ServeStats:
    latencies: list = field(default_factory=list)
    domain_latencies: list = field(default_factory=list)
    vn_latencies: list = field(default_factory=list)
    lups: float = 0.0
    vn_kpoints: int = 0
    wall: float = 0.0
    ticks: int = 0
    admission_stalls: int = 0
    rejected: int = 0
    max_resident: int = 0
    peak_bytes: int = 0
    gpu_busy_s: float = 0.0   # device time of the ticks (their start and end events)

    def summary(self, requests=None, warmup=0):
        """Latency percentiles over requests with rid >= warmup (arrival order)."""
        if requests is not None:
            lat = np.array([r.t_done - r.arrival for r in requests
                            if r.rid >= warmup and r.t_done is not None and r.error is None])
        else:
            lat = np.array(self.latencies)
        pct = (lambda p: 1e3 * float(np.percentile(lat, p)) if lat.size else None)
        return {"p50_ms": pct(50), "p99_ms": pct(99),
                "mean_ms": 1e3 * float(lat.mean()) if lat.size else None,
                "aggregate_mlups": self.lups / self.wall / 1e6 if self.wall else 0.0,
                "vn_kpoints_per_s": self.vn_kpoints / self.wall if self.wall else 0.0,
                "ticks": self.ticks, "admission_stalls": self.admission_stalls,
                "rejected": self.rejected, "max_resident": self.max_resident,
                "peak_gb": self.peak_bytes / 1e9, "wall_s": self.wall,
                "device_busy": self.gpu_busy_s / self.wall if self.wall else 0.0}


class Server:
    def __init__(self, executor, budget_bytes=200 << 30, max_slots=256, tick=None,
                 tick_target_s=0.02, clock=time.perf_counter, sleep=time.sleep):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.max_slots = int(max_slots)
        self.fixed_tick = tick
        self.tick_target = tick_target_s
        self.clock = clock
        self.sleep = sleep
        self.rate_est = 5e10  # LUPS, refined from measured ticks

    def _tick_len(self, active):
        if self.fixed_tick:
            return int(self.fixed_tick)
        cells = sum(a[0].spec.nx * a[0].spec.ny for a in active)
        want = self.tick_target * self.rate_est / max(cells, 1)
        t = 2 ** int(round(math.log2(max(16.0, min(1024.0, want)))))
        return int(t)

    def run(self, requests, order_of_admission=None, depth=2):
        """Serve ``requests`` (sorted by arrival, times in seconds) in real time
        with up to ``depth`` ticks in flight. Returns ServeStats; each request
        gets t_admit, t_done, result."""
        st = ServeStats()
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        queue = collections.deque()
        active = []      # [req, state, remaining, footprint]
        inflight = collections.deque()  # [ticket, finishing entries, lattice updates]
        vn_jobs = []     # [req, job]
        used = 0
        prep = getattr(self.ex, "prepare", None)
        t0 = self.clock()
        while pending or queue or active or inflight or vn_jobs:
            now = self.clock() - t0
            while pending and pending[0].arrival <= now:
                r = pending.popleft()
                queue.append(r)
                if r.kind == "domain" and prep is not None:
                    prep(r)
            # admission, first come first served
            while queue:
                r = queue[0]
                if r.kind == "vn":
                    queue.popleft()
                    r.t_admit = now
                    vn_jobs.append([r, self.ex.vn_submit(r)])
                    continue
                fp = self.ex.footprint(r)
                if fp > self.budget:
                    queue.popleft()
                    r.error = "footprint %d exceeds the budget %d" % (fp, self.budget)
                    r.t_done = now
                    st.rejected += 1
                    continue
                if used + fp > self.budget or len(active) >= self.max_slots:
                    st.admission_stalls += 1
                    break
                queue.popleft()
                state = self.ex.admit(r)
                used += fp
                st.peak_bytes = max(st.peak_bytes, used)
                r.t_admit = self.clock() - t0
                if order_of_admission is not None:
                    order_of_admission.append(r.rid)
                active.append([r, state, r.steps, fp])
            st.max_resident = max(st.max_resident, len(active))
            # enqueue the next tick while the previous ones run
            if active and len(inflight) < depth:
                tick = self._tick_len(active)
                steps = [min(tick, a[2]) for a in active]
                fin = [a for s, a in zip(steps, active) if s == a[2]]
                ticket = self.ex.launch([a[1] for a in active], steps, tick, [a[1] for a in fin])
                done_lups = sum(s * a[0].spec.nx * a[0].spec.ny for s, a in zip(steps, active))
                inflight.append([ticket, fin, done_lups])
                st.ticks += 1
                for s, a in zip(steps, active):
                    a[2] -= s
                active = [a for a in active if a[2] > 0]
                continue  # admit and launch again before waiting
            # retire completed ticks in order; wait for the oldest when the
            # pipeline is full, or when nothing else is left to do
            while inflight and (self.ex.done(inflight[0][0]) or
                                (len(inflight) >= depth and active) or
                                (not active and not queue and not vn_jobs)):
                ticket, fin, done_lups = inflight.popleft()
                self.ex.wait(ticket)
                res = self.ex.results(ticket)
                t_now = self.clock() - t0
                for a, rr in zip(fin, res):
                    a[0].result = rr
                    a[0].t_done = t_now
                    used -= a[3]
                    lat = a[0].t_done - a[0].arrival
                    st.latencies.append(lat)
                    st.domain_latencies.append(lat)
                st.lups += done_lups
                gs = self.ex.gpu_seconds(ticket) if hasattr(self.ex, "gpu_seconds") else 0.0
                st.gpu_busy_s += gs
                if gs > 0 and done_lups > 0:
                    self.rate_est = 0.7 * self.rate_est + 0.3 * done_lups / gs
            still = []
            for r, job in vn_jobs:
                res = self.ex.vn_poll(job)
                if res is None:
                    still.append([r, job])
                else:
                    r.result = res
                    r.t_done = self.clock() - t0
                    lat = r.t_done - r.arrival
                    st.latencies.append(lat)
                    st.vn_latencies.append(lat)
                    st.vn_kpoints += r.nk * r.nk
            vn_jobs = still
            if not active and not queue:
                if inflight or vn_jobs:
                    self.sleep(0.0002)
                elif pending:
                    wait = pending[0].arrival - (self.clock() - t0)
                    if wait > 0:
                        self.sleep(min(wait, 0.05))
            elif queue and not active and inflight:
                self.sleep(0.0002)  # memory frees as the in-flight ticks retire
        st.wall = self.clock() - t0
        return st
