"""Continuous-batching server for sweep requests on one GPU.

Two request kinds:
* a domain job: one periodic lattice (size, steps, sponge strength and width,
  damping variant, Mach number) run from a centred Gaussian pulse; the result
  is its FP64 diagnostics vector (mass, momentum, energy sums, max deviation,
  non-finite count) after the requested number of steps;
* a Von Neumann job: the eigenvalues of the amplification matrix on an
  n_k x n_k wavenumber grid for one parameter set.

Scheduling. Requests enter a FIFO queue when they arrive. A domain job is
admitted when its device footprint fits the free HBM budget and a slot is
free; its lattice then stays resident until it is done. The server runs ticks:
each tick advances every resident domain by up to ``tick`` steps in one
batched persistent launch per step (the members that need fewer steps stop
early), then retires finished domains and admits waiting ones, so requests
that arrive while others are on the GPU join at the next tick boundary.
Von Neumann jobs run on a second stream and overlap the ticks. Latency is
measured from a request's arrival to its result being on the host.

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
    second stream. Device memory comes from torch's caching allocator."""

    def __init__(self, keep_state=False, blocks_per_cu=8):
        import torch
        from . import lbm
        self.torch = torch
        self.lbm = lbm
        lbm.load()
        self.stream = torch.cuda.Stream()
        self.vn_stream = torch.cuda.Stream()
        self.batch = None
        self.blocks_per_cu = blocks_per_cu
        self.keep_state = keep_state
        self._members = []

    def footprint(self, req):
        spec = req.spec
        cfg = self.lbm.make_config(spec.nx, spec.ny, storage=spec.storage, variant=spec.variant)
        return self.lbm.lbm_required_bytes(cfg) + 8 * (spec.nx + spec.ny) + 8 * spec.nx * spec.ny

    def admit(self, req):
        torch, lbm = self.torch, self.lbm
        spec = req.spec
        cfg = lbm.make_config(spec.nx, spec.ny, storage=spec.storage, variant=spec.variant, s=spec.s,
                              rho_base=spec.rho0, ux_base=spec.base_state[1], stream=self.stream)
        nbytes = lbm.lbm_required_bytes(cfg) // 2
        with torch.cuda.stream(self.stream):
            bufs = [torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda") for _ in range(2)]
            rho, _, _ = spec.fields()
            rho_dev = torch.from_numpy(rho).pin_memory().to("cuda", non_blocking=True)
        a = [b[(-b.data_ptr()) % 256:] for b in bufs]  # 256-byte aligned views
        h = lbm.lbm_create_ext(cfg, a[0], a[1])
        cx, cy = spec.chi_1d()
        lbm.lbm_set_sponge_separable(h, cx, cy, "max", spec.qref)
        lbm.lbm_init_fields_dev(h, rho_dev)
        return {"h": h, "bufs": bufs, "rho": rho_dev}

    def tick(self, states, steps, tick):
        lbm = self.lbm
        handles = [s["h"] for s in states]
        if self.batch is None:
            self.batch = lbm.lbm_batch_create(handles, self.stream)
            lbm.lbm_batch_set_grid(self.batch, self.blocks_per_cu)
        elif handles != self._members:
            lbm.lbm_batch_set_members(self.batch, handles)
        self._members = handles
        lbm.lbm_batch_tick(self.batch, tick, steps)
        lbm.lbm_batch_sync(self.batch)

    def result(self, state):
        lbm = self.lbm
        d = lbm.lbm_diagnostics(state["h"])
        out = {"diagnostics": d}
        if self.keep_state:
            out["state"] = lbm.lbm_save_state(state["h"])
        self._release(state)
        return out

    def _release(self, state):
        # the batch drops the handle at the next tick, before it reads the
        # member list again
        self.lbm.lbm_destroy(state["h"])
        state["h"] = None
        state["bufs"] = None
        state["rho"] = None

    def vn_submit(self, req):
        torch, lbm = self.torch, self.lbm
        kx, ky = wl.vn_grid(req.nk)
        with torch.cuda.stream(self.vn_stream):
            dkx = torch.from_numpy(kx).to("cuda", non_blocking=True)
            dky = torch.from_numpy(ky).to("cuda", non_blocking=True)
            eig = torch.empty((1, kx.size, 9, 2), dtype=torch.float64, device="cuda")
            lbm.vn_amplification_dev([req.vn_params], dkx, dky, eig, stream=self.vn_stream)
            host = torch.empty(eig.shape, dtype=torch.float64, pin_memory=True)
            host.copy_(eig, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(self.vn_stream)
        return {"ev": ev, "host": host, "keep": (dkx, dky, eig)}

    def vn_poll(self, job):
        if not job["ev"].query():
            return None
        lam = job["host"].numpy()[0]
        lam = lam[..., 0] + 1j * lam[..., 1]
        return {"max_abs_lambda": float(np.abs(lam).max()), "eig": lam}

    def close(self):
        if self.batch is not None:
            self.lbm.lbm_batch_destroy(self.batch)
            self.batch = None
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
                "peak_gb": self.peak_bytes / 1e9, "wall_s": self.wall}


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

    def run(self, requests, order_of_admission=None):
        """Serve ``requests`` (sorted by arrival, times in seconds) in real time.
        Returns ServeStats; each request gets t_admit, t_done, result."""
        st = ServeStats()
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        queue = collections.deque()
        active = []      # [req, state, remaining, footprint]
        vn_jobs = []     # [req, job]
        used = 0
        t0 = self.clock()
        while pending or queue or active or vn_jobs:
            now = self.clock() - t0
            while pending and pending[0].arrival <= now:
                queue.append(pending.popleft())
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
            if active:
                tick = self._tick_len(active)
                steps = [min(tick, a[2]) for a in active]
                ts = self.clock()
                self.ex.tick([a[1] for a in active], steps, tick)
                dt = self.clock() - ts
                done_lups = sum(s * a[0].spec.nx * a[0].spec.ny for s, a in zip(steps, active))
                st.lups += done_lups
                st.ticks += 1
                if dt > 0 and done_lups > 0:
                    self.rate_est = 0.7 * self.rate_est + 0.3 * done_lups / dt
                keep = []
                for s, a in zip(steps, active):
                    a[2] -= s
                    if a[2] == 0:
                        a[0].result = self.ex.result(a[1])
                        a[0].t_done = self.clock() - t0
                        used -= a[3]
                        lat = a[0].t_done - a[0].arrival
                        st.latencies.append(lat)
                        st.domain_latencies.append(lat)
                    else:
                        keep.append(a)
                active = keep
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
                if vn_jobs:
                    self.sleep(0.0005)
                elif pending:
                    wait = pending[0].arrival - (self.clock() - t0)
                    if wait > 0:
                        self.sleep(min(wait, 0.05))
        st.wall = self.clock() - t0
        return st
