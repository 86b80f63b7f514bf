"""Scheduler logic of the server, on the CPU: a fake executor backed by the
FP64 oracle stands in for the GPU (tiny domains), and a virtual clock makes
the runs deterministic."""
import numpy as np
import pytest

import oracle
from paper_1203_6350_amd import serve, workloads as wl


class VirtualClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-6)


class FakeExecutor:
    """Oracle-backed executor: each tick advances the resident domains and
    costs virtual time proportional to the lattice updates."""

    def __init__(self, clock, lups=1e6, vn_delay=0.01):
        self.clock = clock
        self.lups = lups
        self.vn_delay = vn_delay
        self.resident = 0
        self.max_resident = 0
        self.launched = []

    def footprint(self, req):
        return 72 * req.spec.nx * req.spec.ny

    def admit(self, req):
        sp = req.spec
        rho, ux, uy = sp.fields()
        self.resident += 1
        self.max_resident = max(self.max_resident, self.resident)
        return {"f": oracle.feq_field(rho, ux, uy), "spec": sp}

    def launch(self, states, steps, tick, finishing):
        work = 0
        for st, n in zip(states, steps):
            sp = st["spec"]
            st["f"] = oracle.step(st["f"], n, s=sp.s, chi=sp.chi_2d(), qref=sp.qref,
                                  variant=sp.variant)
            work += n * sp.nx * sp.ny
        self.clock.t += work / self.lups
        self.launched.append(([id(s) for s in states], list(steps)))
        return {"finishing": list(finishing)}

    def done(self, ticket):
        return True

    def wait(self, ticket):
        pass

    def results(self, ticket):
        out = []
        for st in ticket["finishing"]:
            self.resident -= 1
            out.append({"diagnostics": oracle.diagnostics(st["f"], 1.0, st["spec"].u0, 0.0),
                        "f": st["f"]})
        return out

    def vn_submit(self, req):
        return {"ready": self.clock.t + self.vn_delay}

    def vn_poll(self, job):
        return {"max_abs_lambda": 1.0} if self.clock.t >= job["ready"] else None


def small_requests(count=12, rate=50.0, seed=3):
    reqs = serve.make_requests(rate, count, seed=seed, n_range=(6, 14), step_range=(3, 40),
                               nk_range=(4, 8))
    return reqs


def test_every_request_served_and_results_match_alone():
    clock = VirtualClock()
    ex = FakeExecutor(clock)
    reqs = small_requests()
    srv = serve.Server(ex, budget_bytes=1 << 30, tick=8, clock=clock, sleep=clock.sleep)
    st = srv.run(reqs)
    assert all(r.t_done is not None and r.error is None for r in reqs)
    for r in reqs:
        assert r.t_done >= r.arrival
        if r.kind == "domain":
            sp = r.spec
            rho, ux, uy = sp.fields()
            alone = oracle.step(oracle.feq_field(rho, ux, uy), r.steps, s=sp.s, chi=sp.chi_2d(),
                                qref=sp.qref, variant=sp.variant)
            np.testing.assert_array_equal(r.result["f"], alone)
    s = st.summary(reqs)
    assert s["p50_ms"] <= s["p99_ms"]
    assert st.ticks > 0
    # a finished domain takes no part in later ticks, and every domain takes
    # exactly its requested steps
    taken = {}
    for ids, steps in ex.launched:
        for i, n in zip(ids, steps):
            assert n > 0
            taken[i] = taken.get(i, 0) + n
    assert sorted(taken.values()) == sorted(r.steps for r in reqs if r.kind == "domain")


def test_pipelined_ticks_overlap_host_and_device():
    """With two ticks in flight the server enqueues the next tick before it
    waits for the previous one: an executor whose ticks complete only when
    waited for sees a second launch before the first wait."""
    clock = VirtualClock()

    class Lazy(FakeExecutor):
        def __init__(self, clock):
            super().__init__(clock)
            self.log = []

        def launch(self, states, steps, tick, finishing):
            self.log.append("launch")
            return super().launch(states, steps, tick, finishing)

        def done(self, ticket):
            return False

        def wait(self, ticket):
            self.log.append("wait")

    ex = Lazy(clock)
    reqs = [r for r in small_requests(10, rate=1000.0, seed=5) if r.kind == "domain"]
    srv = serve.Server(ex, budget_bytes=1 << 30, tick=4, clock=clock, sleep=clock.sleep)
    srv.run(reqs)
    assert all(r.t_done is not None for r in reqs)
    assert ex.log[:2] == ["launch", "launch"]


def test_admission_respects_budget_and_fifo():
    clock = VirtualClock()
    ex = FakeExecutor(clock, lups=2e5)
    reqs = [r for r in small_requests(30, rate=1000.0, seed=7) if r.kind == "domain"]
    budget = max(72 * r.spec.nx * r.spec.ny for r in reqs) * 2
    order = []
    srv = serve.Server(ex, budget_bytes=budget, tick=4, clock=clock, sleep=clock.sleep)
    st = srv.run(reqs, order_of_admission=order)
    assert st.peak_bytes <= budget
    assert st.admission_stalls > 0  # backpressure happened
    assert order == sorted(order)   # first come, first served
    assert all(r.t_done is not None for r in reqs)


def test_slot_limit_and_rejection():
    clock = VirtualClock()
    ex = FakeExecutor(clock)
    reqs = [r for r in small_requests(20, rate=1000.0, seed=11) if r.kind == "domain"]
    big = max(reqs, key=lambda r: r.spec.nx * r.spec.ny)
    budget = 72 * big.spec.nx * big.spec.ny - 1  # the largest request can never fit
    srv = serve.Server(ex, budget_bytes=budget, max_slots=2, tick=4, clock=clock, sleep=clock.sleep)
    st = srv.run(reqs)
    assert ex.max_resident <= 2
    assert st.rejected >= 1 and big.error is not None
    assert all(r.t_done is not None for r in reqs)


def test_arrivals_are_open_loop_poisson():
    reqs = serve.make_requests(200.0, 4000, seed=1)
    gaps = np.diff([0.0] + [r.arrival for r in reqs])
    assert abs(gaps.mean() - 1 / 200.0) < 0.1 / 200.0
    kinds = [r.kind for r in reqs]
    assert 0.45 < kinds.count("domain") / len(kinds) < 0.55
    ns = np.array([r.spec.nx for r in reqs if r.kind == "domain"])
    assert ns.min() >= 64 and ns.max() <= 1024
    # log-uniform: the median sits near the geometric mean of the range
    assert 180 < np.median(ns) < 330
