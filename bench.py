#!/usr/bin/env python3
"""Benchmark of the fused D2Q9 MRT + absorbing-layer step on one MI355X.

Workload: a single 4096 x 4096 periodic lattice, FP32 deviation storage
(base f^eq(rho0, u0)), uniform mean flow at Mach 0.2 in x, a seeded sum of
32 Gaussian density pulses (amplitudes U[1e-4, 1e-3], half-widths U[4, 16]),
a 64-cell quadratic sponge ramp to chi_max = 0.2 on all sides (separable
form), S = (0, 0, 0, 1.9 x 6), n = m = 1/2. The headline variant is Type II;
Types I and III are timed the same way and reported beside it.

A step is one launch of the fused pull-stream + collide kernel over the whole
lattice; diagnostics (FP64 reductions) run every 100 steps inside the timed
region. Inputs are resident in HBM before timing starts.

Prints one JSON line.
"""
import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBPS = 8000.0
# FP32 (and FP64) vector FMA issue of MI355X without packed FP32 math, which
# this library does not use: 256 CUs x 4 SIMDs x 16 lanes x 2 flop x 2.4 GHz
PEAK_VALU_TFLOPS = 78.6
# Arithmetic of one cell update (FMA = 2 flop) as the collision executes it
# with the default parameters (conserved rates 0, n = m), counted on the
# compiled loop of the four-step kernel (built as the library is, without
# automatic contraction): M g, the shifted conserved moments,
# the equilibrium deviations, relaxation and damping folded with D^-1, and
# M^T; the one reciprocal of rho per cell and of 1 + n chi per row count once.
FLOPS_PER_UPDATE = {"none": 120, "I": 150, "II": 148, "III": 142, "visc": 132}
METRIC = "D2Q9 MRT+sponge MLUPS & %HBM peak; batched-served vs plain MLUPS, p99 latency"
CSRC = os.path.join(ROOT, "paper_1203_6350_amd", "csrc")
# sources of the two step-kernel families: the K-step strip kernel and the
# one-step kernels
KERNEL_SOURCES = {
    "strip": [os.path.join(CSRC, f) for f in ("lbm_strip.h", "lbm_launch.h", "lbm_device.h")],
    "one_step": [os.path.join(CSRC, f) for f in ("lbm_kernels.hip", "lbm_launch.h", "lbm_device.h")],
}
PMC_SUMMARY = os.path.join(ROOT, "profiles", "step_f32_typeII_4096_pmc.txt")
KERNEL_SOURCES["d3q15"] = [os.path.join(CSRC, f) for f in ("lbm3_kernels.hip", "lbm3_device.h",
                                                            "lbm_device.h")]
PMC_SUMMARY3 = os.path.join(ROOT, "profiles", "step3_d3q15_typeII_256cube.txt")
KERNEL_SOURCES["vn"] = [os.path.join(CSRC, "lbm_vn.hip")]


def kernel_hash(family):
    h = hashlib.sha256()
    for p in KERNEL_SOURCES[family]:
        with open(p, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


VALU_SUMMARY = os.path.join(ROOT, "profiles", "step_f32_typeII_4096_valu.txt")


def valu_issue(tuning):
    """VALU issue-busy fraction and lane-instructions per cell update of the
    four-step kernel from the committed SQ-counter summary (one section per
    launch shape), or None when the strip sources changed since or the shape
    was not profiled."""
    if not os.path.exists(VALU_SUMMARY) or tuning.get("kernel") != 4:
        return None
    txt = open(VALU_SUMMARY).read()
    m = re.search(r"strip_kernel_sources_sha256_16:\s*(\w+)", txt)
    if not m or m.group(1) != kernel_hash("strip"):
        return None
    want = (tuning["kernel"], tuning["block"], tuning.get("rows", 0))
    for sec in txt.split("\n== ")[1:]:
        t = re.search(r"--tuning (\d+),(\d+),(\d+)", sec)
        busy = re.search(r"VALU issue busy:.*= ([0-9.]+)\s*$", sec, re.M)
        lane = re.search(r"-> ([0-9.]+) lane-instructions per cell update", sec)
        if t and busy and lane and tuple(int(x) for x in t.groups()) == want:
            return {"valu_issue_busy": float(busy.group(1)),
                    "lane_instructions_per_update": float(lane.group(1))}
    return None


def counter_traffic(tuning):
    """HBM bytes per launch of the given launch shape from the committed
    rocprofv3 --pmc summary, or None when the kernel source changed since the
    counters were taken or that shape was not profiled."""
    if not os.path.exists(PMC_SUMMARY):
        return None
    txt = open(PMC_SUMMARY).read()
    family = "strip" if tuning["kernel"] >= 2 else "one_step"
    m = re.search(r"%s_kernel_sources_sha256_16:\s*(\w+)" % family, txt)
    key = "%d,%d,%d" % (tuning["kernel"], tuning["block"], tuning.get("rows", 0) if tuning["kernel"] >= 2 else 0)
    b = re.search(r"scaled_bytes_per_launch\[" + re.escape(key) + r"\]:\s*([0-9.eE+]+)", txt)
    if not m or not b or m.group(1) != kernel_hash(family):
        return None
    return float(b.group(1))


def counter_traffic3(storage):
    """HBM bytes per launch of the D3Q15 step kernel (256^3 workload) from
    the committed --pmc summary, or None if the kernel sources changed."""
    if not os.path.exists(PMC_SUMMARY3):
        return None
    txt = open(PMC_SUMMARY3).read()
    m = re.search(r"d3q15_kernel_sources_sha256_16:\s*(\w+)", txt)
    b = re.search(r"scaled_bytes_per_launch\[%s\]:\s*([0-9.eE+]+)" % storage, txt)
    if not m or not b or m.group(1) != kernel_hash("d3q15"):
        return None
    return float(b.group(1))


# Untimed steps before the autotuner runs: it times the candidates on the
# lattice's current state, and a freshly initialised workload is 98% exact
# zero deviations, on which the shapes rank differently from a developed
# field (on 4096^2 FP32 it then picked 32-row chunks, 2% slower than fitted
# ones once the field has developed).
DEVELOP_STEPS = 1000


def time_variant(lbm, wl, torch, spec, fields, steps, warmup, diag_every=100, fixed=None):
    rho, ux, uy = fields
    stream = torch.cuda.current_stream()
    lat = lbm.Lattice(spec.nx, spec.ny, rho=rho, ux=ux, uy=uy, storage=spec.storage,
                      variant=spec.variant, s=spec.s, ux_base=spec.base_state[1],
                      f16_scale=5e-4, stream=stream)
    cx, cy = spec.chi_1d()
    lat.set_sponge_separable(cx, cy, "max", spec.qref)
    if fixed is None:
        lat.step(DEVELOP_STEPS)
        tuning, tune_ms = lat.autotune(reps=10)
    else:
        lat.set_tuning(**fixed)
        tuning = lat.tuning()
    per = tuning["kernel"] if tuning["kernel"] >= 2 else 1  # time steps per launch
    launches, rest = divmod(steps, per)
    diag = torch.empty(7, dtype=torch.float64, device="cuda")
    lat.step(warmup)
    torch.cuda.synchronize()
    # launches run in groups between two diagnostics; a pair of events
    # brackets each group, so the mean launch duration includes the gaps
    # between launches but neither the diagnostics nor an event per launch
    # (one after every launch cost about 1% of the rate)
    group = max(1, diag_every // per) if diag_every else max(1, launches)
    marks = []
    t0 = time.perf_counter()
    done_launches = 0
    while done_launches < launches:
        n = min(group, launches - done_launches)
        ea, eb = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ea.record(stream)
        lat.step(n * per)  # n launches of `per` steps
        eb.record(stream)
        marks.append((ea, eb, n))
        done_launches += n
        if diag_every and n == group:
            lbm.lbm_diagnostics_dev(lat.h, diag)
    if rest:
        lat.step(rest)  # the remaining steps as one shorter launch, so exactly `steps` run
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    group_ms = sum(ea.elapsed_time(eb) for ea, eb, _ in marks)
    d = diag.cpu().numpy()
    lat.close()
    wall = t1 - t0
    cells = spec.nx * spec.ny
    done = launches * per + rest
    return dict(wall_s=wall, ms_per_step=1e3 * wall / done, steps=done,
                mlups=cells * done / wall / 1e6, steps_per_launch=per,
                kernel_ms=group_ms / launches if launches else float("nan"),
                diag=[float(x) for x in d], tuning=tuning)


def copy_bandwidth(lbm, torch, nbytes=2 << 30, reps=20):
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    s = torch.cuda.current_stream()
    for _ in range(3):
        lbm.lbm_device_copy(b, a, nbytes, s)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        lbm.lbm_device_copy(b, a, nbytes, s)
    e1.record(s)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes / (ms * 1e-3) / 1e9


def make_domain(lbm, spec, stream):
    rho, ux, uy = spec.fields()
    lat = lbm.Lattice(spec.nx, spec.ny, rho=rho, ux=ux, uy=uy, storage=spec.storage,
                      variant=spec.variant, s=spec.s, ux_base=spec.base_state[1], stream=stream)
    cx, cy = spec.chi_1d()
    lat.set_sponge_separable(cx, cy, "max", spec.qref)
    return lat


def batched_leg(lbm, wl, torch, steps=1000, vn_sets=64, vn_nk=256):
    """256 uneven domains: the batch (persistent launches captured in HIP
    graphs) against plain per-domain launches, three ways: one eager
    one-step launch per domain per step; each domain in its own autotuned
    shape, one after another; the same spread over eight streams. Finite
    members are compared bit for bit with the batch. Plus the Von Neumann
    sweep."""
    specs = wl.batch_c4()
    cells = sum(sp.nx * sp.ny for sp in specs)
    s = torch.cuda.current_stream()
    # plain: one launch per domain per step, all queued on one stream
    plain = [make_domain(lbm, sp, s) for sp in specs]
    for lat in plain:
        lat.step(2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for lat in plain:
        lat.step(steps)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    # plain, each domain in its own autotuned launch shape (K steps per
    # launch where that is fastest), one after another on one stream, and
    # spread round-robin over eight streams
    tuned_t = {}
    for nstreams in (1, 8):
        streams = [s] if nstreams == 1 else [torch.cuda.Stream() for _ in range(nstreams)]
        tuned = [make_domain(lbm, sp, streams[i % nstreams]) for i, sp in enumerate(specs)]
        for lat in tuned:
            lat.autotune(reps=3)
            lat.step(2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for lat in tuned:
            lat.step(steps)
        torch.cuda.synchronize()
        tuned_t[nstreams] = time.perf_counter() - t0
        if nstreams == 8:
            tuned_8 = tuned
        else:
            for lat in tuned:
                lat.close()
    # batched: the same domains, same number of steps
    lats = [make_domain(lbm, sp, s) for sp in specs]
    b = lbm.Batch(lats)
    b.step(2)
    b.sync()
    t0 = time.perf_counter()
    b.step(steps)
    b.sync()
    t_batch = time.perf_counter() - t0
    # Type I members with s + chi > 2 blow up by design (non-finite state);
    # the finite members are compared bit for bit
    same, unstable = True, 0
    for p_, q_ in zip(plain, lats):
        dp_ = p_.diagnostics()
        if dp_[6] > 0:
            unstable += 1
            continue
        same = same and bool((p_.save_state() == q_.save_state()).all())
    for p_, q_ in zip(tuned_8, lats):
        if p_.diagnostics()[6] == 0:
            same = same and bool((p_.save_state() == q_.save_state()).all())
    b.close()
    for lat in plain + lats + tuned_8:
        lat.close()
    out = {"domains": len(specs), "cells": cells, "steps": steps,
           "batched_mlups": cells * steps / t_batch / 1e6,
           "plain_mlups": cells * steps / t_plain / 1e6,
           "speedup": t_plain / t_batch,
           "plain_tuned_mlups": cells * steps / tuned_t[1] / 1e6,
           "speedup_vs_tuned": tuned_t[1] / t_batch,
           "plain_tuned_8streams_mlups": cells * steps / tuned_t[8] / 1e6,
           "speedup_vs_tuned_8streams": tuned_t[8] / t_batch,
           "bitwise_equal_finite_members": same,
           "unstable_members": unstable}
    out.update(vn_sweep_leg(lbm, wl, torch, vn_sets, vn_nk))
    return out


def vn_sweep_leg(lbm, wl, torch, vn_sets=64, vn_nk=256, reps=3):
    """Von Neumann sweep: vn_sets parameter sets on a vn_nk^2 wavenumber grid
    in one launch; the best of `reps` timed launches (after a warm-up)."""
    kx, ky = wl.vn_grid(vn_nk)
    dkx = torch.from_numpy(kx).cuda()
    dky = torch.from_numpy(ky).cuda()
    params = wl.vn_param_sets(vn_sets)
    eig = torch.empty((vn_sets, kx.size, 9, 2), dtype=torch.float64, device="cuda")
    lbm.vn_amplification_dev(params[:2], dkx, dky, eig[:2])
    torch.cuda.synchronize()
    best = None
    for _ in range(reps):
        t0 = time.perf_counter()
        lbm.vn_amplification_dev(params, dkx, dky, eig)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        best = dt if best is None else min(best, dt)
    finite = bool(torch.isfinite(eig).all().item())
    return {"vn_sets": vn_sets, "vn_kpoints": int(kx.size) * vn_sets,
            "vn_kpoints_per_s": kx.size * vn_sets / best, "vn_seconds": best,
            "vn_all_finite": finite}


def serving_leg(torch, rates=(50, 100, 200, 500), count=2000, warmup=200, budget_gb=200):
    """Open-loop Poisson arrivals of domain and Von Neumann requests; latency
    from arrival to result on the host."""
    from paper_1203_6350_amd import serve
    out = {}
    for rate in rates:
        print("bench: serving at %d req/s, %d requests" % (rate, count), file=sys.stderr, flush=True)
        reqs = serve.make_requests(float(rate), count, seed=rate)
        ex = serve.GpuExecutor()
        srv = serve.Server(ex, budget_bytes=int(budget_gb * (1 << 30)))
        st = srv.run(reqs)
        ex.close()
        summ = st.summary(reqs, warmup=warmup)
        summ["offered_mlups"] = sum(r.steps * r.spec.nx * r.spec.ny for r in reqs
                                    if r.kind == "domain") / reqs[-1].arrival / 1e6
        out[str(rate)] = summ
        torch.cuda.empty_cache()
    return out


def characteristics(rho, ux, rho0, u0, lo, hi):
    """Right- and left-going acoustic parts p'_+- = (p' +- rho0 c_s u'_x)/2 of a
    y-uniform state on the physical x-range [lo, hi)."""
    cs = 1.0 / math.sqrt(3.0)
    p = (rho[lo:hi] - rho0) / 3.0
    u = ux[lo:hi] - u0
    return 0.5 * (p + rho0 * cs * u), 0.5 * (p - rho0 * cs * u)


PRECISION_CHIS = (0.05, 0.2, 0.5)


def precision_leg(lbm, wl, n=2048, steps=4000, chis=PRECISION_CHIS, width=48, reference=None):
    """Plane packet (amplitude 1e-4, wavelength 64, 8 wavelengths) in Mach-0.1
    flow entering a 48-cell x-sponge, Type II. Each storage mode and base on
    the n x n lattice against a reference of the n x 1 row (a y-uniform state
    with an x-only sponge evolves row by row like the one-row lattice): the
    FP64 oracle's row (``reference``: chi_max -> (rho, u_x) after `steps`,
    computed and timed by the CPU-baseline leg), or, when that leg is
    skipped, the library's FP64 run of the row. Errors of p' relative to the
    initial wave and to the current reference field; R and T (characteristic
    split over the physical range, normalised by the incident wave)."""
    import numpy as np
    u0 = 0.1 * wl.CS
    rho, ux, uy = wl.plane_packet(n, n, amp=1e-4, wavelength=64.0, n_wavelengths=8,
                                  centre=n / 2, u0=u0)
    cx = wl.quadratic_ramp_1d(n, width, 1.0)
    lo, hi = width, n - width
    p0p, _ = characteristics(rho[0], ux[0], 1.0, u0, lo, hi)
    norm0 = float(np.sqrt((p0p ** 2).sum()))
    out = {"reference": "oracle" if reference else "library FP64 one-row lattice"}
    for chi_max in chis:
        q = (1.0, u0, 0.0)
        if reference:
            rr, ur = reference[chi_max]
        else:
            one = lbm.Lattice(n, 1, rho=rho[:1], ux=ux[:1], uy=uy[:1], storage="f64",
                              variant="II", ux_base=u0)
            one.set_sponge_separable(chi_max * cx, None, "max", q)
            one.step(steps)
            r1, u1, _ = one.moments()
            one.close()
            rr, ur = r1[0], u1[0]
        rp, rm = characteristics(rr, ur, 1.0, u0, lo, hi)
        R_ref = float(np.sqrt((rm ** 2).sum())) / norm0
        T_ref = float(np.sqrt((rp ** 2).sum())) / norm0
        row = {"reference_R": R_ref, "reference_T": T_ref}
        for storage in ("f64", "f32", "f16"):
            for base in ("rest", "ref"):
                lat = lbm.Lattice(n, n, rho=rho, ux=ux, uy=uy, storage=storage, variant="II",
                                  ux_base=u0 if base == "ref" else 0.0, f16_scale=1e-4)
                lat.set_sponge_separable(chi_max * cx, None, "max", q)
                lat.step(steps)
                g_rho, g_ux, _ = lat.moments()
                lat.close()
                pr = g_rho - 1.0
                pref = rr - 1.0
                p_init = rho[0] - 1.0
                sq = ((pr - pref[None, :]) ** 2).sum() / n
                gp, gm = characteristics(g_rho[0], g_ux[0], 1.0, u0, lo, hi)
                R = float(np.sqrt((gm ** 2).sum())) / norm0
                T = float(np.sqrt((gp ** 2).sum())) / norm0
                row["%s_%s" % (storage, base)] = {
                    "pprime_rel_l2": float(np.sqrt(sq / (pref ** 2).sum())),
                    "pprime_err_over_initial": float(np.sqrt(sq / (p_init ** 2).sum())),
                    "rows_identical": bool((g_rho == g_rho[:1]).all()),
                    "R": R, "T": T, "R_abs_err": abs(R - R_ref), "R_rel_err": abs(R - R_ref) / R_ref,
                    "T_abs_err": abs(T - T_ref), "T_rel_err": abs(T - T_ref) / T_ref}
        out["chi_max=%g" % chi_max] = row
    return out


def paper_pulse_leg(lbm, wl, steps=1200, every=20):
    """The comparison of Section 4.1: E_L2(t) for no layer, the viscosity
    ramp and the Type II layer (thickness 2b, 3b, 4b; mean flow 0 and 0.1),
    and the log-log decay slope of E_L2 after the pulse enters the layer."""
    import numpy as np
    out = {}
    for u0 in (0.0, 0.1):
        for m in (2, 3, 4):
            for strategy in ("none", "visc", "II"):
                if strategy == "none" and m != 4:
                    continue
                spec, px, py = wl.paper_pulse(strategy, thickness_b=m, u0=u0)
                rho, ux, uy = spec.fields()
                lat = lbm.Lattice(spec.nx, spec.ny, rho=rho, ux=ux, uy=uy, storage="f64",
                                  variant=spec.variant, s=spec.s, ux_base=u0)
                lat.set_sponge_separable(px, py, "max", spec.qref)
                ts, es = [], []
                for k in range(steps // every):
                    lat.step(every)
                    d = lat.diagnostics()
                    ts.append((k + 1) * every)
                    es.append(math.sqrt(d[3] / (spec.nx * spec.ny)))
                lat.close()
                ts, es = np.array(ts, float), np.array(es)
                # the pulse front reaches the layer at (n/2 - W - 2b)/c_s steps
                t_in = (spec.nx / 2 - spec.width - 20) / wl.CS
                sel = (ts > 1.5 * t_in) & (es > 0)
                slope = float(np.polyfit(np.log(ts[sel]), np.log(es[sel]), 1)[0]) if sel.sum() > 3 else None
                out["u0=%g,%db,%s" % (u0, m, strategy)] = {
                    "E_L2_final": float(es[-1]), "E_L2_at": {int(t): float(e) for t, e in
                                                             zip(ts[4::10], es[4::10])},
                    "loglog_slope": slope}
    return out


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(spec, fields, steps, wl=None):
    """The FP64 oracle, as it stands, on bounded samples of the workloads: the
    headline (all host threads, and one thread for two steps), the 128^2
    parity case, the 2048 x 1 row of the precision study for each chi_max
    (whose final rows the precision leg then takes as its reference), the
    smaller batched domains and the Von Neumann eigenvalues (LAPACK) of a
    seeded sample of wavenumbers. Returns (summary, precision reference)."""
    import numpy as np
    import oracle
    import oracle.vn as ovn
    rho, ux, uy = fields
    threads = len(os.sched_getaffinity(0))

    def run(f0, n, nthreads, **kw):
        t0 = time.perf_counter()
        oracle.step(f0, n, nthreads=nthreads, **kw)
        return time.perf_counter() - t0

    f0 = oracle.feq_field(rho, ux, uy)
    kw = dict(s=spec.s, chi=spec.chi_2d(), qref=spec.qref, variant=spec.variant)
    dt = run(f0, steps, threads, **kw)
    dt1 = run(f0, 2, 1, **kw)
    del f0
    prec_ref = {}
    out = {"value": spec.nx * spec.ny * steps / dt / 1e6, "unit": "MLUPS",
           "cores": threads, "kind": "oracle",
           "sample": "%dx%d workload, %d steps, Type %s, FP64, %.1f s" %
                     (spec.nx, spec.ny, steps, spec.variant, dt),
           "single_thread_mlups": spec.nx * spec.ny * 2 / dt1 / 1e6,
           "host": {"cpu_model": _cpu_model(), "nproc": os.cpu_count(), "threads_used": threads,
                    "OMP_NUM_THREADS": os.environ.get("OMP_NUM_THREADS")}}
    if wl is not None:
        c1 = wl.pulse_c1("II")
        r1, u1, v1 = c1.fields()
        t = run(oracle.feq_field(r1, u1, v1), c1.steps, threads, s=c1.s, chi=c1.chi_2d(),
                qref=c1.qref, variant="II")
        out["c1_128sq_fp64_1000_steps"] = {"mlups": c1.nx * c1.ny * c1.steps / t / 1e6, "s": t}
        n3, steps3 = 2048, 4000
        u0 = 0.1 * wl.CS
        r3, u3, v3 = wl.plane_packet(n3, 1, amp=1e-4, centre=n3 / 2, u0=u0)
        f3 = oracle.feq_field(r3, u3, v3)
        t3 = {}
        for chi_max in PRECISION_CHIS:
            cx = wl.quadratic_ramp_1d(n3, 48, chi_max)
            t0 = time.perf_counter()
            fT = oracle.step(f3, steps3, nthreads=1, chi=cx[None, :], qref=(1.0, u0, 0.0),
                             variant="II")
            t3["chi_max=%g" % chi_max] = time.perf_counter() - t0
            rT, uT, _ = oracle.moments(fT)
            prec_ref[chi_max] = (rT[0], uT[0])
        t = sum(t3.values())
        out["c3_2048x1_row_4000_steps"] = {"mlups": len(t3) * n3 * steps3 / t / 1e6, "s": t,
                                           "runs": t3}
        small = [d for d in wl.batch_c4() if d.nx <= 256]
        cells, t = 0, 0.0
        for d in small:
            rr, uu, vv = d.fields()
            t += run(oracle.feq_field(rr, uu, vv), 20, threads, s=d.s, chi=d.chi_2d(), qref=d.qref,
                     variant=d.variant)
            cells += d.nx * d.ny
        out["c4_domains_n_le_256_20_steps"] = {"domains": len(small), "mlups": cells * 20 / t / 1e6,
                                               "s": t}
        # Von Neumann: LAPACK eigenvalues of G(k) (numpy) on a seeded sample of
        # 1024 wavenumbers of the 256^2 grid for each of the 64 parameter sets
        kx, ky = wl.vn_grid(256)
        pick = np.random.default_rng(12036353).choice(kx.size, 1024, replace=False)
        sets = wl.vn_param_sets(64)
        t0 = time.perf_counter()
        for p in sets:
            ovn.eigenvalues(p["s"], p["chi"], p["qref"], kx[pick], ky[pick], p.get("n", 0.5),
                            p.get("m", 0.5), p["variant"])
        tv = time.perf_counter() - t0
        out["vn_lapack"] = {"kpoints": len(sets) * pick.size, "s": tv,
                            "kpoints_per_s": len(sets) * pick.size / tv, "threads": 1,
                            "sample": "64 parameter sets x 1024 seeded wavenumbers of the 256^2 grid"}
    return out, prec_ref


def qref_leg(lbm, wl, torch, n=4096, steps=400, warmup=20, alpha=1e-3):
    """The headline workload with a per-cell reference state, fixed in time
    or following the flow as a running mean of rate alpha, each in the
    one-cell kernel and in the autotuned strip kernels (where the field rows
    travel with the sponge input). Bytes per cell per launch (FP32): 72 + 12
    (fixed) or 72 + 24 (running mean: read, and written to the second
    buffer); one launch is K steps in the strips."""
    sp = wl.large_c2(variant="II", storage="f32", n=n)
    rho, ux, uy = sp.fields()
    stream = torch.cuda.current_stream()
    lat = lbm.Lattice(sp.nx, sp.ny, rho=rho, ux=ux, uy=uy, storage="f32", variant="II", s=sp.s,
                      ux_base=sp.base_state[1], stream=stream)
    cx, cy = sp.chi_1d()
    lat.set_sponge_separable(cx, cy, "max", sp.qref)
    lat.set_qref_field(rho, ux, uy)
    lat.step(DEVELOP_STEPS)  # the autotuner below times a developed field
    out = {}
    for name, a, tune in (("alpha=0,one_cell", 0.0, "one"), ("alpha=0", 0.0, "auto"),
                          ("alpha=%g,one_cell" % alpha, alpha, "one"),
                          ("alpha=%g" % alpha, alpha, "auto")):
        lat.set_qref_average(a)
        if tune == "one":
            lat.set_tuning(kernel=0, block=256)
        else:
            lat.autotune(reps=5)
        t = lat.tuning()
        per = t["kernel"] if t["kernel"] >= 2 else 1
        lat.step(warmup)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        lat.step(steps)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        b = 72 + (24 if a else 12)
        launch_gbps = b * sp.nx * sp.ny / (ms * per * 1e-3) / 1e9
        out[name] = {"mlups": sp.nx * sp.ny / ms / 1e3, "ms_per_step": ms, "tuning": t,
                     "steps_per_launch": per, "bytes_per_cell_per_launch": b,
                     "hbm_gbps": launch_gbps, "hbm_frac": launch_gbps / PEAK_HBM_GBPS}
    d = lat.diagnostics()
    lat.close()
    out["nonfinite_cells"] = float(d[6])
    return out


def _line_source_run(lbm, wl, cfg):
    nx, ny = cfg["nx"], cfg["ny"]
    u0 = cfg["u0"]
    lat = lbm.Lattice(nx, ny, rho=np.ones((ny, nx)), ux=np.full((ny, nx), u0),
                      uy=np.zeros((ny, nx)), storage="f64", variant=cfg["variant"], s=cfg["s"],
                      ux_base=u0)
    lat.set_sponge_separable(cfg["profile"], None, "max", (1.0, u0, 0.0))
    lat.set_line_source(cfg["source"], True)
    t0 = time.perf_counter()
    lat.step(cfg["t_sample"])
    rho, _, _ = lat.moments()
    dt = time.perf_counter() - t0
    lat.close()
    return rho - 1.0, dt


def line_source_leg(lbm, wl):
    """Section 4.2: the acoustic line source through an absorbing layer at the
    outflow, sampled at T_o + 10 T_p. rho' along the channel against a
    reference channel three times longer without a layer (no reflection can
    reach its first part by then): relative L2 error over the physical region,
    per strategy, with and without mean flow, and the layer thickness that
    Type II needs."""
    out = {}
    for u0 in (0.0, 0.1):
        ref_cfg = wl.paper_line_source("none", thickness=0.0, u0=u0, length_factor=3)
        ref, _ = _line_source_run(lbm, wl, ref_cfg)
        for strat in ("none", "visc", "II"):
            cfg = wl.paper_line_source(strat, u0=u0)
            rp, dt = _line_source_run(lbm, wl, cfg)
            phys = slice(1, cfg["nx"] - cfg["layer_cells"])
            a, b = rp[0, phys], ref[0, phys]
            out["u0=%g,%s" % (u0, strat)] = {
                "rel_l2_error": float(np.sqrt(((a - b) ** 2).sum() / (b ** 2).sum())),
                "rows_identical": bool((rp == rp[:1]).all()), "steps": cfg["t_sample"],
                "mlups": cfg["nx"] * cfg["ny"] * cfg["t_sample"] / dt / 1e6}
    ref_cfg = wl.paper_line_source("none", thickness=0.0, length_factor=3)
    ref, _ = _line_source_run(lbm, wl, ref_cfg)
    thick = {}
    for d in (0.1, 0.2, 0.3, 0.5, 0.8):
        cfg = wl.paper_line_source("II", thickness=d)
        rp, _ = _line_source_run(lbm, wl, cfg)
        phys = slice(1, cfg["nx"] - int(round(0.8 * 200)))   # the same region for every d
        a, b = rp[0, phys], ref[0, phys]
        thick["%g" % d] = float(np.sqrt(((a - b) ** 2).sum() / (b ** 2).sum()))
    out["typeII_thickness_rel_l2"] = thick
    out["wavelength_cells"] = wl.paper_line_source()["wavelength_cells"]
    return out


def storages_leg(lbm, wl, torch, n, steps, warmup):
    """The headline workload in FP64 and FP16 storage (autotuned launch shape)."""
    out = {}
    for st in ("f64", "f16"):
        sp = wl.large_c2(variant="II", storage=st, n=n)
        r = time_variant(lbm, wl, torch, sp, sp.fields(), steps, warmup)
        eb = {"f64": 8, "f16": 2}[st]
        cells = sp.nx * sp.ny
        per = r["steps_per_launch"]
        out[st] = {"mlups": r["mlups"], "tuning": r["tuning"], "steps_per_launch": per,
                   "kernel_ms": r["kernel_ms"],
                   "hbm_gbps": 18 * eb * cells / (r["kernel_ms"] * 1e-3) / 1e9,
                   "alu_tflops": FLOPS_PER_UPDATE["II"] * cells * per / (r["kernel_ms"] * 1e-3) / 1e12,
                   "single_step_equivalent_gbps": 18 * eb * r["mlups"] / 1e3,
                   "nonfinite_cells": r["diag"][6]}
    return out


def d3q15_leg(lbm, wl, torch, n=256, steps=200, warmup=10):
    """The three-dimensional D3Q15 scheme (Appendix A.2) on the n^3 box with
    mean flow, 16 pulses and a six-face separable ramp, Type II, per storage:
    one cell per thread, every stored element read and written once per step
    (30 elements per cell update)."""
    spec = wl.cube_d3q15(n=n)
    F = spec["fields"]()
    prof = spec["profile"]
    stream = torch.cuda.current_stream()
    out = {"workload": "D3Q15 %d^3, Type II, separable ramp 32 cells, Mach 0.17" % n}
    for st in ("f32", "f64", "f16"):
        lat = lbm.Lattice3(n, n, n, rho=F[0], ux=F[1], uy=F[2], uz=F[3], storage=st,
                           variant="II", ux_base=spec["u0"], f16_scale=1e-3, stream=stream)
        lat.set_sponge_separable(prof, prof, prof, "max", spec["qref"])
        lat.step(warmup)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        lat.step(steps)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        rho = lat.moments()[0]
        lat.close()
        b = 30 * {"f64": 8, "f32": 4, "f16": 2}[st]
        cells = n ** 3
        out[st] = {"mlups": cells / ms / 1e3, "ms_per_step": ms, "bytes_per_cell": b,
                   "hbm_gbps": b * cells / (ms * 1e-3) / 1e9,
                   "hbm_frac": b * cells / (ms * 1e-3) / 1e9 / PEAK_HBM_GBPS,
                   "traffic": counter_traffic3(st) if n == 256 else None,
                   "max_abs_rho_dev": float(np.abs(rho - 1.0).max()),
                   "finite": bool(np.isfinite(rho).all())}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--storage", default="f32", choices=["f32", "f64", "f16"])
    ap.add_argument("--variants", default="II,I,III")
    ap.add_argument("--cpu-steps", type=int, default=80)
    ap.add_argument("--no-storages", action="store_true")
    ap.add_argument("--no-qref", action="store_true")
    ap.add_argument("--no-line-source", action="store_true")
    ap.add_argument("--no-d3q15", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-copy", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--no-precision", action="store_true")
    ap.add_argument("--no-pulse", action="store_true")
    ap.add_argument("--vn-only", action="store_true",
                    help="run only the Von Neumann sweep (64 sets x 256^2 wavenumbers; for "
                         "profiling runs) and print its figures")
    ap.add_argument("--tuning", default=None,
                    help="kernel,block,rows: fixed launch shape instead of the autotuner "
                         "(for profiling runs)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the multi-GPU form (row bands per GPU with "
              "a halo exchange) is designed but not built, so --gpus %d is not run." % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    if args.steps < 4 or args.warmup < 0:
        # the timed steps must hold at least one launch of the four-step
        # kernel, whose mean duration the roofline divides by
        print("bench.py: --steps must be at least 4 and --warmup at least 0", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1203_6350_amd import lbm, workloads as wl

    torch.cuda.set_device(0)
    lbm.load()
    if args.vn_only:
        print(json.dumps({"vn_sweep": vn_sweep_leg(lbm, wl, torch)}), flush=True)
        return
    variants = [v for v in args.variants.split(",") if v]
    head = variants[0]
    spec = wl.large_c2(variant=head, storage=args.storage, n=args.n)
    print("bench: building %dx%d inputs" % (spec.nx, spec.ny), file=sys.stderr, flush=True)
    fields = spec.fields()
    eb = {"f64": 8, "f32": 4, "f16": 2}[args.storage]
    bytes_per_cell = 18 * eb
    cells = spec.nx * spec.ny

    results = {}
    for v in variants:
        sv = wl.large_c2(variant=v, storage=args.storage, n=args.n)
        k = args.steps if v == head else max(100, args.steps // 4)
        print("bench: timing Type %s, %d steps" % (v, k), file=sys.stderr, flush=True)
        fixed = None
        if args.tuning:
            kk, bb, rr = (int(x) for x in args.tuning.split(","))
            fixed = dict(kernel=kk, block=bb, rows=rr)
        results[v] = time_variant(lbm, wl, torch, sv, fields, k, args.warmup, fixed=fixed)
    r = results[head]
    # one launch reads and writes every stored element once, whatever number
    # of time steps it advances
    per = r["steps_per_launch"]
    launch_s = r["kernel_ms"] * 1e-3
    hbm_gbps = bytes_per_cell * cells / launch_s / 1e9
    alu_tflops = FLOPS_PER_UPDATE[head] * cells * per / launch_s / 1e12
    copy_gbps = None if args.no_copy else copy_bandwidth(lbm, torch)
    traffic = (counter_traffic(r["tuning"]) if args.storage == "f32" and args.n == 4096
               and head == "II" else None)
    common = {"traffic": traffic,
              "algorithmic_bytes_per_launch": bytes_per_cell * cells,
              "algorithmic_flops_per_launch": FLOPS_PER_UPDATE[head] * cells * per,
              "steps_per_launch": per, "kernel_ms": r["kernel_ms"],
              "hbm_gbps": hbm_gbps, "hbm_frac": hbm_gbps / PEAK_HBM_GBPS,
              "alu_tflops": alu_tflops, "alu_frac": alu_tflops / PEAK_VALU_TFLOPS,
              "single_step_equivalent_gbps": bytes_per_cell * r["mlups"] / 1e3}
    if per >= 3:
        # three or more steps per launch: the vector ALUs, not HBM, bound it;
        # the SQ counters give the issue utilisation the flop rate understates
        roofline = dict({"bound": "alu", "achieved": alu_tflops, "peak": PEAK_VALU_TFLOPS,
                         "unit": "TFLOP/s", "frac": alu_tflops / PEAK_VALU_TFLOPS}, **common)
        issue = (valu_issue(r["tuning"]) if args.storage == "f32" and args.n == 4096
                 and head == "II" else None)
        if issue:
            roofline.update(issue)
    else:
        roofline = dict({"bound": "hbm", "achieved": hbm_gbps, "peak": PEAK_HBM_GBPS,
                         "unit": "GB/s", "frac": hbm_gbps / PEAK_HBM_GBPS}, **common)

    out = {
        "metric": METRIC,
        "value": r["mlups"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": r["steps"],
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f32": "f32", "f64": "f64", "f16": "f32 (f16 storage)"}[args.storage],
        "data": "synthetic",
        "config": {"workload": "D2Q9 MRT + Type %s sponge, %dx%d periodic, %s deviation storage, "
                               "Mach 0.2 mean flow, 32 seeded Gaussian pulses, 64-cell quadratic "
                               "ramp chi_max=0.2" % (head, spec.nx, spec.ny, args.storage.upper()),
                   "nx": spec.nx, "ny": spec.ny, "variant": head, "storage": args.storage,
                   "diagnostics_every": 100},
        "roofline": roofline,
        "per_variant": {v: {"mlups": x["mlups"], "kernel_ms": x["kernel_ms"],
                            "steps_per_launch": x["steps_per_launch"],
                            "achieved_gbps": bytes_per_cell * cells / (x["kernel_ms"] * 1e-3) / 1e9,
                            "nonfinite_cells": x["diag"][6], "max_dev": x["diag"][5],
                            "tuning": x["tuning"]}
                        for v, x in results.items()},
        "copy_kernel_gbps": copy_gbps,
    }
    if copy_gbps:
        out["roofline"]["hbm_frac_of_copy"] = hbm_gbps / copy_gbps
    if not args.no_storages and args.storage == "f32":
        print("bench: FP64 and FP16 storage", file=sys.stderr, flush=True)
        out["storages"] = storages_leg(lbm, wl, torch, args.n, 400, 20)
    if not args.no_qref and args.storage == "f32":
        print("bench: time-averaged reference state", file=sys.stderr, flush=True)
        out["qref_average"] = qref_leg(lbm, wl, torch, n=args.n)
    if not args.no_line_source:
        print("bench: the paper's line source", file=sys.stderr, flush=True)
        out["line_source"] = line_source_leg(lbm, wl)
    if not args.no_d3q15:
        print("bench: D3Q15 256^3", file=sys.stderr, flush=True)
        out["d3q15"] = d3q15_leg(lbm, wl, torch)
    if not args.no_batch:
        print("bench: batched 256-domain leg", file=sys.stderr, flush=True)
        out["batched"] = batched_leg(lbm, wl, torch)
    prec_ref = None
    if not args.no_cpu_baseline:
        print("bench: CPU oracle baseline, %d steps" % args.cpu_steps, file=sys.stderr, flush=True)
        out["cpu_baseline"], prec_ref = cpu_baseline(spec, fields, args.cpu_steps, wl)
    if not args.no_precision:
        print("bench: precision study 2048^2, 4000 steps", file=sys.stderr, flush=True)
        out["precision"] = precision_leg(lbm, wl, reference=prec_ref)
    if not args.no_pulse:
        print("bench: the paper's pulse comparison", file=sys.stderr, flush=True)
        out["paper_pulse"] = paper_pulse_leg(lbm, wl)
    if not args.no_serve:
        out["served"] = serving_leg(torch, count=args.serve_requests,
                                    warmup=args.serve_requests // 10)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
