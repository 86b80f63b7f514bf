"""Seeded synthetic inputs: initial macroscopic fields, sponge-strength
profiles and the parameter sets of the benchmark workloads.

This module holds no lattice Boltzmann arithmetic. It produces the inputs that
both the HIP path and the FP64 oracle consume (rho, u fields, chi profiles,
reference states, relaxation rates), and imports nothing from either side.

Shapes follow the paper's analytic set-ups:
* Gaussian density pulse rho' = eps exp(-ln2 r^2 / b^2) (eq. 3:para0), with
  an optional uniform mean flow (Section 4.1);
* a right-going plane acoustic packet for the reflection study;
* sponge profiles: the quadratic ramp chi_max * xi^2 (the second row of
  Table tab:sigma with exponent 2), the normalised A = n = 4 polynomial of
  eq. normalizedsigma, and the other rows of Table tab:sigma.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 12036350
CS = 1.0 / math.sqrt(3.0)  # lattice sound speed, c_s^2 = 1/3
S_MRT_DEFAULT = (0.0, 0.0, 0.0, 1.9, 1.9, 1.9, 1.9, 1.9, 1.9)
VARIANT_NAMES = ("none", "I", "II", "III")


def rng(config_index: int, salt: int = 0) -> np.random.Generator:
    return np.random.default_rng(SEED_BASE + config_index + 1000 * salt)


# ---------------------------------------------------------------- sponge profiles

def ramp_depth(n: int, width: int) -> np.ndarray:
    """xi(i) = max(0, (W - d(i)) / W), d(i) = min(i, n-1-i): 1 at the edge cell,
    0 from depth W inwards."""
    i = np.arange(n, dtype=np.float64)
    d = np.minimum(i, n - 1 - i)
    if width <= 0:
        return np.zeros(n)
    return np.maximum(0.0, (width - d) / width)


def quadratic_ramp_1d(n: int, width: int, chi_max: float) -> np.ndarray:
    """chi(i) = chi_max * xi(i)^2 along one axis (Table tab:sigma, row 2, n = 2)."""
    return chi_max * ramp_depth(n, width) ** 2


def orszag_profile_1d(n: int, width: int, chi_max: float) -> np.ndarray:
    """sigma = chi * sigma~ with the normalised A = n = 4 polynomial of eq.
    normalizedsigma, mirrored onto both ends of the axis. Inside a layer of
    ``width`` cells the local coordinate runs from x0 (inner edge) to L (the
    domain edge); sigma~ is zero at both ends and 1 at 4/5 of the layer."""
    xi = ramp_depth(n, width)  # 0 at the inner edge, 1 at the outer edge
    t = xi
    sig = 3125.0 * (1.0 - t) * t ** 4 / 256.0
    return chi_max * np.where(xi > 0, sig, 0.0)


def power_profile_1d(n: int, width: int, eta: float, power: int = 3) -> np.ndarray:
    """eta ((x - x0)/(L - x0))^n, Table tab:sigma row 2 (default n = 3)."""
    return eta * ramp_depth(n, width) ** power


def sponge_2d(chi_x: np.ndarray, chi_y: np.ndarray) -> np.ndarray:
    """Full 2-D field of a separable sponge, combined by max: [ny][nx]."""
    return np.maximum(chi_x[None, :], chi_y[:, None])


def clamp_width(width: int, n: int) -> int:
    """Keep a physical region: W <= floor(N/4)."""
    return int(min(width, n // 4))


# ---------------------------------------------------------------- initial fields

def gaussian_pulses(nx: int, ny: int, centres, amps, halfwidths, rho0=1.0,
                    u0=(0.0, 0.0), periodic=True):
    """rho = rho0 + sum_k eps_k exp(-ln2 r_k^2 / b_k^2), u = u0 uniform.

    Distances use the minimum image on the periodic lattice when ``periodic``.
    Returns (rho, ux, uy) as float64 [ny][nx].
    """
    x = np.arange(nx, dtype=np.float64)
    y = np.arange(ny, dtype=np.float64)
    rho = np.full((ny, nx), float(rho0))
    for (cx, cy), a, b in zip(centres, amps, halfwidths):
        dx = x - cx
        dy = y - cy
        if periodic:
            dx = dx - nx * np.round(dx / nx)
            dy = dy - ny * np.round(dy / ny)
        # exp(-ln2 (dx^2 + dy^2)/b^2) evaluated as an outer product
        ex = np.exp(-math.log(2.0) * dx * dx / (b * b))
        ey = np.exp(-math.log(2.0) * dy * dy / (b * b))
        rho += a * np.outer(ey, ex)
    ux = np.full((ny, nx), float(u0[0]))
    uy = np.full((ny, nx), float(u0[1]))
    return rho, ux, uy


def plane_packet(nx: int, ny: int, amp=1e-4, wavelength=64.0, n_wavelengths=8,
                 centre=None, rho0=1.0, u0=0.0):
    """Right-going plane acoustic packet, y-uniform:
    rho' = amp sin(2 pi (x - xc)/lambda) * Hann over n_wavelengths,
    u'_x = c_s rho' / rho0."""
    xc = nx / 2.0 if centre is None else float(centre)
    x = np.arange(nx, dtype=np.float64)
    span = wavelength * n_wavelengths
    t = (x - (xc - span / 2.0)) / span
    hann = np.where((t >= 0) & (t <= 1), 0.5 - 0.5 * np.cos(2 * np.pi * t), 0.0)
    rp = amp * np.sin(2 * np.pi * (x - xc) / wavelength) * hann
    rho = np.broadcast_to(rho0 + rp, (ny, nx)).copy()
    ux = np.broadcast_to(u0 + CS * rp / rho0, (ny, nx)).copy()
    uy = np.zeros((ny, nx))
    return rho, ux, uy


# ---------------------------------------------------------------- workload configs

@dataclass
class DomainSpec:
    """One lattice run: sizes, storage, parameters and initial fields recipe."""
    nx: int
    ny: int
    variant: str = "II"
    storage: str = "f32"
    s: tuple = S_MRT_DEFAULT
    shift_n: float = 0.5
    shift_m: float = 0.5
    chi_max: float = 0.1
    width: int = 20
    u0: float = 0.0
    rho0: float = 1.0
    base: str = "ref"  # "rest": w_i rho0; "ref": f^eq(rho0, u0)
    pulses: list = field(default_factory=list)  # [(cx, cy, amp, b)]
    steps: int = 1000
    seed: int = 0

    def fields(self):
        if not self.pulses:
            return gaussian_pulses(self.nx, self.ny, [], [], [], self.rho0, (self.u0, 0.0))
        c = [(p[0], p[1]) for p in self.pulses]
        a = [p[2] for p in self.pulses]
        b = [p[3] for p in self.pulses]
        return gaussian_pulses(self.nx, self.ny, c, a, b, self.rho0, (self.u0, 0.0))

    def chi_1d(self):
        return (quadratic_ramp_1d(self.nx, self.width, self.chi_max),
                quadratic_ramp_1d(self.ny, self.width, self.chi_max))

    def chi_2d(self):
        cx, cy = self.chi_1d()
        return sponge_2d(cx, cy)

    @property
    def qref(self):
        return (self.rho0, self.u0, 0.0)

    @property
    def base_state(self):
        return (self.rho0, self.u0 if self.base == "ref" else 0.0, 0.0)

    def footprint_bytes(self):
        es = {"f64": 8, "f32": 4, "f16": 2}[self.storage]
        return 2 * 9 * es * self.nx * self.ny + 8 * (self.nx + self.ny)


def pulse_c1(variant="II", steps=1000) -> DomainSpec:
    """128^2 FP64, u0 = 0, centred pulse eps = 1e-3, b = 5, 20-cell quadratic
    ramp to chi_max = 0.1, q_ref at rest."""
    n = 128
    return DomainSpec(nx=n, ny=n, variant=variant, storage="f64", chi_max=0.1,
                      width=20, u0=0.0, pulses=[((n - 1) / 2, (n - 1) / 2, 1e-3, 5.0)],
                      steps=steps, seed=SEED_BASE + 0)


def large_c2(variant="II", storage="f32", steps=2000, n=4096, base="ref") -> DomainSpec:
    """4096^2, Mach 0.2 mean flow in x, 32 seeded pulses (amp U[1e-4,1e-3],
    b U[4,16], centres U[64, n-64)^2), 64-cell ramp to chi_max = 0.2."""
    g = rng(1)
    lo, hi = 64, n - 64
    pulses = []
    for _ in range(32):
        cx, cy = g.uniform(lo, hi, size=2)
        pulses.append((cx, cy, g.uniform(1e-4, 1e-3), g.uniform(4.0, 16.0)))
    return DomainSpec(nx=n, ny=n, variant=variant, storage=storage, chi_max=0.2,
                      width=64, u0=0.2 * CS, pulses=pulses, steps=steps, base=base,
                      seed=SEED_BASE + 1)


def paper_pulse(strategy="II", thickness_b=4, u0=0.0, s=1.9999, n=200, b_cells=10.0,
                storage="f64"):
    """The pulse of Section 4.1 on an n x n lattice: eps = 1e-3, b = n/20 cells,
    centred; absorbing layer of thickness m b on all sides. Type II uses
    chi = 4/s - 0.001 with the normalised A = n = 4 profile of eq.
    normalizedsigma (sigma = chi sigma~); the viscosity strategy ramps the
    rates linearly to 1 over the same layer (its sponge arrays carry the ramp
    coordinate xi); 'none' has no layer. Returns (spec, profile_x, profile_y)."""
    W = int(round(thickness_b * b_cells))
    c = (n - 1) / 2
    S = (0.0, 0.0, 0.0) + (s,) * 6
    spec = DomainSpec(nx=n, ny=n, variant={"none": "none", "visc": "visc"}.get(strategy, strategy),
                      storage=storage, s=S, chi_max=4.0 / s - 0.001, width=W, u0=u0,
                      pulses=[(c, c, 1e-3, b_cells)])
    if strategy == "none":
        prof = np.zeros(n)
    elif strategy == "visc":
        prof = ramp_depth(n, W)
    else:
        prof = orszag_profile_1d(n, W, spec.chi_max)
    return spec, prof, prof.copy()


def right_ramp_depth(n: int, width: int) -> np.ndarray:
    """xi(i) = max(0, (W - (n-1-i)) / W): 1 at the last cell, 0 from depth W
    inwards (a layer at the right end only)."""
    i = np.arange(n, dtype=np.float64)
    if width <= 0:
        return np.zeros(n)
    return np.maximum(0.0, (width - (n - 1 - i)) / width)


def paper_line_source(strategy="II", thickness=0.8, u0=0.0, cells_per_unit=200, length=4.0,
                      height=1.0, amp=1e-3, omega=2.0, re=1e6, length_factor=1):
    """The acoustic line source of Section 4.2 in lattice units: a channel of
    length W = 4H, H = 1, with ``cells_per_unit`` cells per unit length;
    rho_src = 1 + amp sin(2 pi omega t) at x = 0 (omega = 2, i.e. omega /
    cells_per_unit cycles per step; wavelength c_s / omega), mean flow u0
    along x, periodic in y, outflow at the right; Re = 1/nu = 1e6 in the
    paper's units fixes s; chi = 4/s - 0.001 with the normalised profile of
    eq. normalizedsigma over a layer of ``thickness`` at the right end (the
    viscosity strategy ramps the rates to 1 over it; 'none' has no layer).
    ``length_factor`` stretches the channel (the reference run). Returns a
    dict with nx, ny, s, variant, profile (along x), source tuple, and the
    paper's sample time T_o + 10 T_p in steps."""
    nx = int(round(length * cells_per_unit * length_factor))
    ny = int(round(height * cells_per_unit))
    nu = cells_per_unit / re            # lattice viscosity: dt = dx = 1 / cells_per_unit
    s = 1.0 / (nu / CS ** 2 + 0.5)
    chi_max = 4.0 / s - 0.001
    W = int(round(thickness * cells_per_unit))
    xi = right_ramp_depth(nx, W)
    if strategy == "none":
        prof = np.zeros(nx)
    elif strategy == "visc":
        prof = xi
    else:
        prof = chi_max * np.where(xi > 0, 3125.0 * (1.0 - xi) * xi ** 4 / 256.0, 0.0)
    freq = omega / cells_per_unit
    t_sample = int(round(length * cells_per_unit / (CS + u0) + 10.0 / freq))
    return {"nx": nx, "ny": ny, "s": (0.0, 0.0, 0.0) + (s,) * 6,
            "variant": {"none": "none", "visc": "visc"}.get(strategy, strategy),
            "profile": prof, "layer_cells": W, "source": (1.0, amp, freq, 0.0, u0, 0.0),
            "u0": u0, "t_sample": t_sample, "wavelength_cells": CS / freq}


# ---------------------------------------------------------------- three-dimensional inputs

def gaussian_pulses_3d(nx: int, ny: int, nz: int, centres, amps, halfwidths, rho0=1.0,
                       u0=(0.0, 0.0, 0.0)):
    """rho = rho0 + sum_k eps_k exp(-ln2 r_k^2 / b_k^2) on the periodic box
    (minimum-image distances), u = u0 uniform. Returns (rho, ux, uy, uz) as
    float64 [nz][ny][nx]."""
    ax = [np.arange(n, dtype=np.float64) for n in (nx, ny, nz)]
    rho = np.full((nz, ny, nx), float(rho0))
    for c, a, b in zip(centres, amps, halfwidths):
        e = []
        for k, n in enumerate((nx, ny, nz)):
            d = ax[k] - c[k]
            d = d - n * np.round(d / n)
            e.append(np.exp(-math.log(2.0) * d * d / (b * b)))
        rho += a * e[2][:, None, None] * e[1][None, :, None] * e[0][None, None, :]
    return (rho,) + tuple(np.full((nz, ny, nx), float(u)) for u in u0)


def sponge_3d(chi_x: np.ndarray, chi_y: np.ndarray, chi_z: np.ndarray,
              combine="max") -> np.ndarray:
    """Full field [nz][ny][nx] of a separable sponge (max or sum)."""
    a, b, c = chi_x[None, None, :], chi_y[None, :, None], chi_z[:, None, None]
    if combine == "max":
        return np.maximum(np.maximum(a, b), c)
    return (a + b) + c


def cube_d3q15(n=256, variant="II", storage="f32", u0=0.1, chi_max=0.2, width=32,
               npulses=16):
    """n^3 periodic box, mean flow u0 along x, ``npulses`` seeded pulses
    (amp U[1e-4, 1e-3], b U[3, 8], centres U[width, n - width)^3), quadratic
    ramp of ``width`` cells to chi_max on all six faces (separable, max).
    Returns a dict: n, variant, storage, u0, fields(), profile, qref."""
    g = rng(5)
    centres = [tuple(g.uniform(width, n - width, size=3)) for _ in range(npulses)]
    amps = g.uniform(1e-4, 1e-3, npulses)
    bs = g.uniform(3.0, 8.0, npulses)
    prof = quadratic_ramp_1d(n, width, chi_max)
    return {"n": n, "variant": variant, "storage": storage, "u0": u0, "profile": prof,
            "qref": (1.0, u0, 0.0, 0.0),
            "fields": lambda: gaussian_pulses_3d(n, n, n, centres, amps, bs, 1.0, (u0, 0.0, 0.0))}


def batch_c4(count=256, seed_index=3, max_exp=1.0):
    """Uneven domains N = round(64 * 8^U), U ~ U[0, max_exp]; chi_max U[0.01, 0.5];
    W U{8..64} clamped to N/4; Mach U[0, 0.3]; variant U{I, II, III};
    centred pulse eps = 1e-3, b = N/20."""
    g = rng(seed_index)
    out = []
    for k in range(count):
        N = int(round(64 * 8 ** g.uniform(0.0, max_exp)))
        chi_max = float(g.uniform(0.01, 0.5))
        W = clamp_width(int(g.integers(8, 65)), N)
        ma = float(g.uniform(0.0, 0.3))
        var = ("I", "II", "III")[int(g.integers(0, 3))]
        c = (N - 1) / 2
        out.append(DomainSpec(nx=N, ny=N, variant=var, storage="f32", chi_max=chi_max,
                              width=W, u0=ma * CS, pulses=[(c, c, 1e-3, N / 20.0)],
                              steps=1000, seed=SEED_BASE + seed_index * 100000 + k))
    return out


def vn_param_sets(count=64, seed_index=3):
    """Von Neumann parameter sets. Sets 0-11: the paper's cases (BGK, theta = 0
    figures of Section 3.3); the rest are seeded draws with MRT S.
    Each entry: dict(s=9-tuple, chi, qref, variant, n, m)."""
    sets = []
    for s in (1.9, 1.99, 1.99999):
        for dchi in (0.0, -0.1, 0.1):
            sets.append(dict(s=(s,) * 9, chi=4.0 / s + dchi, qref=(1.0, 0.0, 0.0),
                             variant="II", n=0.5, m=0.5))
    sets.append(dict(s=(1.9,) * 9, chi=0.1, qref=(1.0, 0.0, 0.0), variant="I", n=0.5, m=0.5))
    sets.append(dict(s=(1.99,) * 9, chi=0.2, qref=(1.0, 0.0, 0.0), variant="I", n=0.5, m=0.5))
    sets.append(dict(s=(1.99,) * 9, chi=3.0 / 1.99, qref=(1.0, 0.1, 0.0), variant="III", n=0.5, m=0.5))
    g = rng(seed_index, salt=7)
    while len(sets) < count:
        var = ("I", "II", "III")[int(g.integers(0, 3))]
        sets.append(dict(s=S_MRT_DEFAULT, chi=float(g.uniform(0.01, 0.5)),
                         qref=(1.0, float(g.uniform(0.0, 0.3)) * CS, 0.0),
                         variant=var, n=0.5, m=0.5))
    return sets[:count]


def vn_grid(nk: int):
    """Wavenumber grid k = 2 pi (p - nk/2)/nk on [-pi, pi)^2 -> (kx, ky) flat."""
    k1 = 2 * np.pi * (np.arange(nk) - nk // 2) / nk
    kx, ky = np.meshgrid(k1, k1, indexing="xy")
    return kx.ravel().copy(), ky.ravel().copy()
