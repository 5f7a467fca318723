"""Seeded synthetic inputs for the cavity-coupled LLG workloads.

This module holds problem descriptions (grid, cell, material and cavity
parameters) and the seeded generators of initial states and per-cell maps.
It contains none of the method's arithmetic: no field, torque, cavity or
integrator code lives here.  Both the FP64 CPU oracle and the HIP library
receive the same arrays and scalars from it.

Units are SI throughout (T, A/m, J/m, J/m^3, rad/s, s).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

# Physical constants.  The paper fixes hbar (cavity parameter list, section
# "Workflow in Mumax3-cQED"); it gives no value for the gyromagnetic ratio, so
# the usual micromagnetic default is taken.
GAMMA = 1.7595e11          # rad s^-1 T^-1
HBAR = 1.05457182e-34      # J s
MU0 = 4e-7 * math.pi       # T m / A
KB = 1.380649e-23          # J / K (exact, SI 2019)

DRIVE_NONE, DRIVE_SINC, DRIVE_CW = 0, 1, 2
CAVITY_ODE, CAVITY_MEMORY = 0, 1
METHOD_RK4, METHOD_DP45 = 0, 1
MAX_MODES = 8


@dataclasses.dataclass
class Mode:
    """One mode of a multimode cavity: its vacuum field (uniform vector, or
    a per-cell map of shape (3, nz, ny, nx) float32 that replaces it),
    frequency and loss (rad/s), initial amplitude alpha_0 = (x0 - i p0)/2,
    and its own drive d(alpha_k)/dt -= i cdrive_amp f(t)."""
    brms: tuple = (0.0, 0.0, 0.0)
    wc: float = 0.0
    kappa: float = 0.0
    x0: float = 0.0
    p0: float = 0.0
    cdrive_kind: int = DRIVE_NONE
    cdrive_amp: float = 0.0
    cdrive_w: float = 0.0
    brms_map: Optional[np.ndarray] = None


@dataclasses.dataclass
class Problem:
    """One cavity-LLG problem instance (single grid, single cavity mode)."""
    nx: int
    ny: int
    nz: int
    dx: float
    dy: float
    dz: float
    ms: float = 8.0e5
    aex: float = 1.3e-11
    alpha: float = 0.01
    ku1: float = 0.0
    anis_u: tuple = (0.0, 0.0, 1.0)
    bext: tuple = (0.0, 0.0, 0.0)
    # field drive: B_ext(t) = bext + fdrive_amp * f(t) * fdrive_dir, or
    # with a per-cell shape fdrive_map (3, nz, ny, nx) float32 in place of
    # fdrive_dir: bext + fdrive_amp * f(t) * fdrive_map[:, cell]
    fdrive_kind: int = DRIVE_NONE
    fdrive_amp: float = 0.0
    fdrive_w: float = 0.0
    fdrive_dir: tuple = (0.0, 0.0, 0.0)
    enable_demag: bool = True
    brms: tuple = (0.0, 0.0, 0.0)      # T, uniform vacuum field of the mode
    wc: float = 0.0                    # rad/s
    kappa: float = 0.0                 # rad/s
    x0: float = 0.0                    # 2 Re(alpha_0)
    p0: float = 0.0                    # -2 Im(alpha_0)
    # cavity drive: d(alpha)/dt gains -i * cdrive_amp * f(t)
    cdrive_kind: int = DRIVE_NONE
    cdrive_amp: float = 0.0
    cdrive_w: float = 0.0
    gamma: float = GAMMA
    hbar: float = HBAR
    mu0: float = MU0
    method: int = METHOD_RK4
    dt: float = 1e-13
    tol: float = 1e-6
    dt_min: float = 1e-20
    dt_max: float = 1e-10
    # cavity treatment: CAVITY_ODE (alpha integrated with m) or
    # CAVITY_MEMORY (the paper's integrated-out recursion; RK4 only)
    cavity_mode: int = 0
    # second-order uniaxial anisotropy (J/m^3, same axis as ku1) and the
    # precession switch (0: damping term only, relaxation dynamics)
    ku2: float = 0.0
    # Dzyaloshinskii-Moriya constants (J/m^2): interfacial (film normal z)
    # and bulk
    dmi_int: float = 0.0
    dmi_bulk: float = 0.0
    # thermal field (K) and the seed of its counter-based generator
    temperature: float = 0.0
    seed: int = 0
    precession: int = 1
    # optional per-cell maps, float32 arrays of shape (nz, ny, nx)
    ms_map: Optional[np.ndarray] = None
    ku1_map: Optional[np.ndarray] = None
    # optional vacuum field of the mode per cell, float32 (3, nz, ny, nx) in
    # T; replaces the uniform brms when given
    brms_map: Optional[np.ndarray] = None
    fdrive_map: Optional[np.ndarray] = None
    # multimode cavity: a list of Mode (1..MAX_MODES); when given, it
    # replaces the single mode of brms/brms_map/wc/kappa/x0/p0/cdrive_*
    modes: Optional[list] = None

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def ncells(self):
        return self.nx * self.ny * self.nz

    @property
    def vcell(self):
        return self.dx * self.dy * self.dz

    def ms_array(self) -> np.ndarray:
        """Per-cell saturation magnetisation as float64 (nz, ny, nx)."""
        if self.ms_map is not None:
            return np.asarray(self.ms_map, dtype=np.float64)
        return np.full(self.shape, float(self.ms))

    def ku_array(self) -> np.ndarray:
        if self.ku1_map is not None:
            return np.asarray(self.ku1_map, dtype=np.float64)
        return np.full(self.shape, float(self.ku1))


def brms_from_g(g: float, ms_total_volume: float, gamma: float = GAMMA,
                hbar: float = HBAR) -> float:
    """|B_rms| that realises a Dicke collective coupling lambda = g.

    The paper maps one macrospin onto the Dicke model with
    B_rms = sqrt(2/S) lambda / gamma and S hbar = Ms V / gamma (sections
    "The LLG equation in Mumax3" and "Benchmark"), so
    |B_rms| = g * sqrt(2 hbar / (gamma * sum_i Ms_i V_c)).
    `ms_total_volume` is sum_i Ms_i V_c in A m^2.
    """
    return g * math.sqrt(2.0 * hbar / (gamma * ms_total_volume))


def normalise_rows(m: np.ndarray) -> np.ndarray:
    """m has shape (3, ...); returns unit vectors (float64)."""
    n = np.sqrt((m * m).sum(axis=0))
    return m / n


def tilted_uniform_state(shape, tilt_deg: float, noise: float, seed: int,
                         axis: str = "z", toward: str = "x") -> np.ndarray:
    """Uniform m along `axis`, tilted `tilt_deg` toward `toward`, plus seeded
    uniform per-component noise in [-noise, noise] drawn in [c][z][y][x]
    order, normalised and rounded to float32.  Returns (3, nz, ny, nx) f32."""
    nz, ny, nx = shape
    idx = {"x": 0, "y": 1, "z": 2}
    v = np.zeros(3)
    th = math.radians(tilt_deg)
    v[idx[axis]] = math.cos(th)
    if tilt_deg != 0.0:
        v[idx[toward]] = math.sin(th)
    m = np.empty((3, nz, ny, nx))
    for c in range(3):
        m[c] = v[c]
    rng = np.random.default_rng(seed)
    m += rng.uniform(-noise, noise, size=m.shape)
    return normalise_rows(m).astype(np.float32)


def film_texture(nx: int, ny: int, nz: int, dx: float, dy: float,
                 ncentres: int, core_radius: float, seed: int) -> np.ndarray:
    """Textured film: each cell takes its nearest of `ncentres` seeded centres
    (periodic distance not used); in-plane curl about the centre with seeded
    chirality, out-of-plane core m_z = p*exp(-(r/core_radius)^2) with seeded
    polarity.  Returns normalised (3, nz, ny, nx) float32."""
    rng = np.random.default_rng(seed)
    cx = rng.uniform(0, nx * dx, size=ncentres)
    cy = rng.uniform(0, ny * dy, size=ncentres)
    chir = rng.choice([-1.0, 1.0], size=ncentres)
    pol = rng.choice([-1.0, 1.0], size=ncentres)
    xs = (np.arange(nx) + 0.5) * dx
    ys = (np.arange(ny) + 0.5) * dy
    X, Y = np.meshgrid(xs, ys)              # (ny, nx)
    best = np.full(X.shape, np.inf)
    owner = np.zeros(X.shape, dtype=np.int64)
    for k in range(ncentres):
        d2 = (X - cx[k]) ** 2 + (Y - cy[k]) ** 2
        sel = d2 < best
        best[sel] = d2[sel]
        owner[sel] = k
    rx = X - cx[owner]
    ry = Y - cy[owner]
    r = np.sqrt(rx * rx + ry * ry)
    mz = pol[owner] * np.exp(-(r / core_radius) ** 2)
    inpl = np.sqrt(np.clip(1.0 - mz * mz, 0.0, None))
    rr = np.where(r > 0, r, 1.0)
    ux = np.where(r > 0, -ry / rr, 1.0) * chir[owner]
    uy = np.where(r > 0, rx / rr, 0.0) * chir[owner]
    m = np.empty((3, nz, ny, nx))
    m[0] = (ux * inpl)[None]
    m[1] = (uy * inpl)[None]
    m[2] = mz[None]
    return normalise_rows(m).astype(np.float32)


def smooth_map(nx: int, ny: int, nz: int, lo: float, hi: float, nmodes: int,
               kmax: int, seed: int) -> np.ndarray:
    """Seeded smooth scalar field: sum of `nmodes` Fourier modes with integer
    wave numbers |k| <= kmax cycles per side, affinely mapped to exactly
    [lo, hi], identical in every layer.  Returns (nz, ny, nx) float32."""
    rng = np.random.default_rng(seed)
    xs = (np.arange(nx) + 0.5) / nx
    ys = (np.arange(ny) + 0.5) / ny
    X, Y = np.meshgrid(xs, ys)
    f = np.zeros_like(X)
    for _ in range(nmodes):
        while True:
            kx, ky = rng.integers(-kmax, kmax + 1, size=2)
            if 0 < kx * kx + ky * ky <= kmax * kmax:
                break
        ph = rng.uniform(0, 2 * math.pi)
        amp = rng.uniform(0.5, 1.0)
        f += amp * np.cos(2 * math.pi * (kx * X + ky * Y) + ph)
    f = (f - f.min()) / (f.max() - f.min())
    f = lo + (hi - lo) * f
    return np.broadcast_to(f, (nz, ny, nx)).astype(np.float32).copy()


# ---------------------------------------------------------------------------
# Workload definitions.  Sizes and parameters follow the five synthetic
# workloads the path is measured on; where a workload leaves a value open,
# the choice is stated at the workload.
# ---------------------------------------------------------------------------

# Cavity frequency of the small plain workload: the small-angle Kittel
# frequency of the uniform mode about +z, with the film's demagnetising
# factors taken as the whole-box average of the oracle's cell tensor
# (written by tests/golden/make_golden.py, frozen here).
C1_WC = 2.0 * math.pi * 21.8214597e9


def c1_small(wc: float = None, g_over_wc: float = 0.01) -> tuple:
    """32x32x1 cells of 5 nm, Bext 0.1 T along z, RK4 dt=2e-13 s x 5000."""
    p = Problem(nx=32, ny=32, nz=1, dx=5e-9, dy=5e-9, dz=5e-9,
                ms=8.0e5, aex=1.3e-11, alpha=0.01, ku1=0.0,
                bext=(0.0, 0.0, 0.1), method=METHOD_RK4, dt=2e-13)
    p.wc = C1_WC if wc is None else wc
    p.kappa = 1e-3 * p.wc
    g = g_over_wc * p.wc
    p.brms = (brms_from_g(g, p.ms * p.ncells * p.vcell), 0.0, 0.0)
    m0 = tilted_uniform_state(p.shape, 5.0, 1e-3, seed=1001)
    return p, m0, dict(steps=5000, record_every=10)


def c3_film() -> tuple:
    """1024x1024x2 cells of 4 nm textured film, DP45 tol 1e-6 (the initial
    texture here is the unrelaxed one; relaxation is run on the GPU)."""
    p = Problem(nx=1024, ny=1024, nz=2, dx=4e-9, dy=4e-9, dz=4e-9,
                ms=8.0e5, aex=1.3e-11, alpha=0.02,
                bext=(0.02, 0.0, 0.0), method=METHOD_DP45, tol=1e-6,
                dt=1e-14)
    p.wc = 2.0 * math.pi * 4.01e9
    p.kappa = 1e-3 * p.wc
    g = 0.005 * p.wc
    p.brms = (0.0, brms_from_g(g, p.ms * p.ncells * p.vcell), 0.0)
    m0 = film_texture(p.nx, p.ny, p.nz, p.dx, p.dy, 64, 10e-9, seed=1003)
    return p, m0, dict(t_end=5e-9, relax_t=0.5e-9, relax_alpha=0.5)


# uniform-mode frequency of the nanowire (prism factors, anisotropy field),
# frozen from tests/golden/c2_uniform_mode_hz.txt
C2_WC = 2.0 * math.pi * 9.897394623e9


def c2_nanowire() -> tuple:
    """512x32x4 cells of 4 nm, Ku1 5e3 J/m^3 along x, alpha 0.005, DP45;
    cavity at the wire's uniform-mode frequency, g/wc = 0.02 with B_rms
    along y, driven by a sinc pulse of 20 GHz bandwidth whose amplitude
    gives a free-cavity field 2 |B_rms| |alpha| of about 1 mT."""
    p = Problem(nx=512, ny=32, nz=4, dx=4e-9, dy=4e-9, dz=4e-9,
                ms=8.0e5, aex=1.3e-11, alpha=0.005, ku1=5e3,
                anis_u=(1.0, 0.0, 0.0), bext=(0.0, 0.0, 0.0),
                method=METHOD_DP45, tol=1e-6, dt=1e-14)
    p.wc = C2_WC
    p.kappa = 1e-3 * p.wc
    b = brms_from_g(0.02 * p.wc, p.ms * p.ncells * p.vcell)
    p.brms = (0.0, b, 0.0)
    p.cdrive_kind = DRIVE_SINC
    p.cdrive_w = 2.0 * math.pi * 20e9
    # a sinc pulse eps0 sinc(w t) leaves a lossless resonator below the
    # cut-off (wc < w) with |alpha| = (eps0/w) |pi/2 + (i/2) ln((w+wc)/(w-wc))|
    # (the t -> infinity limit of the sine/cosine-integral closed form);
    # eps0 is set so that 2 |B_rms| |alpha| = 1 mT
    w, wc = p.cdrive_w, p.wc
    gain = math.hypot(0.5 * math.pi, 0.5 * math.log((w + wc) / (w - wc))) / w
    p.cdrive_amp = 1e-3 / (2.0 * b) / gain
    m0 = tilted_uniform_state(p.shape, 0.0, 1e-3, seed=1002, axis="x",
                              toward="y")
    return p, m0, dict(t_end=10e-9)


def c5_adjoint() -> tuple:
    """256x256x2 cells of 4 nm with seeded Ms and Ku maps, RK4 dt 1e-13 s."""
    p = Problem(nx=256, ny=256, nz=2, dx=4e-9, dy=4e-9, dz=4e-9,
                ms=8.0e5, aex=1.3e-11, alpha=0.01, ku1=0.0,
                anis_u=(1.0, 0.0, 0.0), bext=(0.1, 0.0, 0.0),
                method=METHOD_RK4, dt=1e-13)
    p.ms_map = smooth_map(p.nx, p.ny, p.nz, 7e5, 9e5, 8, 4, seed=1005)
    p.ku1_map = smooth_map(p.nx, p.ny, p.nz, 0.0, 1e4, 8, 4, seed=10051)
    p.wc = 2.0 * math.pi * 9.31e9
    p.kappa = 1e-3 * p.wc
    g = 0.02 * p.wc
    p.brms = (0.0, brms_from_g(g, 8.0e5 * p.ncells * p.vcell), 0.0)
    p.cdrive_kind = DRIVE_CW
    p.cdrive_w = p.wc
    # resonant CW drive eps0 cos(wc t): of its two counter-rotating halves
    # only e^{-i wc t} is resonant, so the free cavity settles at
    # |alpha| = eps0/(2 kappa); the amplitude gives it a field
    # 2 |B_rms| |alpha| of 1 mT
    p.cdrive_amp = 1e-3 * p.kappa / p.brms[1]
    m0 = tilted_uniform_state(p.shape, 0.0, 1e-3, seed=1005, axis="x",
                              toward="y")
    return p, m0, dict(steps=50000)


def c4_instances(n: int = 512, seed: int = 1004) -> list:
    """Batched sweep: per instance grid U{16..128}^2 x U{1..4} of 5 nm cells,
    g/wc log-uniform 1e-3..1e-1, Bz U(0, 0.3) T, wc/2pi linear 5..15 GHz."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        nx, ny = (int(v) for v in rng.integers(16, 129, size=2))
        nz = int(rng.integers(1, 5))
        g_over_wc = 10.0 ** rng.uniform(-3, -1)
        bz = rng.uniform(0.0, 0.3)
        p = Problem(nx=nx, ny=ny, nz=nz, dx=5e-9, dy=5e-9, dz=5e-9,
                    ms=8.0e5, aex=1.3e-11, alpha=0.01,
                    bext=(0.0, 0.0, bz), method=METHOD_DP45, tol=1e-6,
                    dt=1e-14)
        p.wc = 2.0 * math.pi * (5e9 + 10e9 * k / max(1, n - 1))
        p.kappa = 1e-3 * p.wc
        p.brms = (brms_from_g(g_over_wc * p.wc, p.ms * p.ncells * p.vcell),
                  0.0, 0.0)
        m0 = tilted_uniform_state(p.shape, 5.0, 1e-3, seed=1004 * 1000 + k)
        out.append((p, m0, dict(t_end=2e-9)))
    return out


def dicke_macrospin(wz: float, wc: float, lam: float, kappa: float = 0.0,
                    alpha: float = 0.0, ms: float = 8.0e5,
                    cell: float = 5e-9, m0=None) -> tuple:
    """One cell mapped onto the Dicke model: B_ext = (0, 0, wz/gamma) and
    B_rms = (sqrt(2/S) lambda/gamma, 0, 0), demag off (section "Benchmark")."""
    p = Problem(nx=1, ny=1, nz=1, dx=cell, dy=cell, dz=cell, ms=ms,
                aex=0.0, alpha=alpha, enable_demag=False,
                bext=(0.0, 0.0, wz / GAMMA), method=METHOD_RK4)
    p.wc = wc
    p.kappa = kappa
    p.brms = (brms_from_g(lam, ms * p.vcell), 0.0, 0.0)
    if m0 is None:
        m0 = np.array([math.sin(0.05), 0.0, math.cos(0.05)])
    m0 = np.asarray(m0, dtype=np.float64).reshape(3, 1, 1, 1)
    return p, normalise_rows(m0).astype(np.float32)
