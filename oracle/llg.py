"""FP64 CPU oracle for the cavity-coupled Landau-Lifshitz-Gilbert hot path.

TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the CPU-baseline
leg of the benchmark may import this module; the product path never does, and
this module shares no code with the HIP library.

Plain, slow, obviously correct: every step is the formula written out in
numpy float64, in the order the paper states the problem.

  * LLG in Landau-Lifshitz form with Gilbert damping, Eq. (llg):
        dm/dt = -gamma/(1+alpha^2) [ m x B + alpha m x (m x B) ] .
  * Effective field (sum of contributions listed after Eq. (llg)): Zeeman,
    exchange, uniaxial anisotropy, demagnetisation, plus the cavity field
    B_rms (alpha + alpha^*) that the mean-field equations add,
    Eqs. (eqmotionspinclasical)-(eqmotionaclasical); the cavity field enters
    both the precession and the damping term (end of section "The LLG
    equation in Mumax3").
  * Cavity mode, Eq. (eqmotionaclasical) with the loss omega_c -> omega_c -
    i kappa of section "Introducing the effect of the cavity": with
    S_i = -Ms_i V_c m_i / gamma (moment mu = -gamma S, M = mu/V_c),
        d alpha/dt = -(i wc + kappa) alpha + i (V_c/hbar) sum_i Ms_i m_i.B_rms
                     - i eps(t)            (eps: optional cavity drive).
  * Several cavity modes (section "Ferromagnetic materials in a cavity":
    a multimode cavity is the sum of its modes): each mode k has its own
    vacuum field B_rms,k (uniform or per cell), frequency, loss and drive;
    the cavity field is sum_k B_rms,k (alpha_k + alpha_k^*) and each
    amplitude obeys the single-mode equation with its own coupling sum
    F_k = sum_i Ms_i m_i . B_rms,k,i.
  * Dzyaloshinskii-Moriya interaction, one of the effective-field terms the
    paper lists after Eq. (llg) (defined in the Mumax3 reference it cites):
    interfacial, energy density D [m_z div m - (m.grad) m_z], and bulk,
    D m.(curl m).  Discretised on the bonds between neighbouring magnetic
    cells i, j (unit vector e_ij, spacing d_ij):
        E = sum_bonds c_ij . (m_i x m_j),
        c_ij = D_int V_c (z x e_ij)/d_ij - D_bulk V_c e_ij/d_ij,
    whose continuum limit is the energy density above; the field is
    B_i = -(1/(Ms_i V_c)) dE/dm_i = (1/(Ms_i V_c)) sum_j c_ij x m_j (in the
    interior the central differences of (2D/Ms)(dm_z/dx, dm_z/dy,
    -dm_x/dx - dm_y/dy) and -(2D/Ms) curl m).  At an open edge the missing
    bond is omitted, as for exchange.
  * Thermal field, the last effective-field term listed after Eq. (llg)
    (Brown's fluctuating field): per cell and component a Gaussian of
    variance 2 alpha kB T / (gamma Ms_i V_c dt), drawn afresh for every
    time step and held over its Runge-Kutta stages (fixed-step RK4 only).
    The normals come from the counter-based Philox4x32-10 generator of
    Salmon et al. (SC'11), key (seed mod 2^32, seed >> 32), counter (cell,
    step mod 2^32, step >> 32, 0), its four words made uniform as
    (w + 1/2) 2^-32 and normal by the Box-Muller transform (pairs (u0, u1)
    and (u2, u3); three of the four normals used).
  * A field drive shaped in space: B_ext += amp f(t) b(r), the form the
    paper's example script uses with the mode's field map as b(r) and a
    sinc pulse as f(t) (appendix "Micromagnetic simulations with
    Mumax3-cQED").
  * Time integration: classic RK4 (fixed step) or Dormand-Prince 5(4) with
    FSAL on the joint state (m, alpha); m renormalised after every accepted
    step; time-dependent terms evaluated at the stage times.
  * The integrated-out (memory-kernel) form of the cavity field, Eqs.
    (bcav)-(gammafinal), and the paper's rectangle-rule recursion,
    Eqs. (Sdiscrete)-(gammadiscretefinal), are provided for cross-checks,
    and an RK4 integrator of m driven by that recursion (the paper's own
    scheme: run_rk4_memory).

Readings where the paper is silent: gamma = 1.7595e11 rad/(s T); open
(Neumann) exchange boundaries; zero padding 2n per axis; DP45 error norm
max(max_i |m5-m4|_2, |a5-a4|/max(1,|a5|)) with controller
dt <- dt*clamp(0.9 (tol/err)^(1/5), 0.2, 5), no growth right after a
rejection; sinc(0) = 1.  Several modes: the amplitude part of the DP45
error is the 2-norm over the modes, |a5-a4|_2 / max(1, |a5|_2).
"""
from __future__ import annotations

import math

import numpy as np

from . import demag as _demag

DRIVE_NONE, DRIVE_SINC, DRIVE_CW = 0, 1, 2
KB = 1.380649e-23        # J/K

# Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
# easy as 1, 2, 3", SC'11): multipliers and Weyl key increments.
_PHILOX_M = (0xD2511F53, 0xCD9E8D57)
_PHILOX_W = (0x9E3779B9, 0xBB67AE85)


def philox4x32(ctr, key, rounds=10):
    """Philox4x32 on arrays: ctr (4, n) of uint32 values (held in uint64),
    key (k0, k1).  Each round: (hi0, lo0) = M0 c0, (hi1, lo1) = M1 c2 (64-bit
    products), c <- (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0); the key is
    bumped by the Weyl constants between rounds.  Returns (4, n) uint64
    holding the 32-bit outputs."""
    mask = np.uint64(0xFFFFFFFF)
    c = [np.asarray(x, dtype=np.uint64) & mask for x in ctr]
    k0, k1 = np.uint64(key[0]) & mask, np.uint64(key[1]) & mask
    for r in range(rounds):
        p0 = np.uint64(_PHILOX_M[0]) * c[0]
        p1 = np.uint64(_PHILOX_M[1]) * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & mask
        hi1, lo1 = p1 >> np.uint64(32), p1 & mask
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
        if r + 1 < rounds:
            k0 = (k0 + np.uint64(_PHILOX_W[0])) & mask
            k1 = (k1 + np.uint64(_PHILOX_W[1])) & mask
    return np.stack(c)


# Dormand & Prince (1980) RK5(4)7M tableau.
DP_C = np.array([0.0, 1 / 5, 3 / 10, 4 / 5, 8 / 9, 1.0, 1.0])
DP_A = [
    [],
    [1 / 5],
    [3 / 40, 9 / 40],
    [44 / 45, -56 / 15, 32 / 9],
    [19372 / 6561, -25360 / 2187, 64448 / 6561, -212 / 729],
    [9017 / 3168, -355 / 33, 46732 / 5247, 49 / 176, -5103 / 18656],
    [35 / 384, 0.0, 500 / 1113, 125 / 192, -2187 / 6784, 11 / 84],
]
DP_B5 = np.array([35 / 384, 0.0, 500 / 1113, 125 / 192, -2187 / 6784, 11 / 84,
                  0.0])
DP_B4 = np.array([5179 / 57600, 0.0, 7571 / 16695, 393 / 640,
                  -92097 / 339200, 187 / 2100, 1 / 40])


def drive_shape(kind, w, t):
    """Time profile f(t) of a drive: sinc(w t) with sinc(0)=1, or cos(w t)."""
    if kind == DRIVE_NONE:
        return 0.0
    if kind == DRIVE_SINC:
        x = w * t
        return 1.0 if x == 0.0 else math.sin(x) / x
    if kind == DRIVE_CW:
        return math.cos(w * t)
    raise ValueError(kind)


def normalise(m):
    """m / |m| per cell; cells outside the geometry (m = 0) stay zero."""
    n = np.sqrt((m * m).sum(axis=0))
    return m / np.where(n > 0.0, n, 1.0)


class CavityLLG:
    """The joint (m, alpha) right-hand side and integrators for one Problem.

    m has shape (3, nz, ny, nx); alpha is a Python complex.
    demag: 'fft' (zero-padded FFT convolution), 'direct' (brute force), or
    'auto' (direct for <= 64 cells)."""

    def __init__(self, prob, demag="auto"):
        self.p = prob
        self.shape = (prob.nz, prob.ny, prob.nx)
        self.ms = prob.ms_array()
        # geometry: cells with Ms = 0 hold no magnetisation (m = 0 there);
        # exchange ignores them and averages run over the magnetic cells
        self.inside = self.ms > 0.0
        self.inv_ms = np.where(self.inside, 1.0 / np.where(self.inside,
                                                           self.ms, 1.0), 0.0)
        self.ku = prob.ku_array()
        self.vc = prob.dx * prob.dy * prob.dz
        self.u = np.asarray(prob.anis_u, dtype=np.float64)
        # vacuum field of the mode per cell, (3, nz, ny, nx): the map when
        # one is given (section "Workflow in Mumax3-cQED": B_rms may vary in
        # space), else the uniform vector everywhere
        bmap = getattr(prob, "brms_map", None)
        if bmap is not None:
            self.brms_cells = np.asarray(bmap, dtype=np.float64).reshape(
                (3,) + self.shape)
        else:
            self.brms_cells = np.asarray(prob.brms, dtype=np.float64).reshape(
                3, 1, 1, 1) * np.ones((1,) + self.shape)
        self.brms = np.asarray(prob.brms, dtype=np.float64)
        # multimode cavity: amplitudes are a complex array over the modes
        self.multi = getattr(prob, "modes", None) is not None
        if self.multi:
            modes = list(prob.modes)
            if not 1 <= len(modes) <= 8:
                raise ValueError("1..8 modes")
            cells = []
            for md in modes:
                if md.brms_map is not None:
                    cells.append(np.asarray(md.brms_map, dtype=np.float64)
                                 .reshape((3,) + self.shape))
                else:
                    cells.append(np.asarray(md.brms, dtype=np.float64)
                                 .reshape(3, 1, 1, 1)
                                 * np.ones((1,) + self.shape))
            self.modes = modes
            self.mode_cells = np.stack(cells)            # (M, 3, nz, ny, nx)
            self.mode_wc = np.array([md.wc for md in modes], dtype=float)
            self.mode_kappa = np.array([md.kappa for md in modes],
                                       dtype=float)
        fmap = getattr(prob, "fdrive_map", None)
        self.fdrive_cells = None if fmap is None else np.asarray(
            fmap, dtype=np.float64).reshape((3,) + self.shape)
        self.nfull = None
        self.kf = None
        self.demag_mode = None
        if prob.enable_demag:
            ncell = prob.nx * prob.ny * prob.nz
            mode = demag
            if mode == "auto":
                mode = "direct" if ncell <= 64 else "fft"
            self.demag_mode = mode
            self.nfull = _demag.tensor_full(prob.nx, prob.ny, prob.nz,
                                            prob.dx, prob.dy, prob.dz)
            if mode == "fft":
                self.kf = _demag.demag_kernel_fft(self.nfull, self.shape)
        self.nevals = 0
        self.noise_step = 0        # index of the step the thermal field of
                                   # the next evaluation belongs to
        self._dt_noise = prob.dt   # step size in the thermal variance

    # ---------------------------------------------------------------- fields
    def zeeman(self, t):
        """Static field plus the drive amp f(t) times its direction, or
        times its per-cell shape when a drive map is given."""
        p = self.p
        b = np.asarray(p.bext, dtype=np.float64)
        f = drive_shape(p.fdrive_kind, p.fdrive_w, t)
        if self.fdrive_cells is not None:
            return (b.reshape(3, 1, 1, 1) * np.ones((1,) + self.shape)
                    + p.fdrive_amp * f * self.fdrive_cells)
        b = b + p.fdrive_amp * f * np.asarray(p.fdrive_dir, dtype=np.float64)
        return b.reshape(3, 1, 1, 1) * np.ones((1,) + self.shape)

    def exchange(self, m):
        """B_ex,i = (2A/Ms_i) sum_neighbours (m_j - m_i)/d^2, open boundary:
        neighbours outside the grid or outside the geometry are omitted."""
        p = self.p
        lap = np.zeros_like(m)
        ins = self.inside[None]
        for axis, d in ((3, p.dx), (2, p.dy), (1, p.dz)):
            if m.shape[axis] < 2:
                continue
            lo = [slice(None)] * 4
            hi = [slice(None)] * 4
            lo[axis] = slice(0, -1)
            hi[axis] = slice(1, None)
            pair = ins[tuple(lo)] & ins[tuple(hi)]
            diff = np.where(pair, np.diff(m, axis=axis) / (d * d), 0.0)
            lap[tuple(lo)] += diff
            lap[tuple(hi)] -= diff
        return 2.0 * p.aex * self.inv_ms * lap

    def anisotropy(self, m):
        """Uniaxial, first and second order (energy density
        -Ku1 (u.m)^2 - Ku2 (u.m)^4): B_a = (2 Ku1 (u.m) + 4 Ku2 (u.m)^3)/Ms u."""
        um = np.einsum("c,czyx->zyx", self.u, m)
        ku2 = getattr(self.p, "ku2", 0.0)
        return ((2.0 * self.ku * um + 4.0 * ku2 * um ** 3)
                * self.inv_ms)[None] * self.u.reshape(3, 1, 1, 1)

    def _dmi_bonds(self):
        """(axis, spacing, c-vector per unit D_int, per unit D_bulk) for the
        bonds along x, y, z; a bond joins cell i and its + neighbour."""
        p = self.p
        z = np.array([0.0, 0.0, 1.0])
        out = []
        for axis, d, e in ((3, p.dx, np.array([1.0, 0.0, 0.0])),
                           (2, p.dy, np.array([0.0, 1.0, 0.0])),
                           (1, p.dz, np.array([0.0, 0.0, 1.0]))):
            out.append((axis, d, np.cross(z, e) / d, -e / d))
        return out

    def dmi_energy(self, m):
        """E_dmi = sum over bonds of c_ij . (m_i x m_j) (J)."""
        p = self.p
        di = getattr(p, "dmi_int", 0.0)
        db = getattr(p, "dmi_bulk", 0.0)
        if di == 0.0 and db == 0.0:
            return 0.0
        vc = self.vc
        ins = self.inside[None]
        e = 0.0
        for axis, d, ci, cb in self._dmi_bonds():
            if m.shape[axis] < 2:
                continue
            c = vc * (di * ci + db * cb)
            lo = [slice(None)] * 4
            hi = [slice(None)] * 4
            lo[axis] = slice(0, -1)
            hi[axis] = slice(1, None)
            pair = (ins[tuple(lo)] & ins[tuple(hi)])[0]
            cr = np.cross(m[tuple(lo)], m[tuple(hi)], axis=0)
            e += float((np.einsum("c,c...->...", c, cr) * pair).sum())
        return e

    def dmi(self, m):
        """B_i = (1/(Ms_i V_c)) sum over the bonds of i of c_ij x m_j,
        with c_ij for the bond seen from i (c_ji = -c_ij)."""
        p = self.p
        di = getattr(p, "dmi_int", 0.0)
        db = getattr(p, "dmi_bulk", 0.0)
        B = np.zeros_like(m)
        if di == 0.0 and db == 0.0:
            return B
        ins = self.inside[None]
        for axis, d, ci, cb in self._dmi_bonds():
            if m.shape[axis] < 2:
                continue
            c = (di * ci + db * cb).reshape(3, 1, 1, 1)
            lo = [slice(None)] * 4
            hi = [slice(None)] * 4
            lo[axis] = slice(0, -1)
            hi[axis] = slice(1, None)
            pair = ins[tuple(lo)] & ins[tuple(hi)]
            # cell i (lo) sees j = i + e (hi) through c; j sees i through -c
            B[tuple(lo)] += pair * np.cross(c, m[tuple(hi)], axis=0)
            B[tuple(hi)] -= pair * np.cross(c, m[tuple(lo)], axis=0)
        return B * self.inv_ms[None]

    def demag(self, m):
        if self.demag_mode is None:
            return np.zeros_like(m)
        M = self.ms * m
        if self.demag_mode == "direct":
            return _demag.demag_field_direct(M, self.nfull, self.p.mu0)
        return _demag.demag_field_fft(M, self.kf, self.p.mu0)

    def cavity_field(self, a):
        """B_cav,i = B_rms,i (alpha + alpha^*); several modes: the sum of
        B_rms,k,i (alpha_k + alpha_k^*) over the modes."""
        if self.multi:
            return np.tensordot(2.0 * np.real(a), self.mode_cells, axes=1)
        return self.brms_cells * (2.0 * a.real)

    def thermal(self):
        """Brown's field of step `noise_step` (zero without temperature)."""
        p = self.p
        T = getattr(p, "temperature", 0.0)
        if T <= 0.0:
            return 0.0
        n = self.ms.size
        seed = int(getattr(p, "seed", 0))
        step = int(self.noise_step)
        ctr = np.zeros((4, n), dtype=np.uint64)
        ctr[0] = np.arange(n, dtype=np.uint64)
        ctr[1] = step & 0xFFFFFFFF
        ctr[2] = step >> 32
        w = philox4x32(ctr, (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF))
        u = (w.astype(np.float64) + 0.5) * 2.0 ** -32
        r0 = np.sqrt(-2.0 * np.log(u[0]))
        r1 = np.sqrt(-2.0 * np.log(u[2]))
        eta = np.stack([r0 * np.cos(2 * math.pi * u[1]),
                        r0 * np.sin(2 * math.pi * u[1]),
                        r1 * np.cos(2 * math.pi * u[3])]).reshape(
                            (3,) + self.shape)
        sig = np.sqrt(2.0 * p.alpha * KB * T
                      / (p.gamma * np.where(self.inside, self.ms, 1.0)
                         * self.vc * self._dt_noise))
        return eta * (sig * self.inside)[None]

    def effective_field(self, m, a, t):
        return (self.zeeman(t) + self.exchange(m) + self.anisotropy(m)
                + self.dmi(m) + self.demag(m) + self.cavity_field(a)
                + self.thermal())

    def coupling_sum(self, m):
        """F = sum_i Ms_i m_i . B_rms,i  (A m^-1 T); several modes: the
        array of F_k = sum_i Ms_i m_i . B_rms,k,i."""
        if self.multi:
            return np.array([float((self.ms * (bk * m).sum(axis=0)).sum())
                             for bk in self.mode_cells])
        return float((self.ms * (self.brms_cells * m).sum(axis=0)).sum())

    # -------------------------------------------------------------- dynamics
    def torque(self, m, B):
        """LL torque; with precession switched off only the damping term
        (relaxation dynamics)."""
        p = self.p
        mxB = np.cross(m, B, axis=0)
        mxmxB = np.cross(m, mxB, axis=0)
        prec = 1.0 if getattr(p, "precession", 1) else 0.0
        return -p.gamma / (1.0 + p.alpha ** 2) * (prec * mxB
                                                  + p.alpha * mxmxB)

    def cavity_rate(self, a, F, t):
        p = self.p
        if self.multi:
            eps = np.array([md.cdrive_amp * drive_shape(md.cdrive_kind,
                                                        md.cdrive_w, t)
                            for md in self.modes])
            return (-(1j * self.mode_wc + self.mode_kappa) * a
                    + 1j * (self.vc / p.hbar) * F - 1j * eps)
        eps = p.cdrive_amp * drive_shape(p.cdrive_kind, p.cdrive_w, t)
        return (-(1j * p.wc + p.kappa) * a + 1j * (self.vc / p.hbar) * F
                - 1j * eps)

    def amplitude(self, a0):
        """The cavity state as the integrators hold it: a complex number, or
        a complex array over the modes."""
        if self.multi:
            a = np.asarray(a0, dtype=complex).reshape(-1)
            if a.size == 1 and len(self.modes) > 1:
                a = np.full(len(self.modes), a[0])
            return a.copy()
        return complex(a0)

    def initial_amplitude(self):
        """alpha_0 = (x0 - i p0)/2 of each mode."""
        if self.multi:
            return np.array([0.5 * (md.x0 - 1j * md.p0) for md in self.modes])
        return 0.5 * (self.p.x0 - 1j * self.p.p0)

    @staticmethod
    def anorm(a):
        """|a|, or the 2-norm over the modes."""
        return float(np.sqrt(np.sum(np.abs(a) ** 2)))

    def rhs(self, m, a, t):
        self.nevals += 1
        B = self.effective_field(m, a, t)
        return self.torque(m, B), self.cavity_rate(a, self.coupling_sum(m), t)

    def energy(self, m, a, t=0.0):
        """Total energy of Eq. (startH) in the classical limit (J):
        Zeeman + exchange + anisotropy + DMI + demag - V_c 2Re(a) F
        + hbar wc |a|^2.
        """
        p = self.p
        vc = self.vc
        ez = -vc * (self.ms * (m * self.zeeman(t)).sum(axis=0)).sum()
        ex = 0.0
        for axis, d in ((3, p.dx), (2, p.dy), (1, p.dz)):
            if m.shape[axis] >= 2:
                ex += vc * p.aex * (np.diff(m, axis=axis) ** 2).sum() / (d * d)
        um = np.einsum("c,czyx->zyx", self.u, m)
        ea = -vc * (self.ku * um * um).sum() - vc * (
            getattr(p, "ku2", 0.0) * (self.inside * um ** 4)).sum()
        ed = -0.5 * vc * (self.ms * (m * self.demag(m)).sum(axis=0)).sum()
        if self.multi:
            ec = float(np.sum(-vc * 2.0 * np.real(a) * self.coupling_sum(m)
                              + p.hbar * self.mode_wc * np.abs(a) ** 2))
        else:
            ec = -vc * 2.0 * a.real * self.coupling_sum(m) + \
                p.hbar * p.wc * abs(a) ** 2
        return float(ez + ex + ea + self.dmi_energy(m) + ed + ec)

    # ----------------------------------------------------------- integrators
    def step_rk4(self, m, a, t, dt):
        k1m, k1a = self.rhs(m, a, t)
        k2m, k2a = self.rhs(m + 0.5 * dt * k1m, a + 0.5 * dt * k1a,
                            t + 0.5 * dt)
        k3m, k3a = self.rhs(m + 0.5 * dt * k2m, a + 0.5 * dt * k2a,
                            t + 0.5 * dt)
        k4m, k4a = self.rhs(m + dt * k3m, a + dt * k3a, t + dt)
        mn = m + dt / 6.0 * (k1m + 2 * k2m + 2 * k3m + k4m)
        an = a + dt / 6.0 * (k1a + 2 * k2a + 2 * k3a + k4a)
        return normalise(mn), an

    def dp45_attempt(self, m, a, t, h, k1m, k1a):
        """One Dormand-Prince attempt.  Returns (m5, a5, err, k7m, k7a) with
        m5 not yet renormalised and k7 = f(t+h, m5, a5) (FSAL)."""
        km = [k1m]
        ka = [k1a]
        for s in range(1, 7):
            ms_ = m + h * sum(DP_A[s][j] * km[j] for j in range(s)
                              if DP_A[s][j] != 0.0)
            as_ = a + h * sum(DP_A[s][j] * ka[j] for j in range(s))
            if s == 6:
                m5, a5 = ms_, as_
            dm, da = self.rhs(ms_, as_, t + DP_C[s] * h)
            km.append(dm)
            ka.append(da)
        e = DP_B5 - DP_B4
        errm_vec = h * sum(e[j] * km[j] for j in range(7) if e[j] != 0.0)
        errm = float(np.sqrt((errm_vec ** 2).sum(axis=0)).max())
        erra = self.anorm(h * sum(e[j] * ka[j] for j in range(7))) / max(
            1.0, self.anorm(a5))
        return m5, a5, max(errm, erra), km[6], ka[6]

    # ------------------------------------------------------------------ runs
    def record(self, t, m, a):
        """t, <m> over the magnetic cells, then Re and Im of each mode."""
        mm = m[:, self.inside].mean(axis=1)
        row = [t, mm[0], mm[1], mm[2]]
        for ak in np.atleast_1d(a):
            row += [ak.real, ak.imag]
        return row

    def run_rk4(self, m0, a0, dt, nsteps, record_every=0, t0=0.0):
        """Fixed-step RK4.  Records (t, <m>, Re a, Im a) for the initial state
        and after every `record_every`-th step."""
        m = np.asarray(m0, dtype=np.float64) * self.inside[None]
        a = self.amplitude(a0)
        t = t0
        rec = [self.record(t, m, a)] if record_every else []
        self._dt_noise = dt
        for n in range(1, nsteps + 1):
            m, a = self.step_rk4(m, a, t, dt)
            self.noise_step += 1
            t = t0 + n * dt
            if record_every and n % record_every == 0:
                rec.append(self.record(t, m, a))
        return m, a, t, np.array(rec)

    def run_rk4_memory(self, m0, a0, dt, nsteps, record_every=0):
        """Fixed-step RK4 of m with the cavity integrated out, as the paper
        does it (section "Adapting the memory term"): the cavity field
        B_rms Gamma_n is held over step n (t_n -> t_{n+1}, t_n = n dt, t_0 =
        0 at the reset), Gamma_n from the rectangle-rule recursion
        Eqs. (Sdiscrete), (Cdiscrete), (gammadiscretefinal) on the coupling
        sums F_n of the step-start states (S_0 = C_0 = 0):
          S_n = S_{n-1} + e^{kappa t_n} sin(wc t_n) F_n dt
          C_n = C_{n-1} + e^{kappa t_n} cos(wc t_n) F_n dt
          Gamma_n = e^{-kappa t_n} [cos(wc t_n) (x0 - 2 V_c S_n / hbar)
                                    - sin(wc t_n) (p0 - 2 V_c C_n / hbar)].
        The cavity has no drive here (the paper drives the magnet).  Records
        (t, <m>, Re a, Im a) use the amplitude the sums S_n, C_n give at
        t_{n+1}, a = e^{-(i wc + kappa) t} (a0 + i (V_c/hbar)(C_n + i S_n))
        (so that 2 Re a = Gamma before the term of F_{n+1} is added)."""
        p = self.p
        if p.cdrive_kind != DRIVE_NONE:
            raise ValueError("the memory form takes no cavity drive")
        if self.multi:
            raise ValueError("the memory form is written for one mode")
        m = np.asarray(m0, dtype=np.float64) * self.inside[None]
        a0 = complex(a0)
        x0, p0 = 2.0 * a0.real, -2.0 * a0.imag
        vh = self.vc / p.hbar
        S = C = 0.0

        def amp(t):
            return np.exp(-(1j * p.wc + p.kappa) * t) * (
                a0 + 1j * vh * (C + 1j * S))

        rec = [self.record(0.0, m, a0)] if record_every else []
        for n in range(nsteps):
            tn = n * dt
            if n > 0:
                S, C = memory_sums(p, S, C, tn, self.coupling_sum(m), dt)
            gam = memory_gamma_value(p, vh, S, C, tn, x0, p0)
            # the field B_rms (a + a*) with a = Gamma_n / 2 held fixed
            ah = 0.5 * gam

            def f(mm, tt):
                return self.torque(mm, self.effective_field(mm, ah, tt))

            k1 = f(m, tn)
            k2 = f(m + 0.5 * dt * k1, tn + 0.5 * dt)
            k3 = f(m + 0.5 * dt * k2, tn + 0.5 * dt)
            k4 = f(m + dt * k3, tn + dt)
            m = normalise(m + dt / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4))
            if record_every and (n + 1) % record_every == 0:
                rec.append(self.record((n + 1) * dt, m, amp((n + 1) * dt)))
        return m, amp(nsteps * dt), nsteps * dt, np.array(rec)

    def run_dp45(self, m0, a0, t_end, tol, dt0, record_every=0, t0=0.0,
                 dt_min=1e-20, dt_max=1e-10, max_attempts=10 ** 7):
        """Adaptive Dormand-Prince from t0 to t_end (last step truncated to
        land on t_end).  Returns m, a, t, records, accepted dt list, stats."""
        if getattr(self.p, "temperature", 0.0) > 0.0:
            raise ValueError("the thermal field needs fixed steps (RK4)")
        m = np.asarray(m0, dtype=np.float64) * self.inside[None]
        a = self.amplitude(a0)
        t = t0
        k1m, k1a = self.rhs(m, a, t)
        dt = dt0
        prev_rej = False
        rec = [self.record(t, m, a)] if record_every else []
        dts = []
        nacc = nrej = 0
        for _ in range(max_attempts):
            if t >= t_end:
                break
            h = min(dt, t_end - t)
            m5, a5, err, k7m, k7a = self.dp45_attempt(m, a, t, h, k1m, k1a)
            if not (math.isfinite(err) and np.isfinite(m5).all()):
                err = math.inf
            if err <= tol:
                fac = 5.0 if err == 0.0 else min(5.0, max(
                    0.2, 0.9 * (tol / err) ** 0.2))
                if prev_rej:
                    fac = min(fac, 1.0)
                t = t + h
                m = normalise(m5)
                a = a5
                k1m, k1a = k7m, k7a
                dts.append(h)
                nacc += 1
                prev_rej = False
                if record_every and nacc % record_every == 0:
                    rec.append(self.record(t, m, a))
            else:
                fac = 0.2 if not math.isfinite(err) else max(
                    0.2, 0.9 * (tol / err) ** 0.2)
                prev_rej = True
                nrej += 1
            dt = min(dt_max, h * fac)
            if dt < dt_min:
                raise FloatingPointError("time step underflow")
        return m, a, t, np.array(rec), np.array(dts), dict(accepted=nacc,
                                                           rejected=nrej)

    def relax(self, m0, torque_tol=0.0, max_steps=100000, block=8):
        """Energy minimisation by damped dynamics, the relax() the paper's
        example script calls before it runs (appendix "Micromagnetic
        simulations with Mumax3-cQED"; the relax of the Mumax3 reference):
        the precession term off, the cavity decoupled (no cavity field, the
        amplitude left as it is) and the drives off, Dormand-Prince 5(4)
        steps (tolerance and first step of the problem) in blocks of
        `block` accepted steps.  After each block the torque of the current
        state is taken: with a threshold `torque_tol` > 0 the relaxation
        stops once the largest |dm/dt| is below it; without one, once the
        mean of |dm/dt|^2 over the magnetic cells has not decreased since
        the previous block; in any case after `max_steps` accepted steps.
        Returns (m, stats)."""
        import dataclasses
        p = self.p
        q = dataclasses.replace(p, precession=0, brms=(0.0, 0.0, 0.0),
                                brms_map=None, modes=None,
                                cdrive_kind=DRIVE_NONE, fdrive_kind=DRIVE_NONE,
                                fdrive_map=None, cavity_mode=0)
        o = CavityLLG(q, demag=self.demag_mode or "auto")
        m = np.asarray(m0, dtype=np.float64) * self.inside[None]
        a, t = 0j, 0.0
        dt = p.dt
        tol = p.tol
        k1m, k1a = o.rhs(m, a, t)
        prev_rej = False
        nacc = nrej = nblk = 0
        prev = None
        mx = math.inf
        while True:
            nb = min(block, max_steps - nacc)
            if nb <= 0:
                break
            done = 0
            while done < nb:
                h = dt
                m5, a5, err, k7m, k7a = o.dp45_attempt(m, a, t, h, k1m, k1a)
                if not (math.isfinite(err) and np.isfinite(m5).all()):
                    err = math.inf
                if err <= tol:
                    fac = 5.0 if err == 0.0 else min(5.0, max(
                        0.2, 0.9 * (tol / err) ** 0.2))
                    if prev_rej:
                        fac = min(fac, 1.0)
                    t, m, a = t + h, normalise(m5), a5
                    k1m, k1a = k7m, k7a
                    nacc += 1
                    done += 1
                    prev_rej = False
                else:
                    fac = 0.2 if not math.isfinite(err) else max(
                        0.2, 0.9 * (tol / err) ** 0.2)
                    prev_rej = True
                    nrej += 1
                dt = min(p.dt_max, h * fac)
                if dt < p.dt_min:
                    raise FloatingPointError("time step underflow")
            nblk += 1
            tq, _ = o.rhs(m, a, t)
            n2 = (tq * tq).sum(axis=0)[self.inside]
            mean2, mx = float(n2.mean()), float(np.sqrt(n2.max()))
            if torque_tol > 0.0:
                if mx < torque_tol:
                    break
            elif prev is not None and mean2 >= prev:
                break
            prev = mean2
        return m, dict(accepted=nacc, rejected=nrej, blocks=nblk,
                       max_torque=mx)

    def run_dp45_replay(self, m0, a0, dts, t0=0.0):
        """Dormand-Prince with a prescribed sequence of accepted step sizes
        (every step accepted, FSAL and renormalisation as in run_dp45)."""
        m = np.asarray(m0, dtype=np.float64) * self.inside[None]
        a = self.amplitude(a0)
        t = t0
        k1m, k1a = self.rhs(m, a, t)
        for h in dts:
            m5, a5, err, k1m, k1a = self.dp45_attempt(m, a, t, h, k1m, k1a)
            t += h
            m = normalise(m5)
            a = a5
        return m, a, t


# ---------------------------------------------------------------------------
# Integrated-out cavity (the paper's memory-kernel form), for cross-checks.
# ---------------------------------------------------------------------------
def memory_gamma(ts, Fs, prob, a0):
    """Gamma(t_n) of Eq. (gammafinal) by the trapezoid rule on samples
    F(t_k) = sum_i Ms_i m_i(t_k).B_rms, for every sample time t_n:
      Gamma(t) = 2 e^{-kappa t} Re(a0 e^{-i wc t})
                 - (2 V_c/hbar) int_0^t e^{kappa (tau-t)} sin(wc (tau-t)) F dtau
    """
    vc = prob.dx * prob.dy * prob.dz
    out = np.empty(len(ts))
    for n, t in enumerate(ts):
        tau = ts[: n + 1]
        integrand = np.exp(prob.kappa * (tau - t)) * np.sin(
            prob.wc * (tau - t)) * Fs[: n + 1]
        integral = np.trapezoid(integrand, tau) if n > 0 else 0.0
        out[n] = (2.0 * math.exp(-prob.kappa * t)
                  * (a0 * np.exp(-1j * prob.wc * t)).real
                  - 2.0 * vc / prob.hbar * integral)
    return out


def alpha_a_posteriori(ts, Fs, prob, a0):
    """alpha(t) recovered from the magnetisation history (trapezoid rule):
      alpha = a0 e^{-(kappa + i wc) t}
              + i (V_c/hbar) int_0^t e^{(kappa + i wc)(tau - t)} F dtau ."""
    vc = prob.dx * prob.dy * prob.dz
    out = np.empty(len(ts), dtype=complex)
    for n, t in enumerate(ts):
        tau = ts[: n + 1]
        integrand = np.exp((prob.kappa + 1j * prob.wc) * (tau - t)) * Fs[
            : n + 1]
        integral = np.trapezoid(integrand, tau) if n > 0 else 0.0
        out[n] = a0 * np.exp(-(prob.kappa + 1j * prob.wc) * t) + \
            1j * vc / prob.hbar * integral
    return out


def memory_sums(prob, S, C, t, F, dt):
    """One rectangle-rule term of Eqs. (Sdiscrete), (Cdiscrete):
    S += e^{kappa t} sin(wc t) F dt, C += e^{kappa t} cos(wc t) F dt."""
    e = math.exp(prob.kappa * t)
    return (S + e * math.sin(prob.wc * t) * F * dt,
            C + e * math.cos(prob.wc * t) * F * dt)


def memory_gamma_value(prob, vh, S, C, t, x0, p0):
    """Eq. (gammadiscretefinal) with vh = V_c / hbar:
    Gamma = e^{-kappa t} [cos(wc t)(x0 - 2 vh S) - sin(wc t)(p0 - 2 vh C)]."""
    ek = math.exp(-prob.kappa * t)
    return ek * (math.cos(prob.wc * t) * (x0 - 2.0 * vh * S)
                 - math.sin(prob.wc * t) * (p0 - 2.0 * vh * C))


def memory_gamma_recursive(ts, Fs, prob, x0, p0):
    """The paper's O(1)-per-step recursion, Eqs. (Sdiscrete), (Cdiscrete) and
    (gammadiscretefinal), on uniformly spaced samples t_n = n dt:
      S_n = S_{n-1} + e^{kappa t_n} sin(wc t_n) F_n dt ,  S_0 = C_0 = 0
      C_n = C_{n-1} + e^{kappa t_n} cos(wc t_n) F_n dt
      Gamma_n = e^{-kappa t_n} cos(wc t_n) (x0 - 2 V_c S_n / hbar)
              - e^{-kappa t_n} sin(wc t_n) (p0 - 2 V_c C_n / hbar)."""
    vc = prob.dx * prob.dy * prob.dz
    dt = ts[1] - ts[0]
    S = C = 0.0
    out = np.empty(len(ts))
    for n, t in enumerate(ts):
        if n > 0:
            S += math.exp(prob.kappa * t) * math.sin(prob.wc * t) * Fs[n] * dt
            C += math.exp(prob.kappa * t) * math.cos(prob.wc * t) * Fs[n] * dt
        ek = math.exp(-prob.kappa * t)
        out[n] = (ek * math.cos(prob.wc * t) * (x0 - 2 * vc * S / prob.hbar)
                  - ek * math.sin(prob.wc * t) * (p0 - 2 * vc * C / prob.hbar))
    return out
