"""FP64 CPU oracle for gradients of a cavity observable (test infrastructure).

TEST INFRASTRUCTURE ONLY: only tests/ and the benchmark's CPU-baseline leg
may import this module.

The same discrete map as oracle.llg (fields, LL torque, cavity mode, classic
RK4 on (m, alpha), renormalisation after every step), restated with plain
PyTorch CPU float64 ops so that reverse-mode autograd gives the exact
gradient of the discrete loss

    L = (1/|W|) sum_{n in W} |alpha_n|^2 ,  W = step indices of the window,

with respect to the per-cell Ms map, the per-cell Ku map, the coupling
(|B_rms| along a fixed direction) and the cavity drive amplitude eps0.  The
forward values are pinned to oracle.llg and the gradients to central finite
differences of oracle.llg in the tests.  The demag tensor is taken from
oracle.demag (a constant of the problem).
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import demag as _demag

DRIVE_NONE, DRIVE_SINC, DRIVE_CW = 0, 1, 2


def _shape_fn(kind, w, t):
    if kind == DRIVE_NONE:
        return 0.0
    if kind == DRIVE_SINC:
        x = w * t
        return 1.0 if x == 0.0 else math.sin(x) / x
    return math.cos(w * t)


class TorchCavityLLG:
    """RK4 integration of the joint (m, alpha) system in torch float64."""

    def __init__(self, prob):
        self.p = prob
        self.shape = (prob.nz, prob.ny, prob.nx)
        self.vc = prob.dx * prob.dy * prob.dz
        self.u = torch.tensor(prob.anis_u, dtype=torch.float64)
        self.u = self.u / torch.linalg.norm(self.u)
        self.kf = None
        if prob.enable_demag:
            nf = _demag.tensor_full(prob.nx, prob.ny, prob.nz, prob.dx,
                                    prob.dy, prob.dz)
            self.kf = torch.from_numpy(_demag.demag_kernel_fft(nf,
                                                               self.shape))

    def _demag(self, M):
        if self.kf is None:
            return torch.zeros_like(M)
        nz, ny, nx = self.shape
        Pz, Py, Px = self.kf.shape[1:]
        Mp = torch.zeros((3, Pz, Py, Px), dtype=torch.float64)
        Mp[:, :nz, :ny, :nx] = M
        Mf = torch.fft.fftn(Mp, dim=(1, 2, 3))
        xx, yy, zz, xy, xz, yz = self.kf
        Bf = torch.stack([xx * Mf[0] + xy * Mf[1] + xz * Mf[2],
                          xy * Mf[0] + yy * Mf[1] + yz * Mf[2],
                          xz * Mf[0] + yz * Mf[1] + zz * Mf[2]])
        B = torch.fft.ifftn(Bf, dim=(1, 2, 3)).real
        return -self.p.mu0 * B[:, :nz, :ny, :nx]

    def _exchange(self, m, ms):
        p = self.p
        lap = torch.zeros_like(m)
        for axis, d in ((3, p.dx), (2, p.dy), (1, p.dz)):
            if m.shape[axis] < 2:
                continue
            diff = torch.diff(m, dim=axis) / (d * d)
            lo = [slice(None)] * 4
            hi = [slice(None)] * 4
            lo[axis] = slice(0, -1)
            hi[axis] = slice(1, None)
            pad_lo = torch.zeros_like(m)
            pad_lo[tuple(lo)] = diff
            pad_hi = torch.zeros_like(m)
            pad_hi[tuple(hi)] = diff
            lap = lap + pad_lo - pad_hi
        return 2.0 * p.aex / ms * lap

    def rhs(self, m, a_re, a_im, t, ms, ku, brms, eps0):
        """m: (3, nz, ny, nx); a = a_re + i a_im (0-d tensors)."""
        p = self.p
        bext = torch.tensor(p.bext, dtype=torch.float64)
        f = p.fdrive_amp * _shape_fn(p.fdrive_kind, p.fdrive_w, t)
        bext = bext + f * torch.tensor(p.fdrive_dir, dtype=torch.float64)
        B = bext.view(3, 1, 1, 1) + self._exchange(m, ms)
        um = torch.einsum("c,czyx->zyx", self.u, m)
        B = B + (2.0 * ku / ms * um).unsqueeze(0) * self.u.view(3, 1, 1, 1)
        B = B + self._demag(ms * m)
        B = B + brms.view(3, 1, 1, 1) * (2.0 * a_re)
        mxB = torch.cross(m, B, dim=0)
        dm = -p.gamma / (1.0 + p.alpha ** 2) * (
            mxB + p.alpha * torch.cross(m, mxB, dim=0))
        F = (ms * torch.einsum("c,czyx->zyx", brms, m)).sum()
        eps = eps0 * _shape_fn(p.cdrive_kind, p.cdrive_w, t)
        # d alpha/dt = -(i wc + kappa) alpha + i (V/hbar) F - i eps
        da_re = -p.kappa * a_re + p.wc * a_im
        da_im = -p.wc * a_re - p.kappa * a_im + self.vc / p.hbar * F - eps
        return dm, da_re, da_im

    def loss(self, m0, a0, dt, nsteps, window, ms, ku, brms, eps0):
        """RK4 from (m0, a0); returns (L, m_final, a_final).  `window` =
        (n0, n1): L averages |alpha_n|^2 over step endpoints n0 <= n <= n1."""
        m = torch.as_tensor(m0, dtype=torch.float64)
        a_re = torch.tensor(float(np.real(a0)), dtype=torch.float64)
        a_im = torch.tensor(float(np.imag(a0)), dtype=torch.float64)
        n0, n1 = window
        acc = torch.zeros((), dtype=torch.float64)
        for n in range(1, nsteps + 1):
            t = (n - 1) * dt
            k1 = self.rhs(m, a_re, a_im, t, ms, ku, brms, eps0)
            k2 = self.rhs(m + 0.5 * dt * k1[0], a_re + 0.5 * dt * k1[1],
                          a_im + 0.5 * dt * k1[2], t + 0.5 * dt, ms, ku,
                          brms, eps0)
            k3 = self.rhs(m + 0.5 * dt * k2[0], a_re + 0.5 * dt * k2[1],
                          a_im + 0.5 * dt * k2[2], t + 0.5 * dt, ms, ku,
                          brms, eps0)
            k4 = self.rhs(m + dt * k3[0], a_re + dt * k3[1],
                          a_im + dt * k3[2], t + dt, ms, ku, brms, eps0)
            mh = m + dt / 6.0 * (k1[0] + 2 * k2[0] + 2 * k3[0] + k4[0])
            a_re = a_re + dt / 6.0 * (k1[1] + 2 * k2[1] + 2 * k3[1] + k4[1])
            a_im = a_im + dt / 6.0 * (k1[2] + 2 * k2[2] + 2 * k3[2] + k4[2])
            m = mh / torch.sqrt((mh * mh).sum(dim=0, keepdim=True))
            if n0 <= n <= n1:
                acc = acc + a_re * a_re + a_im * a_im
        return acc / (n1 - n0 + 1), m, torch.complex(a_re, a_im)


def gradient(prob, m0, a0, dt, nsteps, window, brms_dir):
    """Loss and its gradient w.r.t. (Ms map, Ku map, |B_rms|, eps0).
    Returns dict(loss, g_ms (nz,ny,nx), g_ku, g_brms, g_eps0)."""
    o = TorchCavityLLG(prob)
    ms = torch.tensor(prob.ms_array(), dtype=torch.float64,
                      requires_grad=True)
    ku = torch.tensor(prob.ku_array(), dtype=torch.float64,
                      requires_grad=True)
    bdir = torch.tensor(brms_dir, dtype=torch.float64)
    bmag = torch.tensor(float(np.dot(np.asarray(prob.brms), brms_dir)),
                        dtype=torch.float64, requires_grad=True)
    eps0 = torch.tensor(float(prob.cdrive_amp), dtype=torch.float64,
                        requires_grad=True)
    L, _, _ = o.loss(m0, a0, dt, nsteps, window, ms, ku, bmag * bdir, eps0)
    L.backward()
    return dict(loss=float(L.detach()), g_ms=ms.grad.numpy().copy(),
                g_ku=ku.grad.numpy().copy(), g_brms=float(bmag.grad),
                g_eps0=float(eps0.grad))
