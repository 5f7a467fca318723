"""Pins of the oracle's second-order uniaxial anisotropy (Ku2) and of the
precession switch (relaxation dynamics), CPU only.
  * Ku2: small-angle precession about the easy axis along the field at
    omega = gamma (B + (2 Ku1 + 4 Ku2)/Ms)/(1 + a^2), decay a omega (the
    energy density -Ku1 cos^2 - Ku2 cos^4 has stiffness 2 Ku1 + 4 Ku2).
  * Precession off: the linearisation about that equilibrium has two real
    eigenvalues, both -a omega0/(1 + a^2) (pure relaxation, no rotation),
    and the total energy of a textured grid decreases step after step.
"""
import os
import sys

import numpy as np
import pytest

from oracle.llg import CavityLLG
from paper_2410_00966_amd import inputs as I

sys.path.insert(0, os.path.dirname(__file__))
from test_oracle_llg import _jacobian_freqs  # noqa: E402


def _cell(alpha, ku2, precession=1):
    return I.Problem(nx=1, ny=1, nz=1, dx=5e-9, dy=5e-9, dz=5e-9, ms=8e5,
                     ku1=3e4, ku2=ku2, anis_u=(0, 0, 1), alpha=alpha,
                     bext=(0, 0, 0.2), enable_demag=False,
                     precession=precession)


def test_ku2_kittel_frequency_and_decay():
    alpha, ku2 = 0.05, 2e4
    ev = _jacobian_freqs(CavityLLG(_cell(alpha, ku2)), [0, 0, 1], 0j)
    w0 = I.GAMMA * (0.2 + (2 * 3e4 + 4 * ku2) / 8e5)
    mag = ev[np.argmax(np.abs(ev.imag))]
    assert abs(mag.imag) == pytest.approx(w0 / (1 + alpha ** 2), rel=1e-8)
    assert mag.real == pytest.approx(-alpha * w0 / (1 + alpha ** 2), rel=1e-6)


def test_no_precession_relaxes_without_rotation():
    alpha, ku2 = 0.3, 1e4
    ev = _jacobian_freqs(CavityLLG(_cell(alpha, ku2, precession=0)),
                         [0, 0, 1], 0j)
    w0 = I.GAMMA * (0.2 + (2 * 3e4 + 4 * ku2) / 8e5)
    mm = ev[np.argsort(ev.real)][:2]           # the two magnetic modes
    assert np.abs(mm.imag).max() <= 1e-6 * w0
    for e in mm:
        assert e.real == pytest.approx(-alpha * w0 / (1 + alpha ** 2),
                                       rel=1e-6)


def test_no_precession_energy_decreases():
    p = I.Problem(nx=12, ny=10, nz=2, dx=4e-9, dy=4e-9, dz=4e-9, ms=8e5,
                  aex=1.3e-11, alpha=0.5, ku1=2e4, ku2=5e3,
                  anis_u=(0.0, 0.6, 0.8), bext=(0.02, 0.0, 0.0),
                  precession=0, dt=2e-13)
    m = I.film_texture(p.nx, p.ny, p.nz, p.dx, p.dy, 3, 8e-9,
                       seed=6001).astype(np.float64)
    o = CavityLLG(p)
    e = [o.energy(m, 0j)]
    for n in range(60):
        m, _ = o.step_rk4(m, 0j, n * p.dt, p.dt)
        e.append(o.energy(m, 0j))
    e = np.array(e)
    assert (np.diff(e) <= 1e-12 * abs(e[0])).all()
    assert e[-1] < e[0] - 1e-3 * abs(e[0])
