"""Pins of the oracle's memory-form integrator (run_rk4_memory: the paper's
integrated-out cavity with the rectangle-rule recursion of section
"Adapting the memory term"), CPU only.

  * Without coupling (B_rms = 0) the recorded amplitude is the free cavity
    a0 e^{-(i wc + kappa) t} (closed form) and m follows the ODE-form run
    exactly (the cavity cannot act on it).
  * With coupling, the scheme is first order in dt: against a converged
    ODE-form run (the joint (m, alpha) system, RK4 at a small step), the
    error halves when dt halves.  A wrong sign, a swapped sin/cos or a
    dropped e^{kappa t} factor in the recursion leaves an O(1) error that
    does not shrink with dt.
"""
import math

import numpy as np
import pytest

from oracle.llg import CavityLLG
from paper_2410_00966_amd import inputs as I


def _cell(brms_scale=1.0):
    p = I.Problem(nx=1, ny=1, nz=1, dx=5e-9, dy=5e-9, dz=5e-9, ms=8e5,
                  aex=0.0, alpha=0.0, bext=(0.0, 0.0, 0.1),
                  enable_demag=True)
    p.wc = p.gamma * 0.1                      # resonant with the cell
    p.kappa = 0.05 * p.wc
    g = 0.05 * p.wc
    p.brms = (brms_scale * I.brms_from_g(g, p.ms * p.vcell), 0.0, 0.0)
    m0 = I.normalise_rows(np.array([math.sin(0.2), 0.0, math.cos(0.2)])
                          .reshape(3, 1, 1, 1))
    return p, m0


def test_uncoupled_memory_form_is_the_free_cavity():
    p, m0 = _cell(brms_scale=0.0)
    a0 = 0.4 - 0.3j
    dt, n = 2e-13, 400
    o = CavityLLG(p)
    m, a, t, rec = o.run_rk4_memory(m0, a0, dt, n, record_every=50)
    ts = rec[:, 0]
    free = a0 * np.exp(-(1j * p.wc + p.kappa) * ts)
    got = rec[:, 4] + 1j * rec[:, 5]
    assert np.abs(got - free).max() <= 1e-12 * abs(a0)
    mo, _, _, _ = CavityLLG(p).run_rk4(m0, a0, dt, n)
    assert np.abs(m - mo).max() <= 1e-14


def test_coupled_memory_form_converges_at_first_order():
    p, m0 = _cell()
    T = 0.4e-9
    ref, _, _, _ = CavityLLG(p).run_rk4(m0, 0j, 4e-14, int(round(T / 4e-14)))
    errs = []
    for dt in (4e-13, 2e-13, 1e-13):
        m, _, _, _ = CavityLLG(p).run_rk4_memory(m0, 0j, dt,
                                                 int(round(T / dt)))
        errs.append(np.abs(m - ref).max())
    print("errors", errs)
    # the coupling matters at this size: the uncoupled cell is far off
    mu, _, _, _ = CavityLLG(_cell(0.0)[0]).run_rk4(m0, 0j, 4e-13,
                                                   int(round(T / 4e-13)))
    assert np.abs(mu - ref).max() > 20 * errs[-1]
    for e1, e2 in zip(errs, errs[1:]):
        assert 1.6 < e1 / e2 < 2.4
