"""Pins of the oracle's per-cell B_rms (brms_map), CPU only.  The map path
reduces to pinned cases:
  * a map equal to the uniform vector everywhere gives the uniform run;
  * two cells without exchange or demag are independent magnets: with the
    map nonzero on cell 0 only, cell 0 and the cavity follow the single
    coupled cell, and cell 1 follows the single uncoupled cell, exactly.
A map applied at the wrong cell, a coupling sum over the wrong cells or a
permuted component breaks one of these.
"""
import math

import numpy as np

from oracle.llg import CavityLLG
from paper_2410_00966_amd import inputs as I


def _base(nx, ny, nz, demag=True, aex=1.3e-11):
    p = I.Problem(nx=nx, ny=ny, nz=nz, dx=5e-9, dy=5e-9, dz=5e-9, ms=8e5,
                  aex=aex, alpha=0.01, bext=(0.0, 0.0, 0.1),
                  enable_demag=demag, dt=2e-13)
    p.wc = p.gamma * 0.1
    p.kappa = 1e-3 * p.wc
    return p


def test_uniform_map_equals_uniform_vector():
    p = _base(6, 5, 2)
    b = np.array([3e-3, -1e-3, 5e-4])
    p.brms = tuple(b)
    m0 = I.tilted_uniform_state(p.shape, 10.0, 1e-3, seed=4001)
    ref = CavityLLG(p).run_rk4(m0, 0.1j, p.dt, 30)
    q = I.Problem(**{**p.__dict__})
    q.brms = (0.0, 0.0, 0.0)
    q.brms_map = b.reshape(3, 1, 1, 1) * np.ones((1,) + p.shape)
    got = CavityLLG(q).run_rk4(m0, 0.1j, p.dt, 30)
    assert np.abs(got[0] - ref[0]).max() <= 1e-15
    assert abs(got[1] - ref[1]) <= 1e-15 * max(1.0, abs(ref[1]))


def test_map_on_one_of_two_independent_cells():
    b = np.array([2e-3, 1e-3, 0.0])
    p = _base(2, 1, 1, demag=False, aex=0.0)
    p.brms_map = np.zeros((3,) + p.shape)
    p.brms_map[:, 0, 0, 0] = b
    m0 = np.zeros((3,) + p.shape)
    m0[:, 0, 0, 0] = [math.sin(0.2), 0.0, math.cos(0.2)]
    m0[:, 0, 0, 1] = [0.0, math.sin(0.3), math.cos(0.3)]
    n = 200
    m, a, _, _ = CavityLLG(p).run_rk4(m0, 0j, p.dt, n)
    one = _base(1, 1, 1, demag=False, aex=0.0)
    one.brms = tuple(b)
    m1, a1, _, _ = CavityLLG(one).run_rk4(m0[:, :, :, :1], 0j, p.dt, n)
    free = _base(1, 1, 1, demag=False, aex=0.0)
    m2, a2, _, _ = CavityLLG(free).run_rk4(m0[:, :, :, 1:], 0j, p.dt, n)
    assert abs(a) > 1e-3                       # the coupled cell pumps it
    assert np.abs(m[:, :, :, :1] - m1).max() <= 1e-14
    assert abs(a - a1) <= 1e-14 * abs(a1)
    assert np.abs(m[:, :, :, 1:] - m2).max() <= 1e-14
    assert a2 == 0j
