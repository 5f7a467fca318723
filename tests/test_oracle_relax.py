"""Pins of the oracle's relax (the damped-dynamics energy minimisation the
paper's example script calls before its run, appendix "Micromagnetic
simulations with Mumax3-cQED"):

  * a single macrospin with uniaxial anisotropy Ku along z in a field B at
    angle psi from z relaxes to the Stoner-Wohlfarth equilibrium: the root
    of dE/dtheta = Ku sin(2 theta) + Ms |B| sin(theta - psi) (found here by
    bracketing, independently of the dynamics) nearest the start;
  * on a textured film the total energy falls from block to block and the
    stop comes from the torque rule;
  * a state that is already relaxed stops within a few blocks (once the
    torque reaches rounding level), essentially unchanged;
  * the cavity is decoupled: a coupling B_rms changes nothing.
"""
import math

import numpy as np
import pytest
from scipy.optimize import brentq

from oracle.llg import CavityLLG
from paper_2410_00966_amd import inputs as I


def _macrospin(b, psi, ku=3e4, ms=8e5):
    return I.Problem(nx=1, ny=1, nz=1, dx=5e-9, dy=5e-9, dz=5e-9, ms=ms,
                     ku1=ku, anis_u=(0, 0, 1), alpha=0.5,
                     bext=(b * math.sin(psi), 0.0, b * math.cos(psi)),
                     enable_demag=False, dt=1e-13, tol=1e-7)


@pytest.mark.parametrize("b,psi_deg,theta0_deg", [(0.05, 68.2, 10.0),
                                                  (0.02, 120.0, 20.0),
                                                  (0.08, 30.0, 80.0)])
def test_stoner_wohlfarth_equilibrium(b, psi_deg, theta0_deg):
    ku, ms = 3e4, 8e5
    psi, th0 = math.radians(psi_deg), math.radians(theta0_deg)
    p = _macrospin(b, psi, ku, ms)
    m0 = np.array([math.sin(th0), 0.0, math.cos(th0)]).reshape(3, 1, 1, 1)
    m, st = CavityLLG(p).relax(m0, torque_tol=1e2)
    th = math.atan2(m[0].item(), m[2].item())

    def g(x):
        return ku * math.sin(2 * x) + ms * b * math.sin(x - psi)
    # equilibria in [0, pi]: the stable root the start flows to (energy
    # decreases along the path, so the nearest root in the downhill
    # direction)
    xs = np.linspace(0.0, math.pi, 2001)
    gs = np.array([g(x) for x in xs])
    roots = [brentq(g, xs[i], xs[i + 1]) for i in range(len(xs) - 1)
             if gs[i] * gs[i + 1] < 0]
    stable = [r for r in roots
              if 2 * ku * math.cos(2 * r) + ms * b * math.cos(r - psi) > 0]
    ref = min(stable, key=lambda r: abs(r - th))
    assert st["max_torque"] < 1e2
    assert abs(m[1].item()) < 1e-8
    assert th == pytest.approx(ref, abs=1e-6)
    # the start lies in that root's basin: no other stable root between
    lo, hi = sorted((th0, ref))
    assert not any(lo < r < hi for r in stable if r != ref)


def test_textured_film_energy_falls_by_block():
    p = I.Problem(nx=12, ny=10, nz=2, dx=4e-9, dy=4e-9, dz=4e-9, ms=8e5,
                  aex=1.3e-11, alpha=0.5, ku1=2e4, anis_u=(0.0, 0.6, 0.8),
                  bext=(0.02, 0.0, 0.0), dt=1e-13, tol=1e-6)
    m0 = I.film_texture(p.nx, p.ny, p.nz, p.dx, p.dy, 3, 8e-9,
                        seed=6002).astype(np.float64)
    o = CavityLLG(p)
    e = [o.energy(m0, 0j)]
    m = m0
    for _ in range(6):
        m, st = o.relax(m, max_steps=8)
        e.append(o.energy(m, 0j))
    assert (np.diff(e) < 0).all()
    m, st = o.relax(m, max_steps=20000)       # stagnation rule
    assert st["blocks"] >= 2
    assert o.energy(m, 0j) < e[-1]


def test_relaxed_state_stops_at_once():
    p = _macrospin(0.05, math.radians(40.0))
    o = CavityLLG(p)
    m0 = np.array([0.3, 0.0, 1.0]).reshape(3, 1, 1, 1)
    m1, _ = o.relax(m0 / np.linalg.norm(m0), torque_tol=1e-3,
                    max_steps=4000)
    m2, st = o.relax(m1)
    assert st["blocks"] <= 4
    assert np.abs(m2 - m1).max() < 1e-9


def test_cavity_is_decoupled_during_relax():
    p = _macrospin(0.05, math.radians(40.0))
    m0 = np.array([0.3, 0.1, 1.0]).reshape(3, 1, 1, 1)
    m0 = m0 / np.linalg.norm(m0)
    ma, _ = CavityLLG(p).relax(m0, max_steps=64)
    q = I.Problem(**{**p.__dict__})
    q.brms, q.wc, q.kappa = (3e-3, 0.0, 0.0), 2 * math.pi * 9e9, 1e6
    mb, _ = CavityLLG(q).relax(m0, max_steps=64)
    assert np.array_equal(ma, mb)
