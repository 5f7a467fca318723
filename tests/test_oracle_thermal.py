"""Pins of the oracle's thermal field (Brown's fluctuating field, the last
effective-field term listed after Eq. (llg)) and of its counter-based
generator:

  * Philox4x32-10 reproduces the known-answer vectors published with the
    generator (Random123): zero counter and key, all-ones counter and key,
    and the pi-digit counter and key;
  * the Box-Muller normals of many counters have mean 0 and variance 1,
    and different steps or cells give uncorrelated values;
  * Boltzmann equilibrium: independent macrospins (no exchange, no demag)
    in a field B at temperature T settle at <m.b> = coth(x) - 1/x,
    x = Ms V B/(kB T) (the Langevin function), with alpha = 1 so that a
    noise variance off by the LL prefactor 1 + alpha^2 = 2 would show.
"""
import math

import numpy as np
import pytest

from oracle.llg import CavityLLG, philox4x32
from paper_2410_00966_amd import inputs as I


@pytest.mark.parametrize("ctr,key,out", [
    ((0, 0, 0, 0), (0, 0),
     (0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8)),
    ((0xffffffff,) * 4, (0xffffffff, 0xffffffff),
     (0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd)),
    ((0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344),
     (0xa4093822, 0x299f31d0),
     (0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1)),
])
def test_philox_known_answers(ctr, key, out):
    w = philox4x32(np.array(ctr, dtype=np.uint64).reshape(4, 1), key)
    assert tuple(int(x) for x in w.ravel()) == out


def _macrospins(n, T, b, alpha, seed=1):
    ms = 8e5
    v = 2.0 * I.KB * T / (ms * b)        # x = Ms V B / (kB T) = 2
    d = v ** (1.0 / 3.0)
    p = I.Problem(nx=n, ny=n, nz=1, dx=d, dy=d, dz=d, ms=ms, aex=0.0,
                  alpha=alpha, bext=(0.0, 0.0, b), enable_demag=False,
                  dt=1e-13)
    p.temperature, p.seed = T, seed
    return p


def test_normals_moments_and_independence():
    p = _macrospins(32, 300.0, 0.05, 1.0)
    o = CavityLLG(p)
    sig = math.sqrt(2 * p.alpha * I.KB * p.temperature
                    / (p.gamma * p.ms * o.vc * p.dt))
    samples = []
    for step in range(40):
        o.noise_step = step
        samples.append(o.thermal() / sig)
    x = np.stack(samples)                   # (steps, 3, 1, 32, 32)
    flat = x.ravel()
    n = flat.size
    assert abs(flat.mean()) < 5 / math.sqrt(n)
    assert abs(flat.var() - 1.0) < 5 * math.sqrt(2.0 / n)
    # consecutive steps and neighbouring cells uncorrelated
    c_step = (x[1:] * x[:-1]).mean()
    c_cell = (x[..., 1:] * x[..., :-1]).mean()
    assert abs(c_step) < 5 / math.sqrt(x[1:].size)
    assert abs(c_cell) < 5 / math.sqrt(x[..., 1:].size)


def test_boltzmann_equilibrium_langevin():
    """B = 0.2 T: relaxation time (1 + a^2)/(a gamma B) = 570 steps of
    0.1 ps; 3000 steps to equilibrate, 6000 averaged over 48 x 48 spins
    (standard error of the mean about 0.003)."""
    p = _macrospins(48, 300.0, 0.2, 1.0, seed=7)
    o = CavityLLG(p)
    m0 = np.zeros((3,) + p.shape)
    m0[2] = 1.0
    n_eq, n_avg, every = 3000, 6000, 20
    m, _, _, _ = o.run_rk4(m0, 0j, p.dt, n_eq)
    acc = []
    for _ in range(n_avg // every):
        m, _, _, _ = o.run_rk4(m, 0j, p.dt, every)
        acc.append(m[2].mean())
    mz = float(np.mean(acc))
    x = 2.0
    lang = 1.0 / math.tanh(x) - 1.0 / x
    assert mz == pytest.approx(lang, abs=0.012)
