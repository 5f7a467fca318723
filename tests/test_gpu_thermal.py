"""GPU tests of the thermal field (temperature, seed) against the FP64
oracle, whose generator is pinned to the Philox4x32-10 known-answer vectors
and whose field is pinned to Boltzmann equilibrium
(tests/test_oracle_thermal.py):

  * right-hand side element by element (both draw the same normals from
    the same counters);
  * an RK4 run of a film with exchange and demag, per cell, with the noise
    visibly at work; a run split in two equals the whole run bit for bit
    (the step counter carries over);
  * Boltzmann equilibrium of 16384 independent macrospins on the GPU: the
    Langevin average coth x - 1/x;
  * refusals: DP45, the adjoint.
"""
import math
import sys

import numpy as np
import pytest

from paper_2410_00966_amd import inputs as I

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.skip("no GPU")
    return _t


def _film(nx=24, ny=20, nz=2, T=300.0, seed=12345):
    p = I.Problem(nx=nx, ny=ny, nz=nz, dx=3e-9, dy=3e-9, dz=3e-9, ms=8e5,
                  aex=1.3e-11, alpha=0.1, ku1=2e4, anis_u=(0.0, 0.0, 1.0),
                  bext=(0.0, 0.0, 0.1), method=I.METHOD_RK4, dt=5e-14)
    p.temperature, p.seed = T, seed
    p.wc = 2 * math.pi * 10e9
    p.kappa = 1e-3 * p.wc
    p.brms = (I.brms_from_g(0.01 * p.wc, p.ms * p.ncells * p.vcell), 0.0,
              0.0)
    return p


@pytest.mark.parametrize("grid", [(37, 23, 3), (64, 40, 1)])
def test_rhs_with_thermal_field_matches_oracle(torch, grid):
    from oracle.llg import CavityLLG
    from paper_2410_00966_amd.llgc import Sim
    p = _film(*grid, seed=99 + sum(grid))
    rng = np.random.default_rng(sum(grid))
    m = rng.normal(size=(3,) + p.shape)
    m = (m / np.sqrt((m * m).sum(0))).astype(np.float32)
    o = CavityLLG(p)
    Bref = o.effective_field(m.astype(np.float64), 0.1j, 0.0)
    q = I.Problem(**{**p.__dict__})
    q.temperature = 0.0
    Bcold = CavityLLG(q).effective_field(m.astype(np.float64), 0.1j, 0.0)
    s = Sim(p)
    _, B, _ = s.eval_rhs(torch.from_numpy(m), 0.1j, 0.0)
    s.close()
    eB = np.abs(B.cpu().numpy() - Bref).max() / np.abs(Bref).max()
    noise = np.abs(Bref - Bcold).max()
    _say("thermal rhs", grid, "field err", eB, "noise scale", noise)
    assert eB < 2e-5
    assert noise > 0.05 * np.abs(Bref).max()


def test_rk4_with_thermal_field_matches_oracle_and_splits(torch):
    from oracle.llg import CavityLLG
    from paper_2410_00966_amd.llgc import Sim
    p = _film()
    m0 = I.tilted_uniform_state(p.shape, 5.0, 1e-3, seed=8101)
    n = 100
    mref, aref, _, _ = CavityLLG(p).run_rk4(m0.astype(np.float64), 0j,
                                            p.dt, n)
    q = I.Problem(**{**p.__dict__})
    q.temperature = 0.0
    mcold, _, _, _ = CavityLLG(q).run_rk4(m0.astype(np.float64), 0j, q.dt,
                                          n)
    s = Sim(p)
    s.set_state(torch.from_numpy(m0))
    s.run(nsteps=n)
    m, _, a = s.get_state()
    s.set_state(torch.from_numpy(m0))
    s.run(nsteps=40)
    s.run(nsteps=60)
    m2, _, a2 = s.get_state()
    s.close()
    dm = np.abs(m.cpu().numpy() - mref).max()
    _say("thermal rk4 max|dm|", dm, "thermal effect",
         np.abs(mref - mcold).max())
    assert dm <= 1e-4
    assert np.abs(mref - mcold).max() > 100 * dm
    assert torch.equal(m, m2) and a == a2


def test_boltzmann_equilibrium_on_gpu(torch):
    from paper_2410_00966_amd.llgc import Sim
    ms, T, b = 8e5, 300.0, 0.2
    v = 2.0 * I.KB * T / (ms * b)              # x = Ms V B/(kB T) = 2
    d = v ** (1.0 / 3.0)
    p = I.Problem(nx=128, ny=128, nz=1, dx=d, dy=d, dz=d, ms=ms, aex=0.0,
                  alpha=1.0, bext=(0.0, 0.0, b), enable_demag=False,
                  method=I.METHOD_RK4, dt=1e-13)
    p.temperature, p.seed = T, 2024
    m0 = np.zeros((3,) + p.shape, dtype=np.float32)
    m0[2] = 1.0
    s = Sim(p)
    s.set_state(torch.from_numpy(m0))
    s.run(nsteps=3000)                         # about 5 relaxation times
    rec, _ = s.run(nsteps=9000, record_every=20)
    s.close()
    mz = float(rec[1:, 3].mean())
    lang = 1.0 / math.tanh(2.0) - 0.5
    _say("gpu boltzmann <mz>", mz, "langevin", lang)
    assert mz == pytest.approx(lang, abs=0.006)


def test_thermal_refusals(torch):
    from paper_2410_00966_amd.llgc import LLGCError, Sim
    p = _film(64, 8, 1)
    q = I.Problem(**{**p.__dict__})
    q.method = I.METHOD_DP45
    with pytest.raises(LLGCError) as e:
        Sim(q)
    assert e.value.code == -7
    s = Sim(p)
    s.set_state(torch.from_numpy(I.tilted_uniform_state(p.shape, 5.0, 0.0,
                                                        seed=1)))
    with pytest.raises(LLGCError) as e:
        s.adjoint(4, p.dt, 2, 4)
    assert e.value.code == -7
    s.close()
