"""GPU tests of llgc_relax (damped-dynamics energy minimisation, the
script's relax()) against the oracle's relax, which is pinned to the
Stoner-Wohlfarth equilibria of a macrospin (tests/test_oracle_relax.py):

  * a macrospin in a tilted field relaxes to the bracketed root of
    Ku sin 2theta + Ms B sin(theta - psi) = 0;
  * a textured film with demag, anisotropy and DMI: the GPU's relaxed state
    against the oracle's, both stopped by the same torque threshold, per
    cell; t, the cavity amplitude and the parameters are untouched (a run
    after the relax equals a run of a fresh context from the relaxed m);
  * a coupled multimode cavity is decoupled during the relax and restored.
"""
import math
import sys

import numpy as np
import pytest
from scipy.optimize import brentq

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


def test_macrospin_relaxes_to_stoner_wohlfarth(torch):
    from paper_2410_00966_amd.llgc import Sim
    ku, ms, b, psi = 3e4, 8e5, 0.05, math.radians(68.2)
    p = I.Problem(nx=1, ny=1, nz=1, dx=5e-9, dy=5e-9, dz=5e-9, ms=ms,
                  ku1=ku, anis_u=(0, 0, 1), alpha=0.5,
                  bext=(b * math.sin(psi), 0.0, b * math.cos(psi)),
                  enable_demag=False, dt=1e-13, tol=1e-7,
                  method=I.METHOD_DP45)
    th0 = math.radians(10.0)
    m0 = np.array([math.sin(th0), 0.0, math.cos(th0)],
                  dtype=np.float32).reshape(3, 1, 1, 1)
    s = Sim(p)
    s.set_state(torch.from_numpy(m0), 1e-12, 0.1j)
    st = s.relax(torque_tol=1e3)
    m, t, a = s.get_state()
    s.close()
    m = m.cpu().numpy().astype(np.float64).ravel()
    th = math.atan2(m[0], m[2])
    ref = brentq(lambda x: ku * math.sin(2 * x) + ms * b * math.sin(x - psi),
                 0.3, 0.8)
    _say("macrospin relax", st, "theta", th, "ref", ref)
    assert st["max_torque"] < 1e3
    assert th == pytest.approx(ref, abs=2e-6)
    assert t == 1e-12 and a == 0.1j


def _film(method=I.METHOD_RK4):
    p = I.Problem(nx=24, ny=20, nz=2, dx=4e-9, dy=4e-9, dz=4e-9, ms=8e5,
                  aex=1.3e-11, alpha=0.5, ku1=2e4, anis_u=(0.0, 0.6, 0.8),
                  bext=(0.02, 0.0, 0.0), method=method, dt=1e-13, tol=1e-6)
    p.dmi_int = 1e-3
    p.wc = 2 * math.pi * 8e9
    p.kappa = 1e-3 * p.wc
    p.brms = (0.0, I.brms_from_g(0.02 * p.wc, p.ms * p.ncells * p.vcell),
              0.0)
    m0 = I.film_texture(p.nx, p.ny, p.nz, p.dx, p.dy, 3, 8e-9, seed=7301)
    return p, m0


def test_film_relax_matches_oracle_and_restores(torch):
    from oracle.llg import CavityLLG
    from paper_2410_00966_amd.llgc import Sim
    p, m0 = _film()
    tt = 1e9      # rad/s: both stop once the largest torque is below it
    mref, so = CavityLLG(p).relax(m0.astype(np.float64), torque_tol=tt,
                                  max_steps=6000)
    s = Sim(p)
    s.set_state(torch.from_numpy(m0), 2e-12, 0.3 - 0.1j)
    st = s.relax(torque_tol=tt, max_steps=6000)
    m, t, a = s.get_state()
    dm = np.abs(m.cpu().numpy() - mref).max()
    _say("film relax gpu", st, "oracle", so, "max|dm|", dm)
    assert st["max_torque"] < tt and so["max_torque"] < tt
    assert dm <= 2e-3
    assert t == 2e-12 and a == 0.3 - 0.1j
    # parameters restored: an RK4 run now equals a fresh context's run
    # from the relaxed state
    s.run(nsteps=50)
    m1, _, a1 = s.get_state()
    s.close()
    r = Sim(p)
    r.set_state(m, 2e-12, 0.3 - 0.1j)
    r.run(nsteps=50)
    m2, _, a2 = r.get_state()
    r.close()
    assert torch.equal(m1, m2) and a1 == a2


def test_relax_decouples_modes_and_restores_them(torch):
    from paper_2410_00966_amd.llgc import Sim
    p, m0 = _film(method=I.METHOD_DP45)
    b = p.brms[1]
    q = I.Problem(**{**p.__dict__})
    q.modes = [I.Mode(brms=(0.0, b, 0.0), wc=p.wc, kappa=p.kappa),
               I.Mode(brms=(0.0, 0.0, 0.5 * b), wc=1.2 * p.wc,
                      kappa=p.kappa)]
    out = []
    for prob in (p, q):
        s = Sim(prob)
        s.set_state(torch.from_numpy(m0), 0.0,
                    [0.2j, -0.1] if prob is q else 0.2j)
        s.relax(max_steps=64)
        m, t, a = s.get_state()
        out.append(m)
        if prob is q:
            assert np.allclose(a, [0.2j, -0.1], rtol=0, atol=0)
            rec, _ = s.run(t_end=1e-12, record_every=1, rec_cap=400)
            assert rec.shape[1] == 8
        s.close()
    # the cavity does not act during the relax: same relaxed m
    assert torch.equal(out[0], out[1])
