"""GPU tests of the second-order uniaxial anisotropy (Ku2) and the
precession switch against the FP64 oracle (pinned to the Ku2 Kittel
frequency, pure-relaxation eigenvalues and monotone energy): right-hand
side element by element (2e-5), fixed-step relaxation run per cell (1e-4),
and the adjoint's refusal."""
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


def _problem(nx, ny, nz, precession):
    p = I.Problem(nx=nx, ny=ny, nz=nz, dx=4e-9, dy=4e-9, dz=4e-9, ms=8e5,
                  aex=1.3e-11, alpha=0.3, ku1=2e4, ku2=8e3,
                  anis_u=(0.0, 0.6, 0.8), bext=(0.02, 0.0, 0.01),
                  precession=precession, dt=1e-13)
    p.wc = 2 * math.pi * 8e9
    p.kappa = 1e-3 * p.wc
    p.brms = (1e-3, 0.0, 5e-4)
    p.ku1_map = I.smooth_map(nx, ny, nz, 1e4, 3e4, 3, 2, seed=nx + ny)
    return p


@pytest.mark.parametrize("grid,prec", [((37, 23, 3), 1), ((37, 23, 3), 0),
                                       ((64, 40, 1), 0)])
def test_rhs_matches_oracle(torch, grid, prec):
    from oracle.llg import CavityLLG
    from paper_2410_00966_amd.llgc import Sim
    p = _problem(*grid, prec)
    rng = np.random.default_rng(sum(grid) + prec)
    m = rng.normal(size=(3,) + p.shape)
    m = (m / np.sqrt((m * m).sum(0))).astype(np.float32)
    a, t = 0.4 + 0.2j, 2e-12
    o = CavityLLG(p)
    Bref = o.effective_field(m.astype(np.float64), a, t)
    dref, _ = o.rhs(m.astype(np.float64), a, t)
    s = Sim(p)
    dm, B, _ = s.eval_rhs(torch.from_numpy(m), a, t)
    s.close()
    eB = np.abs(B.cpu().numpy() - Bref).max() / np.abs(Bref).max()
    ed = np.abs(dm.cpu().numpy() - dref).max() / np.abs(dref).max()
    _say("ku2/prec rhs", grid, prec, "field err", eB, "torque err", ed)
    assert eB < 2e-5 and ed < 2e-5


def test_relaxation_run_matches_oracle(torch):
    from oracle.llg import CavityLLG
    from paper_2410_00966_amd.llgc import Sim
    p = _problem(24, 20, 2, 0)
    m0 = I.film_texture(p.nx, p.ny, p.nz, p.dx, p.dy, 4, 8e-9, seed=6101)
    n = 150
    mref, _, _, _ = CavityLLG(p).run_rk4(m0.astype(np.float64), 0j, p.dt, n)
    s = Sim(p)
    s.set_state(torch.from_numpy(m0))
    s.run(nsteps=n)
    m, _, _ = s.get_state()
    dm = np.abs(m.cpu().numpy() - mref).max()
    _say("relaxation max|dm|", dm)
    assert dm <= 1e-4
    from paper_2410_00966_amd.llgc import LLGCError
    with pytest.raises(LLGCError) as e:
        s.adjoint(4, p.dt, 2, 4)
    assert e.value.code == -7
    s.close()
