"""GPU tests of the plan autotuner (llgc_autotune).

The tuner only chooses which passes keep their FFTs in registers; the
results must still meet the oracle parity bar of the untuned plan
(right-hand side to 2e-5 of the largest magnitude, fixed-step runs to 1e-4
per cell), the recorded choice must be reused for the same grid shape, and a
batch-plan instance must refuse tuning.
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


def _problem(nx, ny, nz):
    p = I.Problem(nx=nx, ny=ny, nz=nz, dx=4e-9, dy=4e-9, dz=4e-9, ms=8e5,
                  aex=1.3e-11, alpha=0.02, ku1=4e4, anis_u=(0.6, 0.0, 0.8),
                  bext=(0.01, 0.03, 0.1), method=I.METHOD_RK4, dt=5e-14)
    p.wc = 2 * math.pi * 9e9
    p.kappa = 1e-3 * p.wc
    p.brms = (2e-3, -1e-3, 5e-4)
    p.cdrive_kind, p.cdrive_amp, p.cdrive_w = I.DRIVE_CW, 3e7, 5e10
    return p


def _random_m(shape, seed):
    rng = np.random.default_rng(seed)
    m = rng.normal(size=(3,) + shape)
    return (m / np.sqrt((m * m).sum(0))).astype(np.float32)


# padded lengths 64..1024 along both axes, so that every plan kind is a
# candidate somewhere
GRIDS = [(40, 33, 2), (100, 70, 1), (33, 300, 3), (300, 40, 4)]


@pytest.mark.parametrize("grid", GRIDS)
def test_tuned_plan_meets_oracle(torch, grid):
    from oracle.llg import CavityLLG
    from paper_2410_00966_amd.llgc import Sim
    p = _problem(*grid)
    m = _random_m(p.shape, seed=sum(grid))
    s = Sim(p)
    s.set_state(torch.from_numpy(m))
    kind = s.autotune(reps=5)
    _say("grid", grid, "tuned kind", kind)
    assert 0 <= kind < 16
    o = CavityLLG(p)
    a, t = 0.3 - 0.1j, 1e-12
    dm_ref, da_ref = o.rhs(m.astype(np.float64), a, t)
    dm, _, da = s.eval_rhs(torch.from_numpy(m), a, t)
    err = np.abs(dm.cpu().numpy() - dm_ref).max() / np.abs(dm_ref).max()
    _say("  rhs rel err", err)
    assert err < 2e-5
    assert abs(da - da_ref) <= 1e-9 * abs(da_ref)
    # a second context of the same shape reuses the recorded kind
    s2 = Sim(p)
    assert s2.autotune(reps=0) == kind
    s2.close()
    # fixed-step run under the tuned plan against the oracle
    n = 40
    m0 = I.tilted_uniform_state(p.shape, 10.0, 0.02, seed=sum(grid))
    s.set_state(torch.from_numpy(m0), 0.0, 0j)
    s.run(nsteps=n)
    mg, _, _ = s.get_state()
    mref, _, _, _ = o.run_rk4(m0.astype(np.float64), 0j, p.dt, n)
    dmax = np.abs(mg.cpu().numpy() - mref).max()
    _say("  rk4 max|dm|", dmax)
    assert dmax <= 1e-4
    s.close()


def test_batch_plan_refuses_tuning(torch):
    from paper_2410_00966_amd.llgc import Sim, LLGCError
    p = _problem(32, 32, 1)
    s = Sim(p, batch_plan=True)
    with pytest.raises(LLGCError) as e:
        s.autotune(reps=3)
    assert e.value.code == -1
    s.close()


@pytest.mark.parametrize("grid", [(41, 33, 2), (101, 70, 1), (301, 40, 4)])
def test_three_component_x_passes_meet_oracle(torch, grid):
    """Plan kind bit 3 forced at creation (LLGC_X3): RHS and an RK4 run
    against the oracle.  (Shapes no other test tunes: autotune(reps=0)
    would apply a recorded plan.)"""
    import os
    from oracle.llg import CavityLLG
    from paper_2410_00966_amd.llgc import Sim
    p = _problem(*grid)
    os.environ["LLGC_X3"] = "1"
    try:
        s = Sim(p)
    finally:
        os.environ.pop("LLGC_X3", None)
    assert s.autotune(reps=0) & 8
    m = _random_m(p.shape, seed=sum(grid) + 1)
    o = CavityLLG(p)
    a, t = 0.3 - 0.1j, 1e-12
    dm_ref, da_ref = o.rhs(m.astype(np.float64), a, t)
    dm, _, da = s.eval_rhs(torch.from_numpy(m), a, t)
    err = np.abs(dm.cpu().numpy() - dm_ref).max() / np.abs(dm_ref).max()
    _say("x3", grid, "rhs rel err", err)
    assert err < 2e-5
    assert abs(da - da_ref) <= 1e-9 * abs(da_ref)
    m0 = I.tilted_uniform_state(p.shape, 10.0, 0.02, seed=sum(grid))
    s.set_state(torch.from_numpy(m0), 0.0, 0j)
    s.run(nsteps=40)
    mg, _, _ = s.get_state()
    mref, _, _, _ = o.run_rk4(m0.astype(np.float64), 0j, p.dt, 40)
    assert np.abs(mg.cpu().numpy() - mref).max() <= 1e-4
    s.close()
