"""GPU tests of the Dzyaloshinskii-Moriya field (dmi_int, dmi_bulk) against
the FP64 oracle, whose DMI is pinned to its energy gradient, to the
continuum closed forms at second order and to energy conservation
(tests/test_oracle_dmi.py): right-hand side element by element on ragged
grids with empty cells, an RK4 run and a DP45 run per cell, a batch
against standalone solves bit for bit, and the refusal in the adjoint."""
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


def _problem(nx, ny, nz, di, db, method=I.METHOD_RK4, hole=False):
    p = I.Problem(nx=nx, ny=ny, nz=nz, dx=3e-9, dy=4e-9, dz=2e-9, ms=8e5,
                  aex=1.3e-11, alpha=0.05, ku1=5e4, anis_u=(0.0, 0.0, 1.0),
                  bext=(0.0, 0.0, 0.1), method=method, dt=5e-14, tol=1e-6)
    p.dmi_int, p.dmi_bulk = di, db
    p.wc = 2 * math.pi * 10e9
    p.kappa = 1e-3 * p.wc
    p.brms = (I.brms_from_g(0.01 * p.wc, p.ms * p.ncells * p.vcell), 0.0,
              0.0)
    if hole:
        ms = np.full(p.shape, 8e5, dtype=np.float32)
        ms[:, ny // 3: ny // 3 + 3, nx // 2: nx // 2 + 4] = 0.0
        p.ms_map = ms
    return p


@pytest.mark.parametrize("grid,di,db,hole", [
    ((37, 23, 3), 3e-3, 0.0, False),
    ((64, 40, 1), 0.0, 2e-3, True),
    ((20, 33, 4), 1.5e-3, -1e-3, True),
])
def test_rhs_with_dmi_matches_oracle(torch, grid, di, db, hole):
    from oracle.llg import CavityLLG
    from paper_2410_00966_amd.llgc import Sim
    p = _problem(*grid, di, db, hole=hole)
    rng = np.random.default_rng(sum(grid))
    m = rng.normal(size=(3,) + p.shape)
    m = (m / np.sqrt((m * m).sum(0))).astype(np.float32)
    o = CavityLLG(p)
    m = (m * o.inside[None]).astype(np.float32)
    a, t = 0.3 - 0.2j, 1e-12
    Bref = o.effective_field(m.astype(np.float64), a, t)
    dref, daref = o.rhs(m.astype(np.float64), a, t)
    s = Sim(p)
    dm, B, da = s.eval_rhs(torch.from_numpy(m), a, t)
    s.close()
    eB = np.abs(B.cpu().numpy() - Bref).max() / np.abs(Bref).max()
    ed = np.abs(dm.cpu().numpy() - dref).max() / np.abs(dref).max()
    _say("dmi rhs", grid, di, db, "field", eB, "torque", ed)
    assert eB < 2e-5 and ed < 2e-5
    assert abs(da - daref) <= 1e-9 * abs(daref)


def test_rk4_run_with_dmi_matches_oracle(torch):
    from oracle.llg import CavityLLG
    from paper_2410_00966_amd.llgc import Sim
    p = _problem(24, 20, 2, 3e-3, 5e-4)
    m0 = I.tilted_uniform_state(p.shape, 15.0, 1e-2, seed=7101)
    n, every = 300, 30
    mref, aref, _, recref = CavityLLG(p).run_rk4(m0.astype(np.float64), 0j,
                                                 p.dt, n, every)
    s = Sim(p)
    s.set_state(torch.from_numpy(m0))
    rec, _ = s.run(nsteps=n, record_every=every)
    m, _, a = s.get_state()
    s.close()
    dm = np.abs(m.cpu().numpy() - mref).max()
    _say("dmi rk4 max|dm|", dm, "a", a, aref)
    assert dm <= 1e-4
    assert abs(a - aref) <= 1e-5 * abs(aref)
    assert np.abs(rec[:, 1:4] - recref[:, 1:4]).max() <= 1e-4
    # DMI changed the trajectory: the run without it differs
    q = _problem(24, 20, 2, 0.0, 0.0)
    mq, _, _, _ = CavityLLG(q).run_rk4(m0.astype(np.float64), 0j, q.dt, n)
    assert np.abs(mq - mref).max() > 100 * dm


def test_dp45_run_with_dmi_matches_oracle(torch):
    from oracle.llg import CavityLLG
    from paper_2410_00966_amd.llgc import Sim
    p = _problem(20, 16, 2, 2e-3, 0.0, method=I.METHOD_DP45, hole=True)
    p.dt = 1e-14
    m0 = I.tilted_uniform_state(p.shape, 15.0, 1e-2, seed=7102)
    T = 15e-12
    mref, aref, tref, _, _, st = CavityLLG(p).run_dp45(
        m0.astype(np.float64), 0j, T, p.tol, p.dt)
    s = Sim(p)
    s.set_state(torch.from_numpy(m0))
    _, info = s.run(t_end=T)
    m, t, a = s.get_state()
    s.close()
    dm = np.abs(m.cpu().numpy() - mref).max()
    _say("dmi dp45", info["accepted"], st["accepted"], "max|dm|", dm)
    assert t == pytest.approx(tref, rel=1e-12)
    assert abs(info["accepted"] - st["accepted"]) <= max(
        1, 0.02 * st["accepted"])
    assert dm <= 1e-4


def test_batch_with_dmi_equals_standalone(torch):
    from paper_2410_00966_amd.llgc import Batch, Sim
    probs, m0s = [], []
    for k, (sh, di, db) in enumerate([((24, 20, 2), 3e-3, 0.0),
                                      ((40, 16, 1), 0.0, 0.0),
                                      ((17, 33, 3), 0.0, 2e-3)]):
        p = _problem(*sh, di, db, method=I.METHOD_DP45)
        p.dt = 1e-14
        probs.append(p)
        m0s.append(I.tilted_uniform_state(p.shape, 10.0, 1e-2, seed=7200 + k))
    T = 8e-12
    b = Batch(probs)
    for s, m0 in zip(b.sims, m0s):
        s.set_state(torch.from_numpy(m0))
    recs, infos, st = b.run(t_end=T, record_every=4, rec_cap=200)
    outs = [s.get_state() for s in b.sims]
    b.close()
    assert (st == 0).all()
    for k, p in enumerate(probs):
        s = Sim(p, batch_plan=True)
        s.set_state(torch.from_numpy(m0s[k]))
        rec, info = s.run(t_end=T, record_every=4, rec_cap=200)
        m, t, a = s.get_state()
        s.close()
        assert infos[k]["accepted"] == info["accepted"]
        assert torch.equal(outs[k][0], m) and outs[k][2] == a
        assert np.array_equal(recs[k], rec)


def test_adjoint_refuses_dmi(torch):
    from paper_2410_00966_amd.llgc import LLGCError, Sim
    p = _problem(64, 8, 1, 1e-3, 0.0)
    s = Sim(p)
    s.set_state(torch.from_numpy(I.tilted_uniform_state(p.shape, 5.0, 0.0,
                                                        seed=1)))
    with pytest.raises(LLGCError) as e:
        s.adjoint(4, p.dt, 2, 4)
    assert e.value.code == -7
    s.close()
