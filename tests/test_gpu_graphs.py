"""GPU tests of the HIP-graph launch path.

Integrator runs replay captured graphs of their launch sequences (a chunk of
Dormand-Prince attempts, one RK4 step, one round of batched attempts).  A
graph holds the same kernels with the same arguments in the same order as
the direct launches, so every result must equal the direct path's bit for
bit: here the direct path is selected by LLGC_NO_GRAPHS at context creation.
Each run replays its graph many times, each replay feeding the next, and the
runs repeat with changed parameters so that stale graphs would show.
"""
import math
import os
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


def _problem(nx, ny, nz, method, seed):
    rng = np.random.default_rng(seed)
    p = I.Problem(nx=nx, ny=ny, nz=nz, dx=4e-9, dy=4e-9, dz=3e-9,
                  ms=float(rng.uniform(6e5, 9e5)), aex=1.3e-11,
                  alpha=0.02, ku1=2e4, anis_u=(0.6, 0.0, 0.8),
                  bext=(0.01, 0.02, 0.15), method=method, tol=1e-6,
                  dt=5e-14)
    p.wc = 2 * math.pi * 9e9
    p.kappa = 1e-3 * p.wc
    p.brms = (I.brms_from_g(0.02 * p.wc, p.ms * p.ncells * p.vcell), 0, 0)
    p.cdrive_kind, p.cdrive_amp, p.cdrive_w = I.DRIVE_CW, 1e7, p.wc
    m0 = I.tilted_uniform_state(p.shape, 10.0, 0.02, seed=seed)
    return p, m0


def _with_env(direct, fn):
    old = os.environ.pop("LLGC_NO_GRAPHS", None)
    if direct:
        os.environ["LLGC_NO_GRAPHS"] = "1"
    try:
        return fn()
    finally:
        os.environ.pop("LLGC_NO_GRAPHS", None)
        if old is not None:
            os.environ["LLGC_NO_GRAPHS"] = old


def _runs(torch, p, m0, direct, **run):
    """Two runs in a row, then a parameter change and a third run."""
    from paper_2410_00966_amd.llgc import Sim
    s = _with_env(direct, lambda: Sim(p))
    s.set_state(torch.from_numpy(m0), 0.0, 0.1 + 0.05j)
    out = []
    for k in range(3):
        if k == 2:
            q = I.Problem(**{**p.__dict__})
            q.bext = (0.0, 0.05, 0.2)
            s.set_params(q)
        rec, info = s.run(**run)
        m, t, a = s.get_state()
        out.append((m.cpu().numpy(), t, a, rec, info))
    s.close()
    return out


@pytest.mark.parametrize("method", [I.METHOD_DP45, I.METHOD_RK4])
def test_graph_runs_equal_direct_launches(torch, method):
    p, m0 = _problem(48, 40, 2, method, seed=5)
    run = (dict(nsteps=120, record_every=10, rec_cap=64)
           if method == I.METHOD_RK4 else
           dict(nsteps=60, t_end=1.0, record_every=7, rec_cap=64))
    _say("graphs vs direct,", "rk4" if method == I.METHOD_RK4 else "dp45")
    g = _runs(torch, p, m0, False, **run)
    d = _runs(torch, p, m0, True, **run)
    for k, ((mg, tg, ag, rg, ig), (md, td, ad, rd, idd)) in enumerate(zip(g, d)):
        _say(f"  run {k}: accepted {ig['accepted']}/{idd['accepted']} "
             f"max|dm| {np.abs(mg - md).max():.3e}")
        assert ig["accepted"] == idd["accepted"]
        assert ig["rejected"] == idd["rejected"]
        assert tg == td and ag == ad
        assert np.array_equal(mg, md)
        assert np.array_equal(rg, rd)


def test_batch_graph_equals_direct(torch):
    from paper_2410_00966_amd.llgc import Batch
    shapes = [(16, 16, 1), (40, 24, 2), (64, 20, 3), (24, 72, 4)]
    probs, m0s = [], []
    for k, sh in enumerate(shapes):
        p, m0 = _problem(*sh, method=I.METHOD_DP45, seed=40 + k)
        p.bext = (0.0, 0.0, 0.05 + 0.3 * k)      # different step counts
        probs.append(p)
        m0s.append(m0)

    def go(direct):
        b = _with_env(direct, lambda: Batch(probs))
        for s, m0 in zip(b.sims, m0s):
            s.set_state(torch.from_numpy(m0))
        recs, infos, st = b.run(t_end=12e-12, record_every=5, rec_cap=200)
        out = [s.get_state() for s in b.sims]
        b.close()
        return [(m.cpu().numpy(), t, a) for m, t, a in out], recs, infos, st

    _say("batch graphs vs direct")
    og, rg, ig, sg = go(False)
    od, rd, idd, sd = go(True)
    assert (sg == 0).all() and (sd == 0).all()
    for k in range(len(probs)):
        _say(f"  inst {k}: accepted {ig[k]['accepted']}/{idd[k]['accepted']}")
        assert ig[k]["accepted"] == idd[k]["accepted"]
        assert np.array_equal(og[k][0], od[k][0])
        assert og[k][1] == od[k][1] and og[k][2] == od[k][2]
        assert np.array_equal(rg[k], rd[k])


def test_plan_change_between_graph_runs(torch):
    """A run (graph captured), autotuning (plan may change), another run:
    equal to the same sequence with direct launches, where the second
    context takes the recorded kind for the shape (reps=0)."""
    from paper_2410_00966_amd.llgc import Sim
    p, m0 = _problem(100, 70, 2, I.METHOD_DP45, seed=9)

    def seq(direct, reps):
        s = _with_env(direct, lambda: Sim(p))
        s.set_state(torch.from_numpy(m0))
        s.run(nsteps=20, t_end=1.0)
        kind = s.autotune(reps=reps)
        rec, info = s.run(nsteps=40, t_end=1.0, record_every=4, rec_cap=32)
        m, t, a = s.get_state()
        s.close()
        return kind, m.cpu().numpy(), t, a, rec, info

    kg, mg, tg, ag, rg, ig = seq(False, 5)
    kd, md, td, ad, rd, idd = seq(True, 0)
    _say("  kinds", kg, kd, "accepted", ig["accepted"], idd["accepted"])
    assert kg == kd
    assert ig["accepted"] == idd["accepted"]
    assert tg == td and ag == ad
    assert np.array_equal(mg, md)
    assert np.array_equal(rg, rd)
