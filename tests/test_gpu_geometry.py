"""GPU tests of geometry (cells with Ms = 0 in the Ms map are outside the
magnet) against the FP64 oracle, whose geometry handling is pinned by an
embedded block equal to the standalone block: fixed-step runs per cell on
an embedded block and on a disc, records, empty cells held at exactly 0, a
batch with a masked instance bit for bit against its standalone solve, and
the argument checks.
"""
import math
import os
import sys

import numpy as np
import pytest

from paper_2410_00966_amd import inputs as I

sys.path.insert(0, os.path.dirname(__file__))
import test_oracle_geometry as TG  # noqa: E402

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


def _run_both(torch, p, m0, n, every, a0=0j):
    from oracle.llg import CavityLLG
    from paper_2410_00966_amd.llgc import Sim
    mref, aref, _, recref = CavityLLG(p).run_rk4(m0.astype(np.float64), a0,
                                                 p.dt, n, every)
    s = Sim(p)
    s.set_state(torch.from_numpy(m0.astype(np.float32)), 0.0, a0)
    rec, _ = s.run(nsteps=n, record_every=every)
    m, _, a = s.get_state()
    s.close()
    return m.cpu().numpy(), a, rec, mref, aref, recref


def test_embedded_block_matches_oracle(torch):
    small, big, m0, mb, blk = TG._embedded()
    m, a, rec, mref, aref, recref = _run_both(torch, big, mb, 60, 10, 0.2j)
    outside = np.ones(big.shape, bool)
    outside[blk[1:]] = False
    dm = np.abs(m - mref).max()
    _say("embedded block max|dm|", dm, "a", a, aref)
    assert dm <= 1e-4
    assert np.abs(m[:, outside]).max() == 0.0
    assert np.abs(rec[:, 1:4] - recref[:, 1:4]).max() <= 1e-4
    assert abs(a - aref) <= 1e-3 * max(1.0, abs(aref))


def _disc(n=40):
    p = TG._prob(n, n, 1)
    yy, xx = np.mgrid[0:n, 0:n] + 0.5
    r = np.hypot(xx - n / 2, yy - n / 2)
    ms = np.where(r <= 0.45 * n, 8e5, 0.0)[None].astype(np.float32)
    p.ms_map = ms
    p.brms = (I.brms_from_g(0.05 * p.wc, float(ms.sum()) * p.vcell), 0, 0)
    m0 = I.tilted_uniform_state(p.shape, 10.0, 1e-3, seed=5101)
    return p, m0


def test_disc_matches_oracle(torch):
    p, m0 = _disc()
    m, a, rec, mref, aref, recref = _run_both(torch, p, m0, 100, 20)
    inside = np.asarray(p.ms_map) > 0
    dm = np.abs(m - mref).max()
    nrm = np.sqrt((m.astype(np.float64) ** 2).sum(0))
    _say("disc max|dm|", dm, "a", a, aref)
    assert dm <= 1e-4
    assert np.abs(m[:, ~inside]).max() == 0.0
    assert np.abs(nrm[inside] - 1).max() < 1e-6
    assert np.abs(rec[:, 1:4] - recref[:, 1:4]).max() <= 1e-4


def test_batch_with_a_disc_equals_standalone(torch):
    from paper_2410_00966_amd.llgc import Batch, Sim
    p1, m1 = _disc(36)
    p2 = TG._prob(30, 20, 2)
    m2 = I.tilted_uniform_state(p2.shape, 10.0, 1e-3, seed=5102)
    for p in (p1, p2):
        p.method = I.METHOD_DP45
        p.tol = 1e-6
    probs, m0s = [p1, p2], [m1, m2]
    b = Batch(probs)
    for s, m0 in zip(b.sims, m0s):
        s.set_state(torch.from_numpy(m0))
    recs, infos, st = b.run(t_end=8e-12, record_every=3, rec_cap=200)
    outs = [s.get_state() for s in b.sims]
    b.close()
    assert (st == 0).all()
    for k, p in enumerate(probs):
        s = Sim(p, batch_plan=True)
        s.set_state(torch.from_numpy(m0s[k]))
        rec, info = s.run(t_end=8e-12, record_every=3, rec_cap=200)
        m, t, a = s.get_state()
        s.close()
        _say("  inst", k, "accepted", infos[k]["accepted"], info["accepted"])
        assert infos[k]["accepted"] == info["accepted"]
        assert torch.equal(outs[k][0], m) and outs[k][2] == a
        assert np.array_equal(recs[k], rec)


def test_geometry_argument_checks(torch):
    from paper_2410_00966_amd.llgc import Sim, LLGCError
    p, m0 = _disc(32)
    bad = I.Problem(**{**p.__dict__})
    bad.ms_map = -np.asarray(p.ms_map)
    with pytest.raises(LLGCError) as e:
        Sim(bad)
    assert e.value.code == -1
    bad.ms_map = np.zeros_like(np.asarray(p.ms_map))
    with pytest.raises(LLGCError) as e:
        Sim(bad)
    assert e.value.code == -1
    s = Sim(p)
    s.set_state(torch.from_numpy(m0))
    with pytest.raises(LLGCError) as e:
        s.adjoint(4, p.dt, 2, 4)
    assert e.value.code == -7
    s.close()


def test_disc_dp45_matches_oracle_adaptive_run(torch):
    """Adaptive run on the disc with a per-cell B_rms: the same tolerance
    lands both on t_end with close step counts and per-cell agreement."""
    from oracle.llg import CavityLLG
    from paper_2410_00966_amd.llgc import Sim
    p, m0 = _disc(32)
    p.method, p.tol, p.dt = I.METHOD_DP45, 1e-6, 1e-14
    b = np.zeros((3,) + p.shape, np.float32)
    b[0] = np.asarray(p.brms[0]) * (np.asarray(p.ms_map) > 0)
    p.brms_map = b
    T = 15e-12
    s = Sim(p)
    s.set_state(torch.from_numpy(m0))
    _, info = s.run(t_end=T)
    m, t, a = s.get_state()
    s.close()
    mref, aref, tref, _, _, st = CavityLLG(p).run_dp45(
        m0.astype(np.float64), 0j, T, p.tol, p.dt)
    dm = np.abs(m.cpu().numpy() - mref).max()
    _say("disc dp45 accepted", info["accepted"], st["accepted"], "max|dm|",
         dm, "a", a, aref)
    assert t == pytest.approx(T, rel=1e-12)
    assert dm < 1e-4
    assert abs(info["accepted"] - st["accepted"]) <= max(2, st["accepted"] // 50)
    assert np.abs(m.cpu().numpy()[:, np.asarray(p.ms_map) == 0]).max() == 0
