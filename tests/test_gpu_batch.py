"""GPU tests of the batched engine (llgc_batch_*).

* Every instance of a ragged batch against the same problem solved alone
  with the batch plan (`Sim(..., batch_plan=True)`): the batched kernels run
  the same device bodies on the same buffers with the same reduction
  orders, so trajectories, records and step counts must agree bit for bit.
* Batched RK4 instances against the FP64 oracle (per cell, 1e-4, as the
  single-instance parity tests), so the batch is pinned to the oracle and
  not only to the single-instance path.
* A sample of the 512-instance sweep (sizes U{16..128}^2 x U{1..4}) run in
  full as one batch, sampled instances against standalone solves.
* Instances that start finished, instances that finish at different
  attempts (retired from the launches), and argument errors.
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


def _rich(nx, ny, nz, seed, method=I.METHOD_DP45, demag=True):
    """Small problem with every field term, a cavity drive and a field
    drive; parameters vary with `seed`."""
    rng = np.random.default_rng(seed)
    p = I.Problem(nx=nx, ny=ny, nz=nz, dx=5e-9, dy=4e-9, dz=3e-9,
                  ms=float(rng.uniform(6e5, 9e5)), aex=1.3e-11,
                  alpha=float(rng.uniform(0.01, 0.05)),
                  ku1=float(rng.uniform(0, 5e4)), anis_u=(0.6, 0.0, 0.8),
                  bext=(0.01, 0.02, float(rng.uniform(0.05, 0.3))),
                  enable_demag=demag, method=method, tol=1e-6, dt=5e-14)
    p.wc = 2 * math.pi * float(rng.uniform(5e9, 15e9))
    p.kappa = 1e-3 * p.wc
    p.brms = (I.brms_from_g(0.02 * p.wc, p.ms * p.ncells * p.vcell), 0.0,
              0.0)
    p.fdrive_kind, p.fdrive_amp, p.fdrive_w = I.DRIVE_SINC, 0.005, 2e11
    p.fdrive_dir = (0.0, 1.0, 0.0)
    p.cdrive_kind, p.cdrive_amp, p.cdrive_w = I.DRIVE_CW, 1e7, p.wc
    m0 = I.tilted_uniform_state(p.shape, 10.0, 0.02, seed=seed)
    return p, m0


def _standalone(torch, p, m0, a0, t0, **run):
    from paper_2410_00966_amd.llgc import Sim
    s = Sim(p, batch_plan=True)
    s.set_state(torch.from_numpy(m0), t0, a0)
    rec, info = s.run(**run)
    m, t, a = s.get_state()
    s.close()
    return m.cpu().numpy(), t, a, rec, info


def _run_batch(torch, probs, m0s, a0s=None, t0s=None, **run):
    from paper_2410_00966_amd.llgc import Batch
    b = Batch(probs)
    for k, s in enumerate(b.sims):
        s.set_state(torch.from_numpy(m0s[k]), t0s[k] if t0s else 0.0,
                    a0s[k] if a0s else 0j)
    recs, infos, st = b.run(**run)
    out = [s.get_state() for s in b.sims]
    b.close()
    return [(m.cpu().numpy(), t, a) for m, t, a in out], recs, infos, st


def _assert_same(k, got, ref):
    (m, t, a), rec, info = got
    mr, tr, ar, recr, infor = ref
    _say(f"  inst {k}: acc {info['accepted']}/{infor['accepted']} rej "
         f"{info['rejected']}/{infor['rejected']} max|dm| "
         f"{np.abs(m - mr).max():.3e}")
    assert info["accepted"] == infor["accepted"]
    assert info["rejected"] == infor["rejected"]
    assert t == tr and a == ar
    assert np.array_equal(m, mr)
    assert np.array_equal(rec, recr)


SHAPES = [(16, 16, 1), (40, 24, 2), (64, 20, 3), (24, 72, 4), (100, 36, 1),
          (128, 17, 2)]


def test_batch_dp45_bitwise_equals_standalone(torch):
    _say("batch dp45 vs standalone")
    probs, m0s = [], []
    for k, sh in enumerate(SHAPES):
        p, m0 = _rich(*sh, seed=100 + k)
        probs.append(p)
        m0s.append(m0)
    q = probs[2]
    q.ms_map = I.smooth_map(q.nx, q.ny, q.nz, 6e5, 9e5, 4, 2, seed=7)
    probs[3].enable_demag = False
    a0s = [0j, 0.1 + 0.2j, 0j, -0.3j, 0j, 0.05 + 0j]
    T = 20e-12
    outs, recs, infos, st = _run_batch(torch, probs, m0s, a0s, t_end=T,
                                       record_every=3, rec_cap=400)
    assert (st == 0).all()
    for k, p in enumerate(probs):
        ref = _standalone(torch, p, m0s[k], a0s[k], 0.0, t_end=T,
                          record_every=3, rec_cap=400)
        _assert_same(k, (outs[k], recs[k], infos[k]), ref)
        assert outs[k][1] == pytest.approx(T, rel=1e-12)


def test_batch_rk4_against_oracle_and_standalone(torch):
    from oracle.llg import CavityLLG
    _say("batch rk4 vs oracle")
    shapes = [(16, 16, 1), (20, 17, 2), (33, 18, 3)]
    probs, m0s = [], []
    for k, sh in enumerate(shapes):
        p, m0 = _rich(*sh, seed=200 + k, method=I.METHOD_RK4)
        p.dt = 4e-14 + 1e-14 * k
        probs.append(p)
        m0s.append(m0)
    n = 150
    outs, recs, infos, st = _run_batch(torch, probs, m0s, nsteps=n,
                                       record_every=25, rec_cap=16)
    assert (st == 0).all()
    for k, p in enumerate(probs):
        o = CavityLLG(p)
        mref, aref, tref, recref = o.run_rk4(m0s[k].astype(np.float64), 0j,
                                             p.dt, n, 25)
        m, t, a = outs[k]
        dm = np.abs(m - mref).max()
        _say(f"  inst {k}: max|dm| vs oracle {dm:.3e}")
        assert dm <= 1e-4
        assert t == pytest.approx(tref, rel=1e-12)
        assert np.abs(recs[k][:, 1:4] - recref[:, 1:4]).max() <= 1e-4
        assert abs(a - aref) <= 1e-3 * max(1.0, abs(aref))
        ref = _standalone(torch, p, m0s[k], 0j, 0.0, nsteps=n,
                          record_every=25, rec_cap=16)
        _assert_same(k, (outs[k], recs[k], infos[k]), ref)


def test_batch_retires_finished_instances(torch):
    """Instances needing very different step counts (weak vs strong field)
    and one that starts at t_end: each still equals its standalone run."""
    _say("batch retirement")
    probs, m0s, t0s = [], [], []
    for k in range(10):
        p, m0 = _rich(32, 16 + 4 * k, 1 + k % 4, seed=300 + k)
        p.bext = (0.0, 0.0, 0.02 if k % 2 else 1.5)
        probs.append(p)
        m0s.append(m0)
        t0s.append(0.0)
    T = 15e-12
    t0s[4] = T
    outs, recs, infos, st = _run_batch(torch, probs, m0s, t0s=t0s, t_end=T)
    assert (st == 0).all()
    assert infos[4]["accepted"] == 0 and outs[4][1] == T
    acc = [i["accepted"] for i in infos]
    _say("  accepted per instance", acc)
    assert max(acc) > 2 * min(a for a in acc if a > 0)
    for k, p in enumerate(probs):
        ref = _standalone(torch, p, m0s[k], 0j, t0s[k], t_end=T)
        _assert_same(k, (outs[k], recs[k], infos[k]), ref)


def test_sweep_sample_of_the_full_batch(torch):
    """All 512 instances of the size/coupling sweep as one batch over a
    short window; sampled instances against standalone solves."""
    _say("full sweep batch, 512 instances")
    inst = I.c4_instances()
    probs = [p for p, m0, run in inst]
    m0s = [m0 for p, m0, run in inst]
    T = 3e-12
    outs, recs, infos, st = _run_batch(torch, probs, m0s, t_end=T)
    assert (st == 0).all()
    for k in range(len(probs)):
        assert outs[k][1] == pytest.approx(T, rel=1e-12)
        nrm = np.sqrt((outs[k][0].astype(np.float64) ** 2).sum(0))
        assert np.abs(nrm - 1).max() < 1e-6
    for k in (0, 137, 301, 511):
        ref = _standalone(torch, probs[k], m0s[k], 0j, 0.0, t_end=T)
        _assert_same(k, (outs[k], recs[k], infos[k]), ref)


def test_batch_argument_errors(torch):
    from paper_2410_00966_amd.llgc import Batch, LLGCError
    p1, m1 = _rich(16, 16, 1, seed=1)
    p2, m2 = _rich(20, 16, 1, seed=2, method=I.METHOD_RK4)
    b = Batch([p1, p2])
    with pytest.raises(LLGCError) as e:
        b.run(t_end=1e-12)           # no state yet
    assert e.value.code == -6
    b.sims[0].set_state(torch.from_numpy(m1))
    b.sims[1].set_state(torch.from_numpy(m2))
    with pytest.raises(LLGCError) as e:
        b.run(t_end=1e-12)           # mixed methods
    assert e.value.code == -1
    b.close()
