"""GPU tests of the failure semantics of the C ABI: a run that meets a
non-finite state or an underflowing step size reports it (LLGC_E_NONFINITE,
LLGC_E_DT_UNDERFLOW) and leaves the state -- m, t and the cavity amplitude
-- at the last accepted step, for both integrators, and a failing instance
inside a batch fails alone: the healthy instances finish exactly as they
would without it.

The failures are numeric only (a NaN in the state, an FP32 overflow of a
step far too long, a tolerance no step can meet): every kernel still runs
to its end."""
import math
import sys

import numpy as np
import pytest

from paper_2410_00966_amd import inputs as I

pytestmark = pytest.mark.gpu

E_NONFINITE, E_DT_UNDERFLOW = -4, -5


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.skip("no GPU")
    return _t


def _problem(method, nx=24, ny=20, nz=2, seed=8101):
    p = I.Problem(nx=nx, ny=ny, nz=nz, dx=4e-9, dy=4e-9, dz=4e-9, ms=8e5,
                  aex=1.3e-11, alpha=0.02, ku1=1e4, anis_u=(1.0, 0.0, 0.0),
                  bext=(0.0, 0.01, 0.1), method=method, dt=1e-13, tol=1e-6)
    p.wc = 2 * math.pi * 9e9
    p.kappa = 2e-3 * p.wc
    p.brms = (I.brms_from_g(0.02 * p.wc, p.ms * p.ncells * p.vcell), 0.0,
              0.0)
    m0 = I.tilted_uniform_state(p.shape, 10.0, 1e-3, seed=seed)
    return p, m0


def _state(s):
    m, t, a = s.get_state()
    return m.cpu().numpy().copy(), t, a


def test_rk4_overflowing_step_keeps_last_accepted_state(torch):
    """Three good RK4 steps, then one step of 1 us: the FP32 stage values
    overflow within the step.  The run reports LLGC_E_NONFINITE and m, t
    and alpha are those after the third step, bit for bit."""
    from paper_2410_00966_amd.llgc import LLGCError, Sim
    p, m0 = _problem(I.METHOD_RK4)
    s = Sim(p)
    s.set_state(torch.from_numpy(m0), 0.0, 0.01 + 0.02j)
    s.run(nsteps=3)
    m3, t3, a3 = _state(s)
    assert np.isfinite(m3).all() and t3 == pytest.approx(3e-13, rel=1e-12)
    p.dt = 1e-6
    s.set_params(p)
    with pytest.raises(LLGCError) as e:
        s.run(nsteps=2)
    _say("rk4 overflow:", e.value)
    assert e.value.code == E_NONFINITE
    m, t, a = _state(s)
    assert t == t3 and a == a3
    assert np.array_equal(m, m3)
    # the context is usable again with a sane step: same as an unbroken run
    p.dt = 1e-13
    s.set_params(p)
    s.run(nsteps=2)
    m5, t5, a5 = _state(s)
    s.close()
    r = Sim(p)
    r.set_state(torch.from_numpy(m0), 0.0, 0.01 + 0.02j)
    r.run(nsteps=5)
    mr, tr, ar = _state(r)
    r.close()
    assert np.array_equal(m5, mr) and a5 == ar
    assert t5 == pytest.approx(tr, rel=1e-15)


@pytest.mark.parametrize("method", [I.METHOD_RK4, I.METHOD_DP45])
def test_nan_state_is_reported_and_kept(torch, method):
    """A state seeded with one NaN component: the run reports
    LLGC_E_NONFINITE; no step is accepted, so m (NaN included), t and alpha
    are exactly the seeded ones."""
    from paper_2410_00966_amd.llgc import LLGCError, Sim
    p, m0 = _problem(method)
    bad = m0.copy()
    bad[1, 1, 7, 5] = np.nan
    s = Sim(p)
    s.set_state(torch.from_numpy(bad), 2e-12, -0.1 + 0.05j)
    with pytest.raises(LLGCError) as e:
        if method == I.METHOD_RK4:
            s.run(nsteps=4)
        else:
            s.run(t_end=3e-12)
    _say("nan state:", method, e.value)
    assert e.value.code == E_NONFINITE
    m, t, a = _state(s)
    s.close()
    assert t == 2e-12 and a == -0.1 + 0.05j
    assert np.array_equal(m, bad, equal_nan=True)


def test_dp45_underflow_keeps_state_after_progress(torch):
    """DP45 accepts a few steps, then the tolerance is tightened beyond
    reach: the run reports LLGC_E_DT_UNDERFLOW and the state is the one the
    accepted steps left."""
    from paper_2410_00966_amd.llgc import LLGCError, Sim
    p, m0 = _problem(I.METHOD_DP45)
    s = Sim(p)
    s.set_state(torch.from_numpy(m0))
    s.run(nsteps=5, t_end=1.0)
    m5, t5, a5 = _state(s)
    p.tol = 1e-30
    p.dt_min = 1e-17
    s.set_params(p)
    with pytest.raises(LLGCError) as e:
        s.run(t_end=1e-9)
    assert e.value.code == E_DT_UNDERFLOW
    m, t, a = _state(s)
    s.close()
    assert t == t5 and a == a5 and np.array_equal(m, m5)


def _batch_with_bad(torch, method, spoil):
    """Four instances, the third spoiled by `spoil(p, m0)`; returns the
    batch outcome and each healthy instance's standalone batch-plan run."""
    from paper_2410_00966_amd.llgc import Batch, Sim
    shapes = [(16, 16, 1), (40, 24, 2), (32, 20, 2), (24, 48, 3)]
    probs, m0s = [], []
    for k, sh in enumerate(shapes):
        p, m0 = _problem(method, *sh, seed=8200 + k)
        probs.append(p)
        m0s.append(m0)
    spoil(probs[2], m0s[2])
    run = (dict(nsteps=40) if method == I.METHOD_RK4
           else dict(t_end=6e-12))
    b = Batch(probs)
    for k, s in enumerate(b.sims):
        s.set_state(torch.from_numpy(m0s[k]))
    recs, infos, st = b.run(record_every=4, rec_cap=64, check=False, **run)
    outs = [_state(s) for s in b.sims]
    b.close()
    refs = {}
    for k in (0, 1, 3):
        s = Sim(probs[k], batch_plan=True)
        s.set_state(torch.from_numpy(m0s[k]))
        rec, info = s.run(record_every=4, rec_cap=64, **run)
        refs[k] = (_state(s), rec, info)
        s.close()
    return outs, recs, infos, st, refs, m0s


def _check_healthy(outs, recs, infos, refs):
    for k, ((mr, tr, ar), recr, infor) in refs.items():
        m, t, a = outs[k]
        assert infos[k]["accepted"] == infor["accepted"]
        assert infos[k]["rejected"] == infor["rejected"]
        assert t == tr and a == ar
        assert np.array_equal(m, mr)
        assert np.array_equal(recs[k], recr)


def test_batch_nan_instance_fails_alone(torch):
    """RK4 batch, one instance seeded with a NaN: it alone reports
    LLGC_E_NONFINITE and keeps its seeded state; the others equal their
    standalone runs bit for bit."""
    def spoil(p, m0):
        m0[0, 0, 3, 4] = np.nan
    outs, recs, infos, st, refs, m0s = _batch_with_bad(
        torch, I.METHOD_RK4, spoil)
    _say("batch nan status", st)
    assert list(st) == [0, 0, E_NONFINITE, 0]
    m, t, _ = outs[2]
    assert t == 0.0 and np.array_equal(m, m0s[2], equal_nan=True)
    _check_healthy(outs, recs, infos, refs)


def test_batch_underflow_instance_fails_alone(torch):
    """DP45 batch, one instance with tol = 1e-30: it alone reports
    LLGC_E_DT_UNDERFLOW with its initial state kept; the others equal their
    standalone runs bit for bit."""
    def spoil(p, m0):
        p.tol = 1e-30
        p.dt_min = 1e-17
    outs, recs, infos, st, refs, m0s = _batch_with_bad(
        torch, I.METHOD_DP45, spoil)
    _say("batch underflow status", st)
    assert list(st) == [0, 0, E_DT_UNDERFLOW, 0]
    m, t, _ = outs[2]
    assert t == 0.0 and np.array_equal(m, m0s[2])
    _check_healthy(outs, recs, infos, refs)
