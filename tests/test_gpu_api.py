"""GPU tests of the degenerate and error paths of the C ABI: runs that take
no step, a single step, record buffers smaller than the run, the cavity
decoupled from the magnet (B_rms = 0: the free cavity, closed form),
ResetMemoryTerm's analogue, step-size underflow (reported, state kept at
the last accepted step) and calls before a state is set."""
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


def _problem(method=I.METHOD_RK4, brms=(2e-3, 0.0, 0.0)):
    p = I.Problem(nx=24, ny=20, nz=2, dx=4e-9, dy=4e-9, dz=4e-9, ms=8e5,
                  aex=1.3e-11, alpha=0.02, bext=(0.0, 0.0, 0.1),
                  method=method, dt=1e-13, tol=1e-6)
    p.wc = 2 * math.pi * 9e9
    p.kappa = 2e-3 * p.wc
    p.brms = brms
    m0 = I.tilted_uniform_state(p.shape, 10.0, 1e-3, seed=8001)
    return p, m0


def test_runs_without_steps_change_nothing(torch):
    from paper_2410_00966_amd.llgc import Sim
    for method in (I.METHOD_RK4, I.METHOD_DP45):
        p, m0 = _problem(method)
        s = Sim(p)
        s.set_state(torch.from_numpy(m0), 1e-12, 0.2 + 0.1j)
        _, info = s.run(nsteps=0, t_end=1e-12)
        m, t, a = s.get_state()
        s.close()
        assert info["accepted"] == 0 and info["rejected"] == 0
        assert t == 1e-12 and a == 0.2 + 0.1j
        assert np.array_equal(m.cpu().numpy(), m0)


def test_single_step_and_record_truncation(torch):
    from paper_2410_00966_amd.llgc import Sim
    p, m0 = _problem(I.METHOD_DP45)
    s = Sim(p)
    s.set_state(torch.from_numpy(m0))
    info = s.step()
    assert info["accepted"] == 1 and info["rejected"] == 0
    _, t1, _ = s.get_state()
    assert t1 > 0 and t1 == info["t"]
    rec, info = s.run(nsteps=20, t_end=1.0, record_every=1, rec_cap=5)
    assert info["accepted"] == 20
    assert rec.shape == (5, 6)
    assert rec[0, 0] == t1 and np.all(np.diff(rec[:, 0]) > 0)
    s.close()


def test_free_cavity_closed_form(torch):
    from paper_2410_00966_amd.llgc import Sim
    p, m0 = _problem(I.METHOD_RK4, brms=(0.0, 0.0, 0.0))
    a0 = 0.3 - 0.2j
    s = Sim(p)
    assert s.cavity_enabled() == 0
    s.set_state(torch.from_numpy(m0), 0.0, a0)
    n = 500
    rec, _ = s.run(nsteps=n, record_every=50)
    s.close()
    t = rec[:, 0]
    ref = a0 * np.exp(-(1j * p.wc + p.kappa) * t)
    got = rec[:, 4] + 1j * rec[:, 5]
    err = np.abs(got - ref).max() / abs(a0)
    _say("free cavity rel err", err)
    assert err < 1e-9


def test_reset_cavity(torch):
    from paper_2410_00966_amd.llgc import Sim
    p, m0 = _problem()
    s = Sim(p)
    s.set_state(torch.from_numpy(m0), 3e-12, 0.5j)
    s.run(nsteps=10)
    s.reset_cavity(0.4, -0.6)                 # x0 = 2 Re a, p0 = -2 Im a
    _, t, a = s.get_state()
    assert t == 0.0 and a == complex(0.2, 0.3)
    s.close()


def test_step_size_underflow_is_reported(torch):
    from paper_2410_00966_amd.llgc import Sim, LLGCError
    p, m0 = _problem(I.METHOD_DP45)
    p.tol = 1e-30
    p.dt_min = 1e-17
    s = Sim(p)
    s.set_state(torch.from_numpy(m0))
    with pytest.raises(LLGCError) as e:
        s.run(t_end=1e-12)
    assert e.value.code == -5
    m, t, _ = s.get_state()
    assert t == 0.0 and np.array_equal(m.cpu().numpy(), m0)
    s.close()


def test_calls_before_state(torch):
    from paper_2410_00966_amd.llgc import Sim, LLGCError
    p, m0 = _problem()
    s = Sim(p)
    with pytest.raises(LLGCError) as e:
        s.run(nsteps=1)
    assert e.value.code == -6
    s.close()
