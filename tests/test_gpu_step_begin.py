"""GPU test of the Dormand-Prince attempt end fused into the next attempt's
start (k_step_begin): runs with it (the default) and with the separate
one-workgroup controller (LLGC_NO_STEP_BEGIN, read when a context is
created) take the same decisions from the same largest error -- the fused
path reads it as the field pass's atomic maximum of the error bits, the
separate one as the maximum over the per-workgroup partials -- so states,
amplitudes, step counts and records agree bit for bit, rejected attempts
and recorded steps included, and both match the oracle."""
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


def _run(torch, p, m0, fused, timing=True, **run):
    from paper_2410_00966_amd.llgc import Sim
    keep = os.environ.get("LLGC_NO_STEP_BEGIN")
    os.environ.pop("LLGC_NO_STEP_BEGIN", None)
    if not fused:
        os.environ["LLGC_NO_STEP_BEGIN"] = "1"
    try:
        s = Sim(p)
    finally:
        os.environ.pop("LLGC_NO_STEP_BEGIN", None)
        if keep is not None:
            os.environ["LLGC_NO_STEP_BEGIN"] = keep
    s.set_state(torch.from_numpy(m0), 0.0, 0.05j)
    s.set_timing(timing)   # timed runs launch directly, others replay graphs
    rec, info = s.run(**run)
    names = set(s.kernel_times())
    m, t, a = s.get_state()
    s.close()
    return m.cpu().numpy(), t, a, np.asarray(rec), info, names


@pytest.mark.parametrize("grid,dt0,tol", [((64, 48, 2), 1e-14, 1e-6),
                                          ((100, 36, 1), 2e-12, 1e-7)])
def test_step_begin_equals_separate_controller(torch, grid, dt0, tol):
    from oracle.llg import CavityLLG
    p = I.Problem(nx=grid[0], ny=grid[1], nz=grid[2], dx=4e-9, dy=4e-9,
                  dz=4e-9, ms=8e5, aex=1.3e-11, alpha=0.02, ku1=1e4,
                  anis_u=(1.0, 0.0, 0.0), bext=(0.02, 0.01, 0.05),
                  method=I.METHOD_DP45, dt=dt0, tol=tol)
    p.wc = 2 * math.pi * 9e9
    p.kappa = 1e-3 * p.wc
    p.brms = (0.0, I.brms_from_g(0.02 * p.wc, p.ms * p.ncells * p.vcell),
              0.0)
    m0 = I.tilted_uniform_state(p.shape, 20.0, 1e-2, seed=9307)
    run = dict(t_end=4e-12, record_every=3)
    mf, tf, af, rf, inf_, nf = _run(torch, p, m0, True, **run)
    ms, ts, as_, rs, ins, ns = _run(torch, p, m0, False, **run)
    mg, tg, ag, rg, ing, _ = _run(torch, p, m0, True, timing=False, **run)
    _say("step_begin", grid, "accepted", inf_["accepted"], "rejected",
         inf_["rejected"], "records", len(rf))
    assert "k_step_begin" in nf and "k_finish_step" not in nf
    assert "k_finish_step" in ns and "k_step_begin" not in ns
    assert inf_["accepted"] == ins["accepted"]
    assert inf_["rejected"] == ins["rejected"]
    assert tf == ts and af == as_
    assert inf_["dt"] == ins["dt"] and inf_["last_err"] == ins["last_err"]
    assert np.array_equal(mf, ms)
    assert rf.shape == rs.shape and len(rf) >= 2
    assert np.array_equal(rf, rs)
    # the captured chunks replay the same launches
    assert ing["accepted"] == inf_["accepted"] and tg == tf and ag == af
    assert np.array_equal(mg, mf) and np.array_equal(rg, rf)
    if dt0 > 1e-13:
        # the first attempts, far above the tolerance, are rejected
        assert inf_["rejected"] >= 1
    o = CavityLLG(p)
    mref, aref, _, _, _, _ = o.run_dp45(m0.astype(np.float64), 0.05j,
                                        4e-12, p.tol, p.dt)
    de = np.abs(mf - mref).max()
    _say("  fused vs oracle max|dm|", de, "|da|", abs(af - aref))
    assert de <= 1e-4
