"""GPU test of the fused field + forward x passes (k_xfield_fwd), which
integrator chunks use on grids that leave the GPU part-idle: runs with the
fusion forced on and forced off (LLGC_FUSE / LLGC_NO_FUSE, read when a
context is created) agree -- the transforms are the same, only the grouping
of the FP64 coupling sums over tiles differs -- and both match the oracle."""
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


def _run(torch, p, m0, env, **run):
    from paper_2410_00966_amd.llgc import Sim
    keep = {k: os.environ.get(k) for k in ("LLGC_FUSE", "LLGC_NO_FUSE")}
    for k in keep:
        os.environ.pop(k, None)
    os.environ[env] = "1"
    try:
        s = Sim(p)
    finally:
        for k, v in keep.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    s.set_state(torch.from_numpy(m0), 0.0, 0.05j)
    s.set_timing(True)
    rec, info = s.run(record_every=5, **run)
    names = set(s.kernel_times())
    m, t, a = s.get_state()
    s.close()
    return m.cpu().numpy(), t, a, rec, info, names


@pytest.mark.parametrize("method,grid", [(I.METHOD_DP45, (300, 40, 2)),
                                         (I.METHOD_RK4, (130, 70, 3))])
def test_fused_equals_separate_passes_and_oracle(torch, method, grid):
    from oracle.llg import CavityLLG
    p = I.Problem(nx=grid[0], ny=grid[1], nz=grid[2], dx=4e-9, dy=4e-9,
                  dz=4e-9, ms=8e5, aex=1.3e-11, alpha=0.02, ku1=1e4,
                  anis_u=(1.0, 0.0, 0.0), bext=(0.02, 0.01, 0.05),
                  method=method, dt=5e-14 if method == I.METHOD_RK4 else 1e-14,
                  tol=1e-6)
    p.wc = 2 * math.pi * 9e9
    p.kappa = 1e-3 * p.wc
    p.brms = (0.0, I.brms_from_g(0.02 * p.wc, p.ms * p.ncells * p.vcell),
              0.0)
    m0 = I.tilted_uniform_state(p.shape, 20.0, 1e-2, seed=9301)
    run = (dict(nsteps=60) if method == I.METHOD_RK4 else dict(t_end=5e-12))
    mf, tf, af, rf, inf_, nf = _run(torch, p, m0, "LLGC_FUSE", **run)
    ms, ts, as_, rs, ins, ns = _run(torch, p, m0, "LLGC_NO_FUSE", **run)
    assert "k_xfield_fwd" in nf and "k_xfield_fwd" not in ns
    dm = np.abs(mf - ms).max()
    _say("fused vs separate", grid, "max|dm|", dm, "|da|", abs(af - as_))
    assert tf == ts and inf_["accepted"] == ins["accepted"]
    assert dm <= 1e-6
    assert abs(af - as_) <= 1e-9 * abs(as_)
    o = CavityLLG(p)
    if method == I.METHOD_RK4:
        mref, aref, _, _ = o.run_rk4(m0.astype(np.float64), 0.05j, p.dt, 60)
    else:
        mref, aref, _, _, _, _ = o.run_dp45(m0.astype(np.float64), 0.05j,
                                            5e-12, p.tol, p.dt)
    de = np.abs(mf - mref).max()
    _say("  fused vs oracle max|dm|", de)
    assert de <= 1e-4
