"""GPU test of llgc_eval_rhs_noalloc, the right-hand-side evaluation for
callers that cannot allocate: its results equal llgc_eval_rhs's (same
kernels, static scratch instead of the context's buffers) on two calls in a
row, the second on a smaller grid, and a grid whose scratch exceeds the
static array is refused with LLGC_E_UNSUPPORTED."""
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


def _problem(nx, ny, nz, seed):
    rng = np.random.default_rng(seed)
    p = I.Problem(nx=nx, ny=ny, nz=nz, dx=4e-9, dy=4e-9, dz=3e-9,
                  ms=8e5, aex=1.3e-11, alpha=0.02, ku1=2e4,
                  anis_u=(0.0, 0.6, 0.8), bext=(0.02, 0.0, 0.1),
                  method=I.METHOD_RK4, dt=1e-13)
    p.wc = 2 * math.pi * 8e9
    p.kappa = 1e-3 * p.wc
    p.brms = (0.0, I.brms_from_g(0.01 * p.wc, p.ms * p.ncells * p.vcell),
              0.0)
    p.ms_map = I.smooth_map(nx, ny, nz, 7e5, 9e5, 4, 3, seed=seed)
    p.fdrive_kind, p.fdrive_amp, p.fdrive_w = I.DRIVE_SINC, 0.003, 1e11
    p.fdrive_dir = (1.0, 0.0, 0.0)
    m0 = I.tilted_uniform_state(p.shape, 20.0, 0.05, seed=seed + 1)
    a = complex(rng.normal(), rng.normal()) * 1e-3
    return p, m0, a


def _compare(torch, p, m0, a, t):
    from paper_2410_00966_amd.llgc import Sim
    s = Sim(p)
    m = torch.from_numpy(m0).cuda()
    dm_ref, B_ref, da_ref = s.eval_rhs(m, a, t)
    dm = torch.full_like(dm_ref, float("nan"))
    B = torch.full_like(B_ref, float("nan"))
    da = s.eval_rhs_noalloc(m, dm, B, a, t)
    s.close()
    _say(f"  {p.nx}x{p.ny}x{p.nz}: max|d dm| "
         f"{(dm - dm_ref).abs().max().item():.3e}, |d da| "
         f"{abs(da - da_ref):.3e}")
    assert torch.equal(dm, dm_ref) and torch.equal(B, B_ref)
    assert da == da_ref


def test_noalloc_equals_eval_rhs_twice_then_smaller(torch):
    _say("eval_rhs_noalloc vs eval_rhs")
    p1, m1, a1 = _problem(200, 136, 2, seed=9101)
    _compare(torch, p1, m1, a1, 3e-12)
    # second call: a smaller grid (the array keeps the first call's data)
    p2, m2, a2 = _problem(37, 22, 3, seed=9102)
    _compare(torch, p2, m2, a2, 1e-12)
    # and the first grid again, after the smaller one
    _compare(torch, p1, m1, a1, 3e-12)


def test_noalloc_refuses_grids_beyond_the_array(torch):
    from paper_2410_00966_amd.llgc import LLGCError, Sim
    p = I.Problem(nx=1024, ny=1024, nz=2, dx=4e-9, dy=4e-9, dz=4e-9,
                  ms=8e5, aex=1.3e-11, alpha=0.02, method=I.METHOD_RK4,
                  dt=1e-13)
    s = Sim(p)
    m = torch.zeros((3, 2, 1024, 1024), dtype=torch.float32, device="cuda")
    m[2] = 1.0
    dm = torch.empty_like(m)
    with pytest.raises(LLGCError) as e:
        s.eval_rhs_noalloc(m, dm)
    s.close()
    _say("  refused:", e.value)
    assert e.value.code == -7
