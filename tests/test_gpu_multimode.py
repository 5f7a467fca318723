"""GPU tests of the multimode cavity (llgc_set_modes) against the FP64
oracle, whose multimode path is pinned to the bright/dark decomposition of
degenerate modes, to decoupled modes, to the M-mode linearised Dicke
spectrum and to energy conservation (tests/test_oracle_multimode.py):

  * one right-hand side with three modes (uniform fields, one per-cell map,
    drives on two modes): field, torque and every mode's rate;
  * an RK4 run with two modes and an adaptive Dormand-Prince run with three,
    per cell and per amplitude;
  * degenerate modes on the GPU act as one mode with sqrt(2) B_rms (the
    bright mode) while their difference decays freely;
  * returning to the single mode of the parameters (n_modes = 0) gives the
    single-mode results bit for bit; refusals (batch plan, adjoint, memory
    recursion).
"""
import math
import sys

import numpy as np
import pytest

from paper_2410_00966_amd import inputs as I

pytestmark = pytest.mark.gpu

WC = 2 * math.pi * 9e9


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.skip("no GPU")
    return _t


def _film(nx, ny, nz, method=I.METHOD_RK4):
    p = I.Problem(nx=nx, ny=ny, nz=nz, dx=4e-9, dy=4e-9, dz=4e-9, ms=8e5,
                  aex=1.3e-11, alpha=0.01, ku1=2e4, anis_u=(1.0, 0.0, 0.0),
                  bext=(0.05, 0.0, 0.0), method=method, dt=1e-13, tol=1e-6)
    return p


def _b(p, g_over_wc):
    return I.brms_from_g(g_over_wc * WC, p.ms * p.ncells * p.vcell)


def _modes(p, three=False, seed=0):
    """Two (or three) modes of different frequency, loss and coupling; the
    third has a per-cell field (strongest in the middle of the film) and a
    CW drive; the first a sinc drive."""
    b = _b(p, 0.02)
    md = [I.Mode(brms=(0.0, b, 0.2 * b), wc=0.9 * WC, kappa=1e-3 * WC,
                 x0=0.02, p0=-0.01, cdrive_kind=I.DRIVE_SINC,
                 cdrive_amp=2e7, cdrive_w=2 * math.pi * 20e9),
          I.Mode(brms=(0.0, 0.0, 0.7 * b), wc=1.3 * WC, kappa=3e-3 * WC)]
    if three:
        nz, ny, nx = p.shape
        y = (np.arange(ny) + 0.5) / ny
        prof = np.exp(-((y - 0.5) / 0.3) ** 2)
        rng = np.random.default_rng(seed)
        bm = np.zeros((3,) + p.shape)
        bm[1] = 0.8 * b * prof[None, :, None]
        bm[0] = 0.1 * b * rng.standard_normal(p.shape)
        md.append(I.Mode(wc=1.05 * WC, kappa=2e-3 * WC,
                         brms_map=bm.astype(np.float32),
                         cdrive_kind=I.DRIVE_CW, cdrive_amp=1e7,
                         cdrive_w=1.05 * WC))
    return md


@pytest.mark.parametrize("grid", [(37, 23, 3), (64, 40, 1)])
def test_rhs_three_modes_matches_oracle(torch, grid):
    from oracle.llg import CavityLLG
    from paper_2410_00966_amd.llgc import Sim
    p = _film(*grid)
    p.modes = _modes(p, three=True, seed=sum(grid))
    rng = np.random.default_rng(sum(grid))
    m = rng.normal(size=(3,) + p.shape)
    m = (m / np.sqrt((m * m).sum(0))).astype(np.float32)
    a = np.array([0.6 - 0.3j, -0.2 + 0.4j, 0.1 + 0.1j])
    t = 2.2e-12
    o = CavityLLG(p)
    Bref = o.effective_field(m.astype(np.float64), a, t)
    dref, daref = o.rhs(m.astype(np.float64), a, t)
    s = Sim(p)
    assert s.cavity_enabled() == 1
    dm, B, da = s.eval_rhs(torch.from_numpy(m), a, t)
    s.close()
    eB = np.abs(B.cpu().numpy() - Bref).max() / np.abs(Bref).max()
    ed = np.abs(dm.cpu().numpy() - dref).max() / np.abs(dref).max()
    eda = np.abs(da - daref).max() / np.abs(daref).max()
    _say("multimode rhs", grid, "field", eB, "torque", ed, "rates", eda)
    assert eB < 2e-5 and ed < 2e-5
    assert eda <= 1e-9


def test_rk4_two_modes_matches_oracle(torch):
    from oracle.llg import CavityLLG
    from paper_2410_00966_amd.llgc import Sim
    p = _film(24, 20, 2)
    p.modes = _modes(p)
    m0 = I.tilted_uniform_state(p.shape, 10.0, 1e-3, seed=6101, axis="x",
                                toward="y")
    a0 = [0.01 + 0.02j, -0.03j]
    n, every = 400, 40
    mref, aref, _, recref = CavityLLG(p).run_rk4(m0.astype(np.float64), a0,
                                                 p.dt, n, every)
    s = Sim(p)
    s.set_state(torch.from_numpy(m0), 0.0, a0)
    rec, _ = s.run(nsteps=n, record_every=every)
    m, t, a = s.get_state()
    s.close()
    dm = np.abs(m.cpu().numpy() - mref).max()
    ea = np.abs(a - aref).max() / np.abs(aref).max()
    _say("multimode rk4 max|dm|", dm, "amplitudes", a, aref, "rel", ea)
    assert rec.shape == recref.shape == (n // every + 1, 8)
    assert dm <= 1e-4
    assert ea <= 1e-5
    assert np.abs(rec[:, 1:4] - recref[:, 1:4]).max() <= 1e-4
    sc = np.abs(recref[:, 4:]).max()
    assert np.abs(rec[:, 4:] - recref[:, 4:]).max() <= 1e-5 * sc


def test_dp45_three_modes_matches_oracle(torch):
    from oracle.llg import CavityLLG
    from paper_2410_00966_amd.llgc import Sim
    p = _film(20, 16, 2, method=I.METHOD_DP45)
    p.dt = 1e-14
    p.modes = _modes(p, three=True, seed=7)
    m0 = I.tilted_uniform_state(p.shape, 10.0, 1e-3, seed=6102, axis="x",
                                toward="y")
    T = 20e-12
    mref, aref, tref, _, _, st = CavityLLG(p).run_dp45(
        m0.astype(np.float64), 0j, T, p.tol, p.dt)
    s = Sim(p)
    s.set_state(torch.from_numpy(m0))   # amplitudes from x0, p0
    s.set_mode_amplitudes([0.0, 0.0, 0.0])
    _, info = s.run(t_end=T)
    m, t, a = s.get_state()
    s.close()
    dm = np.abs(m.cpu().numpy() - mref).max()
    ea = np.abs(a - aref).max() / np.abs(aref).max()
    _say("multimode dp45", info["accepted"], st["accepted"], "max|dm|", dm,
         "amp rel", ea)
    assert t == pytest.approx(tref, rel=1e-12)
    assert abs(info["accepted"] - st["accepted"]) <= max(
        1, 0.02 * st["accepted"])
    assert dm <= 1e-4 and ea <= 1e-5


def test_degenerate_modes_are_one_bright_mode_on_gpu(torch):
    """Two equal modes with amplitudes a1, a2: the magnet follows the
    single mode of vacuum field sqrt(2) B_rms started at (a1+a2)/sqrt(2),
    and a1 - a2 decays freely."""
    from paper_2410_00966_amd.llgc import Sim
    p = _film(24, 20, 2)
    b = np.array([0.0, _b(p, 0.03), 0.0])
    kap = 1e-3 * WC
    p.modes = [I.Mode(brms=tuple(b), wc=WC, kappa=kap),
               I.Mode(brms=tuple(b), wc=WC, kappa=kap)]
    m0 = I.tilted_uniform_state(p.shape, 10.0, 1e-3, seed=6103, axis="x",
                                toward="y")
    a1, a2 = 0.3 - 0.1j, -0.2 + 0.25j
    n = 500
    s = Sim(p)
    s.set_state(torch.from_numpy(m0), 0.0, [a1, a2])
    s.run(nsteps=n)
    mm, t, am = s.get_state()
    s.close()
    q = _film(24, 20, 2)
    q.brms = tuple(math.sqrt(2.0) * b)
    q.wc, q.kappa = WC, kap
    r = Sim(q)
    r.set_state(torch.from_numpy(m0), 0.0, (a1 + a2) / math.sqrt(2.0))
    r.run(nsteps=n)
    ms, _, as_ = r.get_state()
    r.close()
    dm = float((mm - ms).abs().max())
    bright = (am[0] + am[1]) / math.sqrt(2.0)
    dark = am[0] - am[1]
    free = (a1 - a2) * np.exp(-(1j * WC + kap) * t)
    _say("degenerate: max|dm|", dm, "bright", bright, as_, "dark", dark,
         free)
    assert dm <= 1e-5
    assert abs(bright - as_) <= 1e-6 * abs(as_)
    assert abs(dark - free) <= 1e-9 * abs(free)


def test_back_to_single_mode_and_refusals(torch):
    from paper_2410_00966_amd.llgc import LLGCError, Sim
    p = _film(64, 16, 1)
    p.brms = (0.0, _b(p, 0.02), 0.0)
    p.wc, p.kappa = WC, 1e-3 * WC
    m0 = I.tilted_uniform_state(p.shape, 10.0, 1e-3, seed=6104)
    ref = Sim(p)
    ref.set_state(torch.from_numpy(m0), 0.0, 0.1j)
    rr, _ = ref.run(nsteps=50, record_every=10)
    mr, _, ar = ref.get_state()
    ref.close()
    s = Sim(p)
    s.set_modes(_modes(p))
    s.set_modes([])                       # back to the parameters' mode
    s.set_state(torch.from_numpy(m0), 0.0, 0.1j)
    rs, _ = s.run(nsteps=50, record_every=10)
    ms, _, as_ = s.get_state()
    assert rs.shape == (6, 6)
    assert torch.equal(ms, mr) and as_ == ar and np.array_equal(rs, rr)
    s.set_modes(_modes(p))
    with pytest.raises(LLGCError) as e:
        s.adjoint(4, p.dt, 2, 4)
    assert e.value.code == -7
    q = I.Problem(**{**p.__dict__})
    q.cavity_mode = I.CAVITY_MEMORY
    with pytest.raises(LLGCError) as e:
        s.set_params(q)
    assert e.value.code == -7
    s.close()
    b = Sim(p, batch_plan=True)
    with pytest.raises(LLGCError) as e:
        b.set_modes(_modes(p))
    assert e.value.code == -7
    b.close()
