"""Pins of the oracle's drives against closed forms.

The paper excites the system with a sinc pulse, f(t) = sin(w t)/(w t)
(appendix "Micromagnetic simulations with Mumax3-cQED"), applied as a field
B_ext += amp f(t) b(r) shaped by a map b(r); a drive of the cavity mode
enters d alpha/dt as -i eps0 f(t).  Both are linear forcings of an
oscillator, whose response is the integral of e^{i w0 tau} sinc(w tau),
known in closed form through the sine and cosine integrals:

  int_0^t cos(v tau) sin(w tau)/tau dtau = [Si((w+v)t) + Si((w-v)t)]/2
  int_0^t sin(v tau) sin(w tau)/tau dtau = [Cin((w+v)t) - Cin((w-v)t)]/2

with Cin(x) = int_0^x (1 - cos u)/u du = gamma_E + ln|x| - Ci(|x|).
These pin the sinc shape (unnormalised, sinc(0) = 1, cut-off w) and the
per-cell drive map independently of the integrator code.
"""
import math

import numpy as np
import pytest
from scipy.special import sici

from oracle.llg import CavityLLG, DRIVE_SINC, DRIVE_CW
from paper_2410_00966_amd import inputs as I

W = 2 * math.pi * 20e9        # cut-off of the sinc pulse, rad/s


def _cin(x):
    x = abs(x)
    if x == 0.0:
        return 0.0
    return np.euler_gamma + math.log(x) - sici(x)[1]


def sinc_response(v, w, t):
    """int_0^t e^{i v tau} sinc(w tau) dtau, sinc(x) = sin(x)/x."""
    re = 0.5 * (sici((w + v) * t)[0] + sici((w - v) * t)[0])
    im = 0.5 * (_cin((w + v) * t) - _cin((w - v) * t))
    return (re + 1j * im) / w


def test_sinc_response_reduces_to_si():
    """At v = 0 the integral is Si(w t)/w; far beyond the cut-off the real
    part tends to pi/(2w) and the imaginary part to ln((w+v)/(w-v))/(2w)."""
    t = 3e-10
    assert sinc_response(0.0, W, t) == pytest.approx(sici(W * t)[0] / W,
                                                     rel=1e-14)
    v = 0.4 * W
    big = sinc_response(v, W, 1e-6)
    assert big.real == pytest.approx(math.pi / (2 * W), rel=1e-5)
    assert big.imag == pytest.approx(
        math.log((W + v) / (W - v)) / (2 * W), rel=1e-5)


@pytest.mark.parametrize("ratio", [0.5, 1.7])
def test_sinc_cavity_drive_closed_form(ratio):
    """Uncoupled lossless cavity driven by -i eps0 sinc(w t):
    alpha(t) = -i eps0 e^{-i wc t} int_0^t e^{i wc tau} sinc(w tau) dtau,
    below (wc < w) and above (wc > w) the cut-off."""
    wc = ratio * W
    p = I.Problem(nx=1, ny=1, nz=1, dx=5e-9, dy=5e-9, dz=5e-9,
                  enable_demag=False, aex=0.0, bext=(0.0, 0.0, 0.1))
    p.wc, p.kappa = wc, 0.0
    p.cdrive_kind, p.cdrive_amp, p.cdrive_w = DRIVE_SINC, 1e9, W
    o = CavityLLG(p)
    m0 = np.zeros((3, 1, 1, 1))
    m0[2] = 1.0
    dt = 2e-14
    _, _, _, rec = o.run_rk4(m0, 0j, dt, 6000, record_every=1500)
    for row in rec[1:]:
        t = row[0]
        exact = -1j * p.cdrive_amp * np.exp(-1j * wc * t) * \
            sinc_response(wc, W, t)
        got = row[4] + 1j * row[5]
        assert abs(got - exact) <= 1e-9 * abs(exact), (t, got, exact)


def _two_cell_drive(fmap, amp=1e-5, b0=0.1):
    """Two cells with no exchange, demag or cavity, precessing about
    B0 z, driven by amp sinc(w t) b_i."""
    p = I.Problem(nx=2, ny=1, nz=1, dx=5e-9, dy=5e-9, dz=5e-9,
                  enable_demag=False, aex=0.0, alpha=0.0,
                  bext=(0.0, 0.0, b0))
    p.fdrive_kind, p.fdrive_amp, p.fdrive_w = DRIVE_SINC, amp, W
    p.fdrive_map = np.asarray(fmap, dtype=np.float32).reshape(3, 1, 1, 2)
    return p


def test_field_drive_map_linear_response():
    """Small-angle response of an undamped cell about B0 z to the field
    amp sinc(w t) b: m+ = m_x + i m_y obeys dm+/dt = i w0 m+ - i gamma amp
    (b_x + i b_y) sinc(w t) with w0 = gamma B0, so from m = z
    m+(t) = -i gamma amp (b_x + i b_y) e^{i w0 t}
            int_0^t e^{-i w0 tau} sinc(w tau) dtau
    to first order in the drive (here |m+| ~ 1e-5: the neglected terms are
    ~1e-10 relative).  Each cell follows its own map vector."""
    # (3 components, 2 cells); a longitudinal part would shift w0 and only
    # enter at second order, so the map is transverse here
    fmap = [[1.0, 0.3], [0.0, -0.8], [0.0, 0.0]]
    p = _two_cell_drive(fmap)
    o = CavityLLG(p)
    m0 = np.zeros((3, 1, 1, 2))
    m0[2] = 1.0
    w0 = p.gamma * p.bext[2]
    m = m0
    t = 0.0
    dt = 2e-14
    for seg in range(3):
        m, _, t, _ = o.run_rk4(m, 0j, dt, 2500, t0=t)
        resp = np.exp(1j * w0 * t) * sinc_response(-w0, W, t)
        for i in range(2):
            bx, by = fmap[0][i], fmap[1][i]
            exact = -1j * p.gamma * p.fdrive_amp * (bx + 1j * by) * resp
            got = m[0, 0, 0, i] + 1j * m[1, 0, 0, i]
            assert abs(got - exact) <= 1e-6 * abs(exact), (t, i, got, exact)


def test_uniform_drive_map_equals_direction():
    """A map holding the same vector in every cell is the uniform drive
    along that vector."""
    rng = np.random.default_rng(7)
    p = I.Problem(nx=5, ny=4, nz=2, dx=4e-9, dy=4e-9, dz=4e-9,
                  bext=(0.0, 0.02, 0.05), alpha=0.02)
    p.fdrive_kind, p.fdrive_amp, p.fdrive_w = DRIVE_CW, 3e-3, 2e10
    p.fdrive_dir = (0.25, -0.75, 0.5)   # exact in float32, as the map
    m0 = I.normalise_rows(rng.normal(size=(3, 2, 4, 5)))
    o1 = CavityLLG(p)
    m1, _, _, _ = o1.run_rk4(m0, 0j, 1e-13, 50)
    q = I.Problem(**{**p.__dict__})
    q.fdrive_dir = (0.0, 0.0, 0.0)
    q.fdrive_map = np.broadcast_to(np.asarray(p.fdrive_dir, dtype=np.float32)
                                   .reshape(3, 1, 1, 1), (3, 2, 4, 5)).copy()
    o2 = CavityLLG(q)
    m2, _, _, _ = o2.run_rk4(m0, 0j, 1e-13, 50)
    assert np.abs(m1 - m2).max() < 1e-14
