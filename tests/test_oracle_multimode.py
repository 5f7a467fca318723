"""Pins of the oracle's multimode cavity (section "Ferromagnetic materials in
a cavity": a cavity with several modes is simulated as the sum of its
modes, each with its own vacuum field, frequency and loss).

  * Degenerate modes with equal vacuum fields: the difference a1 - a2 is
    not coupled and decays freely, exactly, for any amplitude; the sum acts
    as one mode with vacuum field sqrt(2) B_rms and amplitude
    (a1 + a2)/sqrt(2) -- the whole nonlinear trajectory equals that
    single-mode run.
  * A mode with no vacuum field decouples: the other modes follow the
    single-mode run, it decays freely.
  * Polaritons: linearising the Dicke macrospin (section "Benchmark") with M
    modes gives the characteristic equation
        (wz^2 - W^2) = sum_k 4 lam_k^2 wz w_k / (w_k^2 - W^2),
    which for one mode is Eq. (dickepolaritons); the oracle's linearised
    right-hand side must have exactly these eigenfrequencies.
  * Energy of Eq. (startH) summed over the modes is conserved without loss
    and damping.
"""
import math

import numpy as np
import pytest

from oracle.llg import CavityLLG
from paper_2410_00966_amd import inputs as I

WC = 2 * math.pi * 10e9


def _film(nx=6, ny=5, nz=2, seed=3):
    p = I.Problem(nx=nx, ny=ny, nz=nz, dx=5e-9, dy=5e-9, dz=5e-9,
                  alpha=0.02, bext=(0.0, 0.0, 0.2), ku1=3e4,
                  anis_u=(1.0, 0.0, 0.0))
    rng = np.random.default_rng(seed)
    m0 = I.normalise_rows(np.array([0.3, 0.1, 1.0]).reshape(3, 1, 1, 1)
                          + 0.2 * rng.normal(size=(3, nz, ny, nx)))
    return p, m0


def _mode(b, wc=WC, kappa=1e-3 * WC, **kw):
    return I.Mode(brms=tuple(b), wc=wc, kappa=kappa, **kw)


def test_degenerate_modes_act_as_one_bright_mode():
    p, m0 = _film()
    b = np.array([0.0, 4e-3, 1e-3])
    a1, a2 = 0.3 - 0.1j, -0.2 + 0.25j
    q = I.Problem(**{**p.__dict__})
    q.modes = [_mode(b), _mode(b)]
    om = CavityLLG(q)
    mm, am, t, recm = om.run_rk4(m0, [a1, a2], 1e-13, 300, record_every=50)
    # the single bright mode
    s = I.Problem(**{**p.__dict__})
    s.brms = tuple(math.sqrt(2.0) * b)
    s.wc, s.kappa = WC, 1e-3 * WC
    os_ = CavityLLG(s)
    ms_, as_, _, recs = os_.run_rk4(m0, (a1 + a2) / math.sqrt(2.0), 1e-13,
                                    300, record_every=50)
    assert np.abs(mm - ms_).max() < 1e-12
    assert abs((am[0] + am[1]) / math.sqrt(2.0) - as_) < 1e-12 * abs(as_)
    assert np.abs(recm[:, 1:4] - recs[:, 1:4]).max() < 1e-12
    # the dark mode decays freely
    free = (a1 - a2) * np.exp(-(1j * WC + 1e-3 * WC) * t)
    assert abs((am[0] - am[1]) - free) < 1e-10 * abs(free)


def test_uncoupled_mode_decays_freely_and_leaves_the_rest():
    p, m0 = _film(seed=4)
    b = (3e-3, 0.0, 2e-3)
    q = I.Problem(**{**p.__dict__})
    q.modes = [_mode(b, wc=0.8 * WC), _mode((0, 0, 0), wc=1.7 * WC,
                                              kappa=0.01 * WC)]
    a0 = [0.1 + 0.2j, 0.5 - 0.3j]
    om = CavityLLG(q)
    mm, am, t, _ = om.run_rk4(m0, a0, 1e-13, 200)
    s = I.Problem(**{**p.__dict__})
    s.brms, s.wc, s.kappa = b, 0.8 * WC, 1e-3 * WC
    ms_, as_, _, _ = CavityLLG(s).run_rk4(m0, a0[0], 1e-13, 200)
    assert np.abs(mm - ms_).max() < 1e-13
    assert abs(am[0] - as_) < 1e-13 * abs(as_)
    free = a0[1] * np.exp(-(1j * 1.7 * WC + 0.01 * WC) * t)
    assert abs(am[1] - free) < 1e-9 * abs(free)


def _jacobian(o, M):
    """Eigenvalues of the RHS linearised about m = z, alpha = 0 in the
    coordinates (m_x, m_y, Re a_k, Im a_k)."""
    n = 2 + 2 * M

    def f(v):
        mx, my = v[0], v[1]
        mz = math.sqrt(1 - mx * mx - my * my)
        m = np.array([mx, my, mz]).reshape(3, 1, 1, 1)
        a = v[2::2] + 1j * v[3::2]
        dm, da = o.rhs(m, a, 0.0)
        out = [dm[0, 0, 0, 0], dm[1, 0, 0, 0]]
        for z in da:
            out += [z.real, z.imag]
        return np.array(out)

    J = np.zeros((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1e-7
        J[:, j] = (f(e) - f(-e)) / 2e-7
    return np.linalg.eigvals(J)


def dicke_multimode_freqs(wz, ws, lams):
    """Positive roots W of (wz^2 - W^2) prod_k (w_k^2 - W^2)
    - sum_k 4 lam_k^2 wz w_k prod_{j != k} (w_j^2 - W^2) = 0."""
    x = np.poly1d([-1.0, 0.0])                  # -W^2 in the variable W^2
    P = np.poly1d([wz ** 2]) + x
    for w in ws:
        P = P * (np.poly1d([w ** 2]) + x)
    for k, (w, lam) in enumerate(zip(ws, lams)):
        term = np.poly1d([4 * lam ** 2 * wz * w])
        for j, wj in enumerate(ws):
            if j != k:
                term = term * (np.poly1d([wj ** 2]) + x)
        P = P - term
    r = np.roots(P.coeffs)
    return np.sort(np.sqrt(r.real))


def test_characteristic_equation_is_the_paper_formula_for_one_mode():
    wz, lam = 1.2 * WC, 0.3 * WC
    got = dicke_multimode_freqs(wz, [WC], [lam])
    r = math.sqrt((wz ** 2 - WC ** 2) ** 2 + 16 * lam ** 2 * wz * WC)
    exp = [math.sqrt((wz ** 2 + WC ** 2 - r) / 2),
           math.sqrt((wz ** 2 + WC ** 2 + r) / 2)]
    assert np.allclose(got, exp, rtol=1e-12)


@pytest.mark.parametrize("ws,lams", [
    ((1.0, 1.6), (0.1, 0.2)),
    ((0.9, 1.05, 1.3), (0.05, 0.15, 0.08)),
    ((1.0, 3.0), (0.2, 0.2)),
])
def test_multimode_polaritons(ws, lams):
    wz = WC
    ws = [w * WC for w in ws]
    lams = [l * WC for l in lams]
    p, _ = I.dicke_macrospin(wz, WC, 0.0)
    ms_v = p.ms * p.vcell
    p.modes = [_mode((I.brms_from_g(l, ms_v), 0.0, 0.0), wc=w, kappa=0.0)
               for w, l in zip(ws, lams)]
    ev = _jacobian(CavityLLG(p), len(ws))
    got = np.sort(np.abs(ev.imag))[::2]
    assert np.allclose(got, dicke_multimode_freqs(wz, ws, lams), rtol=1e-8)
    assert np.abs(ev.real).max() < 1e-6 * WC


def test_well_separated_modes_keep_their_own_splitting():
    """A second mode far above the spin resonance barely moves the
    anticrossing of the resonant one: the lower pair stays within the
    second-order shift lam2^2/(w2 - wz) of Eq. (dickepolaritons)."""
    wz = WC
    lam1, lam2, w2 = 0.02 * WC, 0.02 * WC, 5.0 * WC
    got = dicke_multimode_freqs(wz, [WC, w2], [lam1, lam2])
    r = math.sqrt(16 * lam1 ** 2 * wz * WC)
    single = [math.sqrt((2 * WC ** 2 - r) / 2), math.sqrt((2 * WC ** 2 + r) / 2)]
    assert np.allclose(got[:2], single, atol=2 * lam2 ** 2 / (w2 - wz))
    assert abs((got[1] - got[0]) - (single[1] - single[0])) < 1e-3 * (
        single[1] - single[0])


def test_multimode_energy_conserved():
    """alpha = kappa = 0, static field: the energy of Eq. (startH) with one
    term -V_c 2 Re(a_k) F_k + hbar w_k |a_k|^2 per mode is conserved (RK4
    drift falls ~16x per halving of dt)."""
    p, m0 = _film(nx=4, ny=3, nz=1, seed=9)
    p.alpha = 0.0
    # cavity, coupling and spin energies of one order (~1e-19 J)
    p.modes = [_mode((3e-4, 0, 0), wc=WC, kappa=0.0),
               _mode((0, 4e-4, 1e-4), wc=1.4 * WC, kappa=0.0)]
    o = CavityLLG(p)
    a0 = np.array([0.4 + 0.1j, -0.2 + 0.3j]) * 2e2
    e0 = o.energy(m0, a0)
    drifts = []
    for dt, n in ((4e-14, 200), (2e-14, 400)):
        m, a, _, _ = o.run_rk4(m0, a0, dt, n)
        drifts.append(abs(o.energy(m, a) - e0) / abs(e0))
    assert drifts[1] < 3e-6
    assert 12.0 < drifts[0] / drifts[1] < 64.0


def test_multimode_dp45_matches_fine_rk4():
    p, m0 = _film(nx=4, ny=4, nz=1, seed=5)
    p.modes = [_mode((3e-3, 0, 0), wc=0.9 * WC),
               _mode((0, 2e-3, 0), wc=1.2 * WC, cdrive_kind=I.DRIVE_CW,
                     cdrive_amp=1e-2 * WC, cdrive_w=1.2 * WC)]
    o = CavityLLG(p)
    m5, a5, t5, _, dts, st = o.run_dp45(m0, [0j, 0j], 2e-11, 1e-9, 1e-14)
    m4, a4, _, _ = o.run_rk4(m0, [0j, 0j], 2e-11 / 4000, 4000)
    assert abs(t5 - 2e-11) < 1e-24
    assert np.abs(m5 - m4).max() < 1e-6
    assert np.abs(a5 - a4).max() < 1e-6 * max(1.0, np.abs(a4).max())
    assert st["accepted"] > 5
