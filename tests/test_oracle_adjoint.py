"""Pins of the gradient oracle (oracle/adjoint.py), CPU only.

oracle/adjoint.py restates the discrete RK4 map with PyTorch float64 ops so
that reverse-mode autograd gives the exact gradient of the windowed photon
number.  It is pinned to something other than itself:
  * its forward values (final state, amplitude, loss) equal the numpy
    oracle's RK4 run (oracle/llg.py, separate code) to rounding;
  * its gradients equal central finite differences of the numpy oracle's
    loss along seeded directions in the Ms map, the Ku map, |B_rms| and the
    cavity drive amplitude (the directional derivative of a smooth map,
    FD error O(h^2)).
"""
import copy
import math

import numpy as np
import pytest

from oracle.adjoint import gradient, TorchCavityLLG
from oracle.llg import CavityLLG
from paper_2410_00966_amd import inputs as I


def _problem():
    nx, ny, nz = 6, 5, 2
    p = I.Problem(nx=nx, ny=ny, nz=nz, dx=4e-9, dy=4e-9, dz=4e-9, ms=8e5,
                  aex=1.3e-11, alpha=0.01, ku1=0.0, anis_u=(1.0, 0.0, 0.0),
                  bext=(0.1, 0.02, 0.0), dt=1e-13)
    p.ms_map = I.smooth_map(nx, ny, nz, 7e5, 9e5, 3, 2, seed=11)
    p.ku1_map = I.smooth_map(nx, ny, nz, 0.0, 1e4, 3, 2, seed=12)
    p.wc = 2 * math.pi * 9.31e9
    p.kappa = 1e-3 * p.wc
    p.brms = (0.0, I.brms_from_g(0.05 * p.wc, 8e5 * p.ncells * p.vcell), 0.0)
    p.cdrive_kind, p.cdrive_w, p.cdrive_amp = I.DRIVE_CW, p.wc, 2e8
    m0 = I.tilted_uniform_state(p.shape, 20.0, 0.05, seed=13, axis="x",
                                toward="y")
    return p, m0.astype(np.float64)


N_STEPS, WINDOW, A0 = 24, (13, 24), 0.3 - 0.1j


def _numpy_loss(p, m0):
    o = CavityLLG(p)
    _, _, _, rec = o.run_rk4(m0, A0, p.dt, N_STEPS, record_every=1)
    a = rec[:, 4] + 1j * rec[:, 5]              # row n = after step n
    n0, n1 = WINDOW
    return float(np.mean(np.abs(a[n0:n1 + 1]) ** 2))


def test_forward_matches_numpy_oracle():
    import torch
    p, m0 = _problem()
    o = CavityLLG(p)
    mref, aref, _, _ = o.run_rk4(m0, A0, p.dt, N_STEPS)
    t = TorchCavityLLG(p)
    brms = torch.tensor(p.brms, dtype=torch.float64)
    L, m, a = t.loss(m0, A0, p.dt, N_STEPS, WINDOW,
                     torch.tensor(p.ms_array()), torch.tensor(p.ku_array()),
                     brms, torch.tensor(p.cdrive_amp, dtype=torch.float64))
    assert np.abs(m.numpy() - mref).max() < 1e-13
    assert abs(complex(a) - aref) < 1e-12 * max(1.0, abs(aref))
    assert float(L) == pytest.approx(_numpy_loss(p, m0), rel=1e-12)


def test_gradient_matches_central_differences_of_numpy_oracle():
    p, m0 = _problem()
    bdir = np.array([0.0, 1.0, 0.0])
    g = gradient(p, m0, A0, p.dt, N_STEPS, WINDOW, bdir)
    L0 = _numpy_loss(p, m0)
    assert g["loss"] == pytest.approx(L0, rel=1e-12)
    rng = np.random.default_rng(14)
    ms0, ku0 = p.ms_array().astype(np.float64), p.ku_array().astype(np.float64)

    def loss_at(dms=0.0, dku=0.0, db=0.0, de=0.0):
        q = copy.deepcopy(p)
        q.ms_map = ms0 + dms
        q.ku1_map = ku0 + dku
        q.brms = tuple(np.asarray(p.brms) + db * bdir)
        q.cdrive_amp = p.cdrive_amp + de
        return _numpy_loss(q, m0)

    checks = []
    for _ in range(2):
        d = rng.standard_normal(ms0.shape)
        h = 1e-3 * 8e5 / np.abs(d).max()
        fd = (loss_at(dms=h * d) - loss_at(dms=-h * d)) / (2 * h)
        checks.append(("ms", fd, float((g["g_ms"] * d).sum())))
        d = rng.standard_normal(ku0.shape)
        h = 1e-3 * 1e4 / np.abs(d).max()
        fd = (loss_at(dku=h * d) - loss_at(dku=-h * d)) / (2 * h)
        checks.append(("ku", fd, float((g["g_ku"] * d).sum())))
    hb = 1e-4 * np.linalg.norm(p.brms)
    checks.append(("brms", (loss_at(db=hb) - loss_at(db=-hb)) / (2 * hb),
                   g["g_brms"]))
    he = 1e-4 * p.cdrive_amp
    checks.append(("eps0", (loss_at(de=he) - loss_at(de=-he)) / (2 * he),
                   g["g_eps0"]))
    for name, fd, ad in checks:
        assert ad == pytest.approx(fd, rel=1e-5), (name, fd, ad)
        assert abs(fd) > 0.0, name
