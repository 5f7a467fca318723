"""Pins of the oracle's Dzyaloshinskii-Moriya field (one of the effective-
field terms listed after Eq. (llg); the energy densities are those of the
Mumax3 reference the paper builds on: interfacial D [m_z div m - (m.grad)
m_z], bulk D m.(curl m)).

  * The field is the negative gradient of the oracle's DMI energy, B_i =
    -(1/(Ms_i V_c)) dE/dm_i, checked by central differences of the energy
    on a random state with an empty cell (both kinds, anisotropic cells).
  * Continuum limit: in the interior of a smooth texture the field equals
    the closed forms (2D/Ms)(dm_z/dx, dm_z/dy, -dm_x/dx - dm_y/dy)
    (interfacial) and -(2D/Ms) curl m (bulk) evaluated analytically, with
    an error that falls 4x when the cell size halves (second order): a
    wrong sign, chirality or factor fails.
  * Chirality: interfacial DMI lowers the energy of the cycloid that
    rotates one way in the x-z plane and raises it for the other, by the
    continuum amount -D q (per unit area, q the wave number) at small q.
  * Energy of Eq. (startH) with DMI is conserved at alpha = kappa = 0 (RK4
    drift falls >= 16x when dt halves).
"""
import math

import numpy as np
import pytest

from oracle.llg import CavityLLG, normalise
from paper_2410_00966_amd import inputs as I


def _prob(nx, ny, nz, d=(2e-9, 3e-9, 4e-9), di=0.0, db=0.0, ms=8e5):
    p = I.Problem(nx=nx, ny=ny, nz=nz, dx=d[0], dy=d[1], dz=d[2], ms=ms,
                  aex=1.3e-11, alpha=0.0, enable_demag=False)
    p.dmi_int, p.dmi_bulk = di, db
    return p


@pytest.mark.parametrize("di,db", [(3e-3, 0.0), (0.0, 2e-3), (1.5e-3, -1e-3)])
def test_field_is_energy_gradient(di, db):
    p = _prob(5, 4, 3, di=di, db=db)
    ms = np.full(p.shape, 8e5)
    ms[1, 2, 3] = 0.0                     # an empty cell: bonds omitted
    ms[0, 0, 0] = 5e5
    p.ms_map = ms.astype(np.float32)
    o = CavityLLG(p)
    rng = np.random.default_rng(11)
    m = normalise(rng.normal(size=(3,) + p.shape)) * o.inside[None]
    B = o.dmi(m)
    h = 1e-6
    for (c, z, y, x) in [(0, 0, 0, 0), (2, 1, 1, 2), (1, 2, 3, 4),
                         (0, 1, 2, 2), (2, 0, 2, 3), (1, 1, 3, 3)]:
        if not o.inside[z, y, x]:
            continue
        mp, mm = m.copy(), m.copy()
        mp[c, z, y, x] += h
        mm[c, z, y, x] -= h
        g = (o.dmi_energy(mp) - o.dmi_energy(mm)) / (2 * h)
        ref = -g / (o.ms[z, y, x] * o.vc)
        assert B[c, z, y, x] == pytest.approx(ref, rel=1e-7, abs=1e-12)
    assert np.all(B[:, 1, 2, 3] == 0.0)


def _texture(x, y, z, L):
    """A smooth non-uniform texture (not normalised: the field is linear
    in m) and its analytic first derivatives."""
    k = 2 * math.pi / L
    mx = np.sin(k * x) * np.cos(0.5 * k * y)
    my = np.cos(0.7 * k * x + 0.3 * k * z)
    mz = np.cos(k * y) * np.sin(0.4 * k * x)
    d = {
        "mx_x": k * np.cos(k * x) * np.cos(0.5 * k * y),
        "mx_y": -0.5 * k * np.sin(k * x) * np.sin(0.5 * k * y),
        "mx_z": 0.0 * x,
        "my_x": -0.7 * k * np.sin(0.7 * k * x + 0.3 * k * z),
        "my_y": 0.0 * x,
        "my_z": -0.3 * k * np.sin(0.7 * k * x + 0.3 * k * z),
        "mz_x": 0.4 * k * np.cos(k * y) * np.cos(0.4 * k * x),
        "mz_y": -k * np.sin(k * y) * np.sin(0.4 * k * x),
        "mz_z": 0.0 * x,
    }
    return np.stack([mx, my, mz]), d


def _interior_error(n, di, db):
    L = 40e-9
    h = L / n
    p = _prob(n, n, n, d=(h, h, h), di=di, db=db)
    o = CavityLLG(p)
    zz, yy, xx = np.meshgrid(*(((np.arange(n) + 0.5) * h,) * 3),
                             indexing="ij")
    m, d = _texture(xx, yy, zz, L)
    B = o.dmi(m)
    ms = p.ms
    ref = np.zeros_like(B)
    # interfacial: (2D/Ms)(dmz/dx, dmz/dy, -dmx/dx - dmy/dy)
    ref[0] += 2 * di / ms * d["mz_x"]
    ref[1] += 2 * di / ms * d["mz_y"]
    ref[2] += -2 * di / ms * (d["mx_x"] + d["my_y"])
    # bulk: -(2D/Ms) curl m
    curl = np.stack([d["mz_y"] - d["my_z"], d["mx_z"] - d["mz_x"],
                     d["my_x"] - d["mx_y"]])
    ref += -2 * db / ms * curl
    sl = (slice(None), slice(1, -1), slice(1, -1), slice(1, -1))
    return np.abs(B[sl] - ref[sl]).max() / np.abs(ref[sl]).max()


@pytest.mark.parametrize("di,db", [(3e-3, 0.0), (0.0, 2e-3)])
def test_continuum_limit_second_order(di, db):
    e1 = _interior_error(16, di, db)
    e2 = _interior_error(32, di, db)
    assert e1 < 0.05
    assert e1 / e2 == pytest.approx(4.0, rel=0.15)


def test_interfacial_chirality():
    """Cycloids m = (sin qx, 0, cos qx) with q of either sign in a chain:
    each bond holds +-D V_c sin(q dx)/dx, so the two rotation senses differ
    in sign; the continuum energy density D [m_z div m - (m.grad) m_z] of
    this cycloid is +D q."""
    D, n, h = 3e-3, 32, 2e-9
    p = _prob(n, 1, 1, d=(h, h, h), di=D)
    o = CavityLLG(p)
    x = (np.arange(n) + 0.5) * h
    for q in (2 * math.pi / (40 * h), 2 * math.pi / (15 * h)):
        def cyc(qq):
            return np.stack([np.sin(qq * x), 0 * x, np.cos(qq * x)]).reshape(
                3, 1, 1, n)
        ep, em = o.dmi_energy(cyc(q)), o.dmi_energy(cyc(-q))
        per_bond = D * o.vc * math.sin(q * h) / h
        assert ep == pytest.approx((n - 1) * per_bond, rel=1e-12, abs=0)
        assert em == pytest.approx(-(n - 1) * per_bond, rel=1e-12, abs=0)
        # continuum: energy density +D q for this rotation sense
        assert ep / ((n - 1) * o.vc) == pytest.approx(D * q,
                                                      rel=(q * h) ** 2)


def test_energy_conserved_with_dmi():
    p = _prob(6, 5, 2, d=(3e-9, 3e-9, 3e-9), di=2e-3, db=1e-3)
    p.bext = (0.0, 0.0, 0.05)
    p.enable_demag = True
    o = CavityLLG(p)
    rng = np.random.default_rng(5)
    m0 = normalise(np.array([0.2, 0.1, 1.0]).reshape(3, 1, 1, 1)
                   + 0.3 * rng.normal(size=(3,) + p.shape))
    e0 = o.energy(m0, 0j)
    drift = []
    for dt in (4e-14, 2e-14):
        m, _, _, _ = o.run_rk4(m0, 0j, dt, int(round(2e-12 / dt)))
        drift.append(abs(o.energy(m, 0j) - e0))
    assert drift[0] > 0 and drift[0] / drift[1] >= 16.0
