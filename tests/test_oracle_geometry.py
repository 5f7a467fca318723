"""Pins of the oracle's geometry handling (cells with Ms = 0 are outside the
magnet), CPU only.  A magnetic block embedded in a larger grid of empty
cells is the same magnet as that block on its own grid: with exchange
(outside neighbours omitted, as at the open boundary), anisotropy, demag
(empty cells carry no moment) and the cavity coupling, its trajectory,
cavity amplitude and averages equal the standalone block's, and so does
the effective field on its cells; the empty cells stay at m = 0.  Planted mistakes (exchange reaching into empty cells,
averages over all cells) are caught.
"""
import math

import numpy as np
import pytest

from oracle import llg as L
from oracle.llg import CavityLLG
from paper_2410_00966_amd import inputs as I


def _prob(nx, ny, nz):
    p = I.Problem(nx=nx, ny=ny, nz=nz, dx=4e-9, dy=5e-9, dz=3e-9, ms=8e5,
                  aex=1.3e-11, alpha=0.02, ku1=3e4, anis_u=(0.6, 0.0, 0.8),
                  bext=(0.01, 0.02, 0.1), dt=1e-13)
    p.wc = 2 * math.pi * 9e9
    p.kappa = 1e-3 * p.wc
    p.brms = (2e-3, -1e-3, 5e-4)
    return p


def _embedded(nx=5, ny=4, nz=2, off=(3, 2)):
    small = _prob(nx, ny, nz)
    big = _prob(nx + 6, ny + 5, nz)
    ms = np.zeros(big.shape)
    ox, oy = off
    ms[:, oy:oy + ny, ox:ox + nx] = small.ms
    big.ms_map = ms
    m0 = I.tilted_uniform_state(small.shape, 15.0, 0.05, seed=5001)
    mb = np.zeros((3,) + big.shape)
    mb[:, :, oy:oy + ny, ox:ox + nx] = m0
    # junk outside: the integrator must clear it
    mb[:, :, 0, 0] = 0.6
    return small, big, m0, mb, (slice(None), slice(None),
                                slice(oy, oy + ny), slice(ox, ox + nx))


def test_embedded_block_is_the_standalone_block():
    small, big, m0, mb, blk = _embedded()
    # effective field on the magnetic cells (an empty neighbour's exchange
    # would add a part along m: invisible in the torque, visible here)
    Bs = CavityLLG(small).effective_field(m0.astype(np.float64), 0.2j, 0.0)
    Bb = CavityLLG(big).effective_field(mb * (big.ms_map > 0)[None], 0.2j,
                                        0.0)
    assert np.abs(Bb[blk] - Bs).max() <= 1e-12 * np.abs(Bs).max()
    n = 40
    ms_, as_, _, rs = CavityLLG(small).run_rk4(m0, 0.2j, small.dt, n, 10)
    mbg, abg, _, rb = CavityLLG(big).run_rk4(mb, 0.2j, small.dt, n, 10)
    assert np.abs(mbg[blk] - ms_).max() <= 1e-12
    assert abs(abg - as_) <= 1e-12 * abs(as_)
    assert np.abs(rb - rs).max() <= 1e-12
    outside = np.ones(big.shape, bool)
    outside[blk[1:]] = False
    assert np.abs(mbg[:, outside]).max() == 0.0


def test_exchange_into_empty_cells_is_caught(monkeypatch):
    def exchange(self, m):
        p = self.p
        lap = np.zeros_like(m)
        for axis, d in ((3, p.dx), (2, p.dy), (1, p.dz)):
            if m.shape[axis] < 2:
                continue
            diff = np.diff(m, axis=axis) / (d * d)
            lo = [slice(None)] * 4
            hi = [slice(None)] * 4
            lo[axis] = slice(0, -1)
            hi[axis] = slice(1, None)
            lap[tuple(lo)] += diff
            lap[tuple(hi)] -= diff
        return 2.0 * p.aex * self.inv_ms * lap
    monkeypatch.setattr(L.CavityLLG, "exchange", exchange)
    with pytest.raises(AssertionError):
        test_embedded_block_is_the_standalone_block()


def test_average_over_all_cells_is_caught(monkeypatch):
    def record(self, t, m, a):
        mm = m.reshape(3, -1).mean(axis=1)
        return [t, mm[0], mm[1], mm[2], a.real, a.imag]
    monkeypatch.setattr(L.CavityLLG, "record", record)
    with pytest.raises(AssertionError):
        test_embedded_block_is_the_standalone_block()
