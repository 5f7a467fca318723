"""Pins of the oracle's demagnetising tensor and demag field against results
fixed by the mathematics: Aharoni's closed-form prism factor, the trace
identity, the point-dipole far field, brute-force direct sums and symmetry.
"""
import math

import numpy as np
import pytest

from oracle import demag as D


@pytest.mark.parametrize("dims", [(1, 1, 1), (2.0, 1.0, 0.5), (3.0, 0.7, 0.2),
                                  (0.1, 5.0, 1.0), (4e-9, 4e-9, 4e-9)])
def test_self_term_equals_aharoni_prism(dims):
    """The zero-offset cell tensor is the prism's own demagnetising tensor;
    Aharoni (1998) gives its diagonal in closed form, independently."""
    dx, dy, dz = dims
    N = D.tensor_newell(0.0, 0.0, 0.0, dx, dy, dz)
    a, b, c = dx / 2, dy / 2, dz / 2
    assert N[2] == pytest.approx(D.aharoni_prism_factor(a, b, c), rel=1e-11)
    assert N[0] == pytest.approx(D.aharoni_prism_factor(b, c, a), rel=1e-11)
    assert N[1] == pytest.approx(D.aharoni_prism_factor(c, a, b), rel=1e-11)
    assert N[0] + N[1] + N[2] == pytest.approx(1.0, abs=1e-12)
    assert np.abs(N[3:]).max() < 1e-13


def test_cube_self_term_is_one_third():
    N = D.tensor_newell(0.0, 0.0, 0.0, 5e-9, 5e-9, 5e-9)
    assert np.allclose(N[:3], 1.0 / 3.0, atol=1e-13)


def _box_average(Nfull, nx, ny, nz):
    cx = nx - np.abs(np.arange(-(nx - 1), nx))
    cy = ny - np.abs(np.arange(-(ny - 1), ny))
    cz = nz - np.abs(np.arange(-(nz - 1), nz))
    w = cz[:, None, None] * cy[None, :, None] * cx[None, None, :]
    return np.array([(Nfull[c] * w).sum() for c in range(6)]) / (nx * ny * nz)


@pytest.mark.parametrize("grid,cell", [((6, 4, 3), (2.0, 1.0, 0.7)),
                                       ((32, 32, 1), (5e-9, 5e-9, 5e-9)),
                                       ((20, 3, 2), (1.0, 1.0, 1.0))])
def test_box_average_equals_aharoni(grid, cell):
    """A box of uniformly magnetised cells is a uniformly magnetised prism:
    (1/N) sum_ij N(r_i - r_j) must equal the prism's Aharoni factors.  This
    pins every offset of the cell tensor in aggregate (all three regimes are
    exercised on the 32x32 grid)."""
    nx, ny, nz = grid
    dx, dy, dz = cell
    Nf = D.tensor_full(nx, ny, nz, dx, dy, dz)
    avg = _box_average(Nf, nx, ny, nz)
    a, b, c = nx * dx / 2, ny * dy / 2, nz * dz / 2
    assert avg[2] == pytest.approx(D.aharoni_prism_factor(a, b, c), rel=1e-9)
    assert avg[0] == pytest.approx(D.aharoni_prism_factor(b, c, a), rel=1e-9)
    assert avg[1] == pytest.approx(D.aharoni_prism_factor(c, a, b), rel=1e-9)
    assert np.abs(avg[3:]).max() < 1e-12


def test_far_field_is_point_dipole():
    V = 1.0
    for X, Y, Z in [(60.0, 7.0, 1.0), (30.0, 30.0, 2.0), (3.0, 80.0, 0.0)]:
        q = D.tensor_tent_quadrature(X, Y, Z, 1.0, 1.0, 1.0)[:, 0]
        p = D.tensor_point_dipole(X, Y, Z, V)
        r = math.sqrt(X * X + Y * Y + Z * Z)
        assert np.abs(q - p).max() / np.abs(p).max() < 20 * r ** -4


@pytest.mark.parametrize("d", [D.NEAR - 1, D.NEAR, D.NEAR + 1])
def test_newell_and_quadrature_agree_at_the_seam(d):
    for X, Y, Z in [(d, 0.0, 0.0), (d, d - 2.0, 1.0), (1.0, d, 2.0)]:
        n = D.tensor_newell(X, Y, Z, 1.0, 1.0, 1.0)
        q = D.tensor_tent_quadrature(X, Y, Z, 1.0, 1.0, 1.0)[:, 0]
        assert np.abs(n - q).max() / np.abs(q).max() < 3e-9


def test_tensor_symmetries():
    nx, ny, nz = 9, 7, 3
    Nf = D.tensor_full(nx, ny, nz, 1.0, 1.3, 0.8)
    # even/odd parity in each offset direction
    par = D._PARITY
    for c in range(6):
        sx, sy, sz = par[c]
        assert np.allclose(Nf[c][:, :, ::-1], sx * Nf[c], atol=1e-14)
        assert np.allclose(Nf[c][:, ::-1, :], sy * Nf[c], atol=1e-14)
        assert np.allclose(Nf[c][::-1, :, :], sz * Nf[c], atol=1e-14)
    # cube cells: swapping x<->y offsets swaps xx<->yy and keeps xy
    Nc = D.tensor_full(6, 6, 2, 1.0, 1.0, 1.0)
    sw = lambda a: np.swapaxes(a, 1, 2)
    assert np.allclose(sw(Nc[0]), Nc[1], atol=1e-14)
    assert np.allclose(sw(Nc[3]), Nc[3], atol=1e-14)
    assert np.allclose(sw(Nc[4]), Nc[5], atol=1e-14)


def test_fft_convolution_equals_direct_sum():
    rng = np.random.default_rng(7)
    nz, ny, nx = 3, 4, 5
    M = rng.normal(size=(3, nz, ny, nx)) * 8e5
    Nf = D.tensor_full(nx, ny, nz, 2e-9, 3e-9, 1.5e-9)
    Bd = D.demag_field_direct(M, Nf, 4e-7 * math.pi)
    Bf = D.demag_field_fft(M, D.demag_kernel_fft(Nf, (nz, ny, nx)),
                           4e-7 * math.pi)
    assert np.abs(Bd - Bf).max() < 1e-12 * np.abs(Bd).max()


def test_direct_sum_by_hand_two_cells():
    """Two cells along x: field in cell 0 = -mu0 (N(0) M0 + N(-dx) M1)."""
    Nf = D.tensor_full(2, 1, 1, 1.0, 1.0, 1.0)
    M = np.zeros((3, 1, 1, 2))
    M[:, 0, 0, 0] = (1.0, 2.0, 3.0)
    M[:, 0, 0, 1] = (-0.5, 0.25, 4.0)
    B = D.demag_field_direct(M, Nf, 1.0)
    N0 = D.tensor_newell(0.0, 0.0, 0.0, 1.0, 1.0, 1.0)
    N1 = D.tensor_newell(-1.0, 0.0, 0.0, 1.0, 1.0, 1.0)
    T = lambda n: np.array([[n[0], n[3], n[4]], [n[3], n[1], n[5]],
                            [n[4], n[5], n[2]]])
    expect = -(T(N0) @ M[:, 0, 0, 0] + T(N1) @ M[:, 0, 0, 1])
    assert np.allclose(B[:, 0, 0, 0], expect, rtol=1e-13, atol=1e-14)


def test_uniform_box_field_average():
    """Uniform M along z: the box-averaged demag field is -mu0 Ms N_zz(box)."""
    nx, ny, nz = 8, 6, 2
    M = np.zeros((3, nz, ny, nx))
    M[2] = 8e5
    Nf = D.tensor_full(nx, ny, nz, 1.0, 1.0, 1.0)
    B = D.demag_field_fft(M, D.demag_kernel_fft(Nf, (nz, ny, nx)), 1.0)
    expect = -8e5 * D.aharoni_prism_factor(nx / 2, ny / 2, nz / 2)
    assert B[2].mean() == pytest.approx(expect, rel=1e-10)
    assert abs(B[0].mean()) < 1e-6 and abs(B[1].mean()) < 1e-6
