"""FP64 CPU oracle: cell-averaged demagnetising tensor and demag field.

TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the CPU-baseline
leg of the benchmark may import this module; the product path never does.

What is computed
----------------
The paper lists demagnetisation among the effective-field terms of the
finite-difference LLG (section "The LLG equation in Mumax3", the sum of field
contributions after Eq. (llg)).  For cells that are uniformly magnetised
orthorhombic boxes, the field in cell i is

    B_d,i = -mu0 * sum_j N(r_i - r_j) . (Ms_j m_j)

where N(Delta) is the demagnetising tensor of a source box averaged over a
target box displaced by Delta.  Its plain definition is the double volume
average of the point-dipole kernel,

    N(Delta) = (1/V) int_target int_source Npt(r - r') dr dr' ,
    Npt(s)   = -(1/(4 pi |s|^3)) (3 s^ s^T - I) .

Three evaluations of that one definition are used, by distance (Chebyshev
distance d in cells):
  * d <= NEAR: Newell, Williams & Dunlop (1993) closed forms f and g with the
    27-point second-difference stencil (exact, cancels badly far away);
  * NEAR < d <= FAR (or everywhere beyond NEAR for non-cubic cells): Gauss-
    Legendre quadrature of Npt over the difference vector w = u - v of the two
    uniform box positions, whose density per axis is the tent
    (d_a - |w_a|)/d_a^2 on [-d_a, d_a];
  * d > FAR with cubic cells: the point dipole V*Npt(Delta), whose relative
    error is O((a/d)^4) for cubes.
The demag field is then either the brute-force direct sum (small grids) or
the zero-padded FFT convolution (numpy's pocketfft as the FFT primitive).
"""
from __future__ import annotations

import math

import numpy as np

COMPONENTS = ("xx", "yy", "zz", "xy", "xz", "yz")

NEAR = 8       # Newell closed forms up to this Chebyshev distance (cells)
FAR = 48       # point dipole beyond this distance (cubic cells only)
GL_HALF = 4    # Gauss-Legendre points on each half of the tent, per axis


def _asinh_ratio(num, den):
    """asinh(num/den), taken as 0 where den == 0 (every such term in f and g
    carries a prefactor that vanishes there)."""
    out = np.zeros(np.broadcast(num, den).shape)
    num = np.broadcast_to(num, out.shape)
    den = np.broadcast_to(den, out.shape)
    ok = den > 0
    out[ok] = np.arcsinh(num[ok] / den[ok])
    return out


def _atan_ratio(num, den):
    """atan(num/den), taken as 0 where den == 0 (prefactor vanishes)."""
    out = np.zeros(np.broadcast(num, den).shape)
    num = np.broadcast_to(num, out.shape)
    den = np.broadcast_to(den, out.shape)
    ok = den != 0
    out[ok] = np.arctan(num[ok] / den[ok])
    return out


def newell_f(x, y, z):
    """Newell's f(x,y,z) (even in every argument, symmetric in y and z)."""
    x = np.abs(np.asarray(x, dtype=np.float64))
    y = np.abs(np.asarray(y, dtype=np.float64))
    z = np.abs(np.asarray(z, dtype=np.float64))
    x2, y2, z2 = x * x, y * y, z * z
    R = np.sqrt(x2 + y2 + z2)
    t1 = 0.5 * y * (z2 - x2) * _asinh_ratio(y, np.sqrt(x2 + z2))
    t2 = 0.5 * z * (y2 - x2) * _asinh_ratio(z, np.sqrt(x2 + y2))
    t3 = -x * y * z * _atan_ratio(y * z, x * R)
    t4 = (2.0 * x2 - y2 - z2) * R / 6.0
    return t1 + t2 + t3 + t4


def newell_g(x, y, z):
    """Newell's g(x,y,z) (odd in x and y, even in z, symmetric in x and y)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    x2, y2, z2 = x * x, y * y, z * z
    R = np.sqrt(x2 + y2 + z2)
    t1 = x * y * z * _asinh_ratio(z, np.sqrt(x2 + y2))
    t2 = y / 6.0 * (3.0 * z2 - y2) * _asinh_ratio(x, np.sqrt(y2 + z2))
    t3 = x / 6.0 * (3.0 * z2 - x2) * _asinh_ratio(y, np.sqrt(x2 + z2))
    t4 = -z2 * z / 6.0 * _atan_ratio(x * y, z * R)
    t5 = -z * y2 / 2.0 * _atan_ratio(x * z, y * R)
    t6 = -z * x2 / 2.0 * _atan_ratio(y * z, x * R)
    t7 = -x * y * R / 3.0
    return t1 + t2 + t3 + t4 + t5 + t6 + t7


def _stencil27(fun, X, Y, Z, a, b, c):
    """sum_{i,j,k in -1,0,1} w_i w_j w_k fun(X+i a, Y+j b, Z+k c) with
    w = (-1, 2, -1): Newell's sixth-order difference."""
    w = {-1: -1.0, 0: 2.0, 1: -1.0}
    acc = np.zeros(np.broadcast(X, Y, Z).shape)
    for i in (-1, 0, 1):
        for j in (-1, 0, 1):
            for k in (-1, 0, 1):
                acc += w[i] * w[j] * w[k] * fun(X + i * a, Y + j * b, Z + k * c)
    return acc


def tensor_newell(X, Y, Z, dx, dy, dz):
    """Exact cell-averaged tensor (6 comps) at physical offsets X, Y, Z."""
    s = 1.0 / (4.0 * math.pi * dx * dy * dz)
    Nxx = _stencil27(newell_f, X, Y, Z, dx, dy, dz) * s
    Nyy = _stencil27(newell_f, Y, X, Z, dy, dx, dz) * s
    Nzz = _stencil27(newell_f, Z, Y, X, dz, dy, dx) * s
    Nxy = _stencil27(newell_g, X, Y, Z, dx, dy, dz) * s
    Nxz = _stencil27(newell_g, X, Z, Y, dx, dz, dy) * s
    Nyz = _stencil27(newell_g, Y, Z, X, dy, dz, dx) * s
    return np.stack([Nxx, Nyy, Nzz, Nxy, Nxz, Nyz])


def tensor_point_dipole(X, Y, Z, V):
    """V * Npt(Delta): the far-field limit."""
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    Z = np.asarray(Z, dtype=np.float64)
    r2 = X * X + Y * Y + Z * Z
    r = np.sqrt(r2)
    pre = -V / (4.0 * math.pi * r2 * r)
    return np.stack([pre * (3 * X * X / r2 - 1), pre * (3 * Y * Y / r2 - 1),
                     pre * (3 * Z * Z / r2 - 1), pre * 3 * X * Y / r2,
                     pre * 3 * X * Z / r2, pre * 3 * Y * Z / r2])


def _tent_rule(h, n):
    """Nodes/weights integrating g(w) (h-|w|)/h^2 over [-h, h] with n
    Gauss-Legendre points on each half."""
    xi, wi = np.polynomial.legendre.leggauss(n)
    # right half [0, h]: w = h (xi+1)/2, density (h - w)/h^2, dw = h/2 dxi
    wr = h * (xi + 1.0) / 2.0
    ww = (h - wr) / (h * h) * (h / 2.0) * wi
    nodes = np.concatenate([-wr[::-1], wr])
    weights = np.concatenate([ww[::-1], ww])
    return nodes, weights


def tensor_tent_quadrature(X, Y, Z, dx, dy, dz, n=GL_HALF):
    """N(Delta) = V * E[Npt(Delta + w)], w per axis tent-distributed; valid
    (and accurate) when the offset is at least two cells away on some axis."""
    X = np.asarray(X, dtype=np.float64).ravel()
    Y = np.asarray(Y, dtype=np.float64).ravel()
    Z = np.asarray(Z, dtype=np.float64).ravel()
    V = dx * dy * dz
    nxs, wxs = _tent_rule(dx, n)
    nys, wys = _tent_rule(dy, n)
    nzs, wzs = _tent_rule(dz, n)
    acc = np.zeros((6, X.size))
    for ax, wa in zip(nxs, wxs):
        for ay, wb in zip(nys, wys):
            for az, wc in zip(nzs, wzs):
                acc += (wa * wb * wc) * tensor_point_dipole(X + ax, Y + ay,
                                                            Z + az, V)
    return acc


def _is_cubic(dx, dy, dz):
    return abs(dx - dy) <= 1e-12 * dx and abs(dx - dz) <= 1e-12 * dx


def tensor_octant(nx, ny, nz, dx, dy, dz):
    """Tensor for non-negative offsets (ix, iy, iz) in [0,nx)x[0,ny)x[0,nz).
    Returns array (6, nz, ny, nx)."""
    iz, iy, ix = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx),
                             indexing="ij")
    cheb = np.maximum(np.maximum(ix, iy), iz)
    out = np.zeros((6, nz, ny, nx))
    near = cheb <= NEAR
    if near.any():
        out[:, near] = tensor_newell(ix[near] * dx, iy[near] * dy,
                                     iz[near] * dz, dx, dy, dz)
    far_lim = FAR if _is_cubic(dx, dy, dz) else np.iinfo(np.int64).max
    mid = (cheb > NEAR) & (cheb <= far_lim)
    if mid.any():
        out[:, mid] = tensor_tent_quadrature(ix[mid] * dx, iy[mid] * dy,
                                             iz[mid] * dz, dx, dy, dz)
    far = cheb > far_lim
    if far.any():
        out[:, far] = tensor_point_dipole(ix[far] * dx, iy[far] * dy,
                                          iz[far] * dz, dx * dy * dz)
    # components odd in an offset direction vanish on that zero plane exactly
    for c, (sx, sy, sz) in _PARITY.items():
        if sx < 0:
            out[c][:, :, 0] = 0.0
        if sy < 0:
            out[c][:, 0, :] = 0.0
        if sz < 0:
            out[c][0, :, :] = 0.0
    return out


# parity of each component under Delta_x -> -Delta_x, Delta_y, Delta_z
_PARITY = {  # (sx, sy, sz)
    0: (1, 1, 1), 1: (1, 1, 1), 2: (1, 1, 1),
    3: (-1, -1, 1), 4: (-1, 1, -1), 5: (1, -1, -1),
}


def tensor_full(nx, ny, nz, dx, dy, dz):
    """Tensor on all offsets Delta in [-(n-1), n-1] per axis.
    Returns (6, 2nz-1, 2ny-1, 2nx-1), index (iz+nz-1, iy+ny-1, ix+nx-1)."""
    oc = tensor_octant(nx, ny, nz, dx, dy, dz)
    full = np.zeros((6, 2 * nz - 1, 2 * ny - 1, 2 * nx - 1))
    for c in range(6):
        sx, sy, sz = _PARITY[c]
        for gz in (1, -1):
            for gy in (1, -1):
                for gx in (1, -1):
                    sign = (sx if gx < 0 else 1) * (sy if gy < 0 else 1) * \
                           (sz if gz < 0 else 1)
                    zi = nz - 1 + gz * np.arange(nz)
                    yi = ny - 1 + gy * np.arange(ny)
                    xi = nx - 1 + gx * np.arange(nx)
                    full[c][np.ix_(zi, yi, xi)] = sign * oc[c]
    return full


def _as_matrix(Nfull_at):
    """Nfull_at: (6, ...) -> (3, 3, ...) symmetric."""
    xx, yy, zz, xy, xz, yz = Nfull_at
    return np.array([[xx, xy, xz], [xy, yy, yz], [xz, yz, zz]])


def demag_field_direct(M, Nfull, mu0):
    """Brute force: B_i = -mu0 sum_j N(r_i - r_j) M_j.
    M: (3, nz, ny, nx) in A/m.  Nfull from tensor_full."""
    _, nz, ny, nx = M.shape
    B = np.zeros_like(M, dtype=np.float64)
    T = _as_matrix(Nfull)
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                # T index of offset (target - source) for every source cell
                zi = k + nz - 1 - np.arange(nz)
                yi = j + ny - 1 - np.arange(ny)
                xi = i + nx - 1 - np.arange(nx)
                sub = T[np.ix_(range(3), range(3), zi, yi, xi)]
                B[:, k, j, i] = -mu0 * np.einsum("abzyx,bzyx->a", sub, M)
    return B


def padded_size(n):
    """Zero padding used by the oracle: 2n per axis, none for a single cell."""
    return 1 if n == 1 else 2 * n


def demag_kernel_fft(Nfull, shape):
    """Place N(Delta) on the padded periodic grid and transform (complex)."""
    nz, ny, nx = shape
    Pz, Py, Px = padded_size(nz), padded_size(ny), padded_size(nx)
    K = np.zeros((6, Pz, Py, Px))
    for dz in range(-(nz - 1), nz):
        for dy in range(-(ny - 1), ny):
            K[:, dz % Pz, dy % Py, (np.arange(-(nx - 1), nx)) % Px] = \
                Nfull[:, dz + nz - 1, dy + ny - 1, :]
    return np.fft.fftn(K, axes=(1, 2, 3))


def demag_field_fft(M, Kf, mu0):
    """Zero-padded FFT convolution: B = -mu0 * IFFT(K_hat . FFT(M_padded)),
    cropped to the physical grid.  Kf from demag_kernel_fft."""
    _, nz, ny, nx = M.shape
    Pz, Py, Px = Kf.shape[1:]
    Mp = np.zeros((3, Pz, Py, Px))
    Mp[:, :nz, :ny, :nx] = M
    Mf = np.fft.fftn(Mp, axes=(1, 2, 3))
    xx, yy, zz, xy, xz, yz = Kf
    Bf = np.stack([xx * Mf[0] + xy * Mf[1] + xz * Mf[2],
                   xy * Mf[0] + yy * Mf[1] + yz * Mf[2],
                   xz * Mf[0] + yz * Mf[1] + zz * Mf[2]])
    B = np.fft.ifftn(Bf, axes=(1, 2, 3)).real
    return -mu0 * B[:, :nz, :ny, :nx]


def aharoni_prism_factor(a, b, c):
    """Aharoni (J. Appl. Phys. 83, 3432, 1998): demagnetising factor along z
    of a uniformly magnetised rectangular prism of edges 2a x 2b x 2c
    (x, y, z).  Independent closed form used to pin the tensor."""
    r = math.sqrt(a * a + b * b + c * c)
    ab = math.sqrt(a * a + b * b)
    bc = math.sqrt(b * b + c * c)
    ac = math.sqrt(a * a + c * c)
    t = ((b * b - c * c) / (2 * b * c) * math.log((r - a) / (r + a))
         + (a * a - c * c) / (2 * a * c) * math.log((r - b) / (r + b))
         + b / (2 * c) * math.log((ab + a) / (ab - a))
         + a / (2 * c) * math.log((ab + b) / (ab - b))
         + c / (2 * a) * math.log((bc - b) / (bc + b))
         + c / (2 * b) * math.log((ac - a) / (ac + a))
         + 2 * math.atan(a * b / (c * r))
         + (a ** 3 + b ** 3 - 2 * c ** 3) / (3 * a * b * c)
         + (a * a + b * b - 2 * c * c) / (3 * a * b * c) * r
         + c / (a * b) * (ac + bc)
         - (ab ** 3 + bc ** 3 + ac ** 3) / (3 * a * b * c))
    return t / math.pi
