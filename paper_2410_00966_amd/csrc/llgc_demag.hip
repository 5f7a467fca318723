// Demagnetising-kernel setup on the device, in float64 (once per grid).
//
// The demag field of uniformly magnetised box cells is a convolution with
// the cell-averaged tensor N(Delta) (demagnetisation is one of the
// effective-field contributions of the finite-difference LLG, section
// "The LLG equation in Mumax3").  N(Delta) is the double volume average of
// the point-dipole kernel over a target and a source box:
//   * Chebyshev distance <= kNewellCells: Newell, Williams and Dunlop (1993)
//     closed forms f, g with the 27-point sixth-order difference;
//   * beyond: Gauss-Legendre quadrature of the point-dipole kernel over the
//     difference of the two uniform box positions, whose density per axis is
//     the tent (d - |w|)/d^2 on [-d, d] (kGLHalf points per half-axis).
// The zero-padded periodic transform of N over x and y is real for the
// components even in both offsets and purely imaginary or real by parity
// otherwise, so it is built as separable cosine/sine sums of the
// non-negative-offset octant (k_dct_x, k_dct_y) and stored mirror-reduced:
// K[kx][ky][kslot(comp, dz)], kx <= Px/2, ky <= Py/2, comp = xx yy zz xy xz
// yz (xz and yz as coefficients of -i, not stored at dz = 0 where they
// vanish), scaled by -mu0/(Px Py).
#include <hip/hip_runtime.h>
#include <math.h>

namespace llgc {

constexpr int kNewellCells = 7;
constexpr int kGLHalf = 5;
constexpr int kGLNodes = 2 * kGLHalf;

__device__ inline double ratio_asinh(double n, double d) {
  return d > 0.0 ? asinh(n / d) : 0.0;
}
__device__ inline double ratio_atan(double n, double d) {
  return d != 0.0 ? atan(n / d) : 0.0;
}

// Newell f: even in every argument, symmetric in (y, z).
__device__ double newell_f(double x, double y, double z) {
  x = fabs(x); y = fabs(y); z = fabs(z);
  const double x2 = x * x, y2 = y * y, z2 = z * z;
  const double R = sqrt(x2 + y2 + z2);
  double r = (2.0 * x2 - y2 - z2) * R / 6.0;
  if (z2 != x2) r += 0.5 * y * (z2 - x2) * ratio_asinh(y, sqrt(x2 + z2));
  if (y2 != x2) r += 0.5 * z * (y2 - x2) * ratio_asinh(z, sqrt(x2 + y2));
  if (x > 0.0) r -= x * y * z * ratio_atan(y * z, x * R);
  return r;
}

// Newell g: odd in x and y, even in z, symmetric in (x, y).
__device__ double newell_g(double x, double y, double z) {
  const double x2 = x * x, y2 = y * y, z2 = z * z;
  const double R = sqrt(x2 + y2 + z2);
  double r = -x * y * R / 3.0;
  r += x * y * z * ratio_asinh(z, sqrt(x2 + y2));
  r += y / 6.0 * (3.0 * z2 - y2) * ratio_asinh(x, sqrt(y2 + z2));
  r += x / 6.0 * (3.0 * z2 - x2) * ratio_asinh(y, sqrt(x2 + z2));
  r -= z2 * z / 6.0 * ratio_atan(x * y, z * R);
  r -= z * y2 / 2.0 * ratio_atan(x * z, y * R);
  r -= z * x2 / 2.0 * ratio_atan(y * z, x * R);
  return r;
}

template <bool G>
__device__ double stencil27(double X, double Y, double Z, double a, double b,
                            double c) {
  const double w[3] = {-1.0, 2.0, -1.0};
  double acc = 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k) {
        const double x = X + (i - 1) * a, y = Y + (j - 1) * b,
                     z = Z + (k - 1) * c;
        acc += w[i] * w[j] * w[k] * (G ? newell_g(x, y, z) : newell_f(x, y, z));
      }
  return acc;
}

// Gauss-Legendre rule on [-1, 1] (kGLHalf points), filled by the host.
struct GLRule {
  double x[kGLHalf], w[kGLHalf];
};

// N(Delta) at offset (ix, iy, iz) >= 0 for all 6 components.
// out layout: [comp][iz][iy][ix] (octant, float64).
__global__ void k_tensor(double* __restrict__ out, int nx, int ny, int nz,
                         double dx, double dy, double dz, GLRule gl) {
  const int ix = blockIdx.x * blockDim.x + threadIdx.x;
  const int iy = blockIdx.y, iz = blockIdx.z;
  if (ix >= nx) return;
  const size_t n = (size_t)nx * ny * nz;
  const size_t o = ((size_t)iz * ny + iy) * nx + ix;
  const double X = ix * dx, Y = iy * dy, Z = iz * dz;
  double v[6];
  const int cheb = max(ix, max(iy, iz));
  if (cheb <= kNewellCells) {
    const double s = 1.0 / (4.0 * M_PI * dx * dy * dz);
    v[0] = s * stencil27<false>(X, Y, Z, dx, dy, dz);
    v[1] = s * stencil27<false>(Y, X, Z, dy, dx, dz);
    v[2] = s * stencil27<false>(Z, Y, X, dz, dy, dx);
    v[3] = s * stencil27<true>(X, Y, Z, dx, dy, dz);
    v[4] = s * stencil27<true>(X, Z, Y, dx, dz, dy);
    v[5] = s * stencil27<true>(Y, Z, X, dy, dz, dx);
  } else {
    // tent-weighted nodes per axis: both halves of [-d, d]
    double nxs[kGLNodes], wxs[kGLNodes], nys[kGLNodes], wys[kGLNodes],
        nzs[kGLNodes], wzs[kGLNodes];
    for (int q = 0; q < kGLHalf; ++q) {
      const double u = 0.5 * (gl.x[q] + 1.0);       // in [0, 1]
      const double wt = 0.5 * gl.w[q] * (1.0 - u);  // tent density * jacobian
      nxs[q] = u * dx; nxs[kGLHalf + q] = -u * dx;
      nys[q] = u * dy; nys[kGLHalf + q] = -u * dy;
      nzs[q] = u * dz; nzs[kGLHalf + q] = -u * dz;
      wxs[q] = wxs[kGLHalf + q] = wt;
      wys[q] = wys[kGLHalf + q] = wt;
      wzs[q] = wzs[kGLHalf + q] = wt;
    }
    for (int c = 0; c < 6; ++c) v[c] = 0.0;
    const double V = dx * dy * dz;
    for (int a = 0; a < kGLNodes; ++a)
      for (int b = 0; b < kGLNodes; ++b)
        for (int c = 0; c < kGLNodes; ++c) {
          const double x = X + nxs[a], y = Y + nys[b], zz = Z + nzs[c];
          const double r2 = x * x + y * y + zz * zz;
          const double ir2 = 1.0 / r2;
          const double pre = -wxs[a] * wys[b] * wzs[c] * V /
                             (4.0 * M_PI * r2 * sqrt(r2));
          v[0] += pre * (3.0 * x * x * ir2 - 1.0);
          v[1] += pre * (3.0 * y * y * ir2 - 1.0);
          v[2] += pre * (3.0 * zz * zz * ir2 - 1.0);
          v[3] += pre * 3.0 * x * y * ir2;
          v[4] += pre * 3.0 * x * zz * ir2;
          v[5] += pre * 3.0 * y * zz * ir2;
        }
  }
  // components odd in an offset vanish on that zero plane
  if (ix == 0) { v[3] = 0.0; v[4] = 0.0; }
  if (iy == 0) { v[3] = 0.0; v[5] = 0.0; }
  if (iz == 0) { v[4] = 0.0; v[5] = 0.0; }
  for (int c = 0; c < 6; ++c) out[c * n + o] = v[c];
}

// Parity of each component in x and y: cos sums for even, sin for odd.
__device__ inline bool odd_x(int comp) { return comp == 3 || comp == 4; }
__device__ inline bool odd_y(int comp) { return comp == 3 || comp == 5; }

// out1[comp][iz][iy][kx] = sum_ix w(ix) N[comp][iz][iy][ix] trig(2 pi kx ix/Px)
// grid (ceil(Hx/256), ny*nz, 6); tw = (cos, sin)(2 pi m / Px), m < Px.
__global__ void k_dct_x(const double* __restrict__ N, double* __restrict__ o1,
                        int nx, int ny, int nz, int Px, int Hx,
                        const double2* __restrict__ tw) {
  const int kx = blockIdx.x * blockDim.x + threadIdx.x;
  const int row = blockIdx.y, comp = blockIdx.z;
  if (kx >= Hx) return;
  const size_t n = (size_t)nx * ny * nz;
  const double* src = N + comp * n + (size_t)row * nx;
  const bool odd = odd_x(comp);
  double acc = 0.0;
  for (int ix = 0; ix < nx; ++ix) {
    const double2 t = tw[((long long)kx * ix) & (Px - 1)];
    const double wgt = (ix == 0) ? 1.0 : 2.0;
    acc += wgt * src[ix] * (odd ? t.y : t.x);
  }
  o1[((size_t)comp * ny * nz + row) * Hx + kx] = acc;
}

// K[kx][ky][comp][iz] = scale * sgn * sum_iy w(iy) o1[comp][iz][iy][kx] trig
// grid (ceil(Hx/256), Hy, 6*nz)
__global__ void k_dct_y(const double* __restrict__ o1, float* __restrict__ K,
                        int ny, int nz, int Py, int Hx, int Hy,
                        const double2* __restrict__ tw, double scale) {
  const int kx = blockIdx.x * blockDim.x + threadIdx.x;
  const int ky = blockIdx.y;
  const int comp = blockIdx.z / nz, iz = blockIdx.z % nz;
  if (kx >= Hx) return;
  const bool odd = odd_y(comp);
  const double* src = o1 + ((size_t)comp * ny * nz + (size_t)iz * ny) * Hx;
  double acc = 0.0;
  for (int iy = 0; iy < ny; ++iy) {
    const double2 t = tw[((long long)ky * iy) & (Py - 1)];
    const double wgt = (iy == 0) ? 1.0 : 2.0;
    acc += wgt * src[(size_t)iy * Hx + kx] * (odd ? t.y : t.x);
  }
  // xy: both transforms odd -> (-i sin)(-i sin) = -sin sin
  const double sgn = (comp == 3) ? -1.0 : 1.0;
  if (comp >= 4 && iz == 0) return;   // xz, yz vanish at dz = 0
  K[((size_t)kx * Hy + ky) * kentry(nz) + kslot(comp, iz, nz)] =
      (float)(scale * sgn * acc);
}

}  // namespace llgc
