// Stage kernels of the cavity-coupled LLG right-hand side and Runge-Kutta
// integration on gfx950.
//
// One right-hand-side evaluation (one Runge-Kutta stage) is three kernels:
//   k_xfwd   : Ms * y_s -> real-to-complex FFT along x of the zero-padded
//              rows (two real rows per complex transform), written
//              transposed into the half spectrum; also the FP64 partial sums
//              of F = sum_i Ms_i m_i . B_rms, finished by the last workgroup,
//              which advances the cavity amplitude to the next stage.
//   k_yspec  : per kx column, FFT along y, symmetric 3x3 demag-kernel
//              product with the z offsets summed directly, inverse FFT
//              along y, stored back in place (pruned to the physical rows).
//   k_xfield : inverse complex-to-real FFT along x (physical outputs only)
//              giving B_demag in LDS, then exchange, anisotropy, Zeeman and
//              cavity fields, the LL torque (Eq. (llg) with B_cav in both
//              terms) and the Runge-Kutta epilogue (next stage input, or the
//              renormalised end-of-step state, or the Dormand-Prince error);
//              its last workgroup commits RK4 steps or runs the adaptive
//              step controller.
// k_begin starts a Dormand-Prince attempt (renormalise and commit an
// accepted step, FSAL, form the second stage input) and k_record samples
// the average magnetisation.
#include <hip/hip_runtime.h>
#include <math.h>

#include "llgc_common.hpp"
#include "llgc_fft.hpp"

namespace llgc {

constexpr int VPT = 32;   // complex values per thread in an FFT pass

// ---------------------------------------------------------------- tableaus
// classic RK4
__constant__ double c_rk4_c[5] = {0.0, 0.0, 0.5, 0.5, 1.0};
// Dormand & Prince (1980) RK5(4)7M, 1-based stage index
__constant__ double c_dp_c[8] = {0.0, 0.0, 1.0 / 5, 3.0 / 10, 4.0 / 5,
                                 8.0 / 9, 1.0, 1.0};
__constant__ double c_dp_a[8][7] = {
    {0}, {0},
    {1.0 / 5},
    {3.0 / 40, 9.0 / 40},
    {44.0 / 45, -56.0 / 15, 32.0 / 9},
    {19372.0 / 6561, -25360.0 / 2187, 64448.0 / 6561, -212.0 / 729},
    {9017.0 / 3168, -355.0 / 33, 46732.0 / 5247, 49.0 / 176,
     -5103.0 / 18656},
    {35.0 / 384, 0.0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784,
     11.0 / 84}};
__constant__ double c_dp_e[7] = {
    35.0 / 384 - 5179.0 / 57600, 0.0, 500.0 / 1113 - 7571.0 / 16695,
    125.0 / 192 - 393.0 / 640, -2187.0 / 6784 + 92097.0 / 339200,
    11.0 / 84 - 187.0 / 2100, -1.0 / 40};

__device__ inline double drive_shape(int kind, double w, double t) {
  if (kind == 1) {
    double x = w * t;
    return x == 0.0 ? 1.0 : sin(x) / x;
  }
  if (kind == 2) return cos(w * t);
  return 0.0;
}

__device__ inline double stage_c(const Prm& P, int s) {
  return P.method == 0 ? c_rk4_c[s] : c_dp_c[s];
}

// ------------------------------------------------------------- reductions
__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ inline float wave_max(float v) {
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  return v;
}

// Block-wide sum of NV doubles; result valid in thread 0.
template <int NV>
__device__ inline void block_sum(double (&v)[NV], double* red) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
  __syncthreads();
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < NV; ++k) red[w * NV + k] = v[k];
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double a = 0.0;
      for (int i = 0; i < nw; ++i) a += red[i * NV + k];
      v[k] = a;
    }
  }
}

__device__ inline float block_max(float v, float* red) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  v = wave_max(v);
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    float a = red[0];
    for (int i = 1; i < nw; ++i) a = fmaxf(a, red[i]);
    v = a;
  }
  return v;
}

// Publishes a block's partial results and returns true in the workgroup
// that finished last (all partials then visible to it).
__device__ inline bool last_block(unsigned int* counter, unsigned int nblk,
                                  bool* flag) {
  if (threadIdx.x == 0) {
    __threadfence();
    unsigned int prev = atomicAdd(counter, 1u);
    *flag = (prev == nblk - 1);
  }
  __syncthreads();
  bool last = *flag;
  if (last) __threadfence();
  return last;
}

// ------------------------------------------------------------ cavity stage
// Cavity rate at stage s and the amplitude for stage s+1 (or the end of the
// step / the embedded error).  d alpha/dt = -(i wc + kappa) alpha
// + i (V_c/hbar) F - i eps(t).
__device__ void cavity_stage(const Prm& P, Ctl* c, int s, double F) {
  const double dt = c->dt;
  const double ts = c->t + stage_c(P, s) * dt;
  const double eps = P.camp * drive_shape(P.ckind, P.cw, ts);
  const double ar = c->as_re[s], ai = c->as_im[s];
  const double kr = -P.kappa * ar + P.wc * ai;
  const double ki = -P.wc * ar - P.kappa * ai + P.vc_hbar * F - eps;
  c->ka_re[s] = kr;
  c->ka_im[s] = ki;
  c->F_last = F;
  if (P.method == 0) {
    if (s < 4) {
      const double h = (s == 3 ? 1.0 : 0.5) * dt;
      c->as_re[s + 1] = c->a_re + h * kr;
      c->as_im[s + 1] = c->a_im + h * ki;
    } else {
      c->anext_re = c->a_re + dt / 6.0 *
          (c->ka_re[1] + 2.0 * c->ka_re[2] + 2.0 * c->ka_re[3] + kr);
      c->anext_im = c->a_im + dt / 6.0 *
          (c->ka_im[1] + 2.0 * c->ka_im[2] + 2.0 * c->ka_im[3] + ki);
    }
  } else {
    if (s < 7) {
      double sr = 0.0, si = 0.0;
      for (int j = 1; j <= s; ++j) {
        sr += c_dp_a[s + 1][j - 1] * c->ka_re[j];
        si += c_dp_a[s + 1][j - 1] * c->ka_im[j];
      }
      c->as_re[s + 1] = c->a_re + dt * sr;
      c->as_im[s + 1] = c->a_im + dt * si;
    } else {
      double er = 0.0, ei = 0.0;
      for (int j = 1; j <= 7; ++j) {
        er += c_dp_e[j - 1] * c->ka_re[j];
        ei += c_dp_e[j - 1] * c->ka_im[j];
      }
      const double amag = sqrt(c->as_re[7] * c->as_re[7] +
                               c->as_im[7] * c->as_im[7]);
      c->err_a = dt * sqrt(er * er + ei * ei) / fmax(1.0, amag);
    }
  }
}

// ================================================================== k_xfwd
// grid (ceil(ny/R), nz); LDS: (R/2) * Px complex.  mode 0: integrate
// (cavity stage in the last block), mode 1: evaluate (store rate only).
template <int T>
__global__ __launch_bounds__(T) void k_xfwd(
    Prm P, const float* __restrict__ ys, float2* __restrict__ spec,
    Ctl* __restrict__ ctl, double* __restrict__ partials, int stage, int R,
    const float2* __restrict__ tw, int logTw, int mode) {
  extern __shared__ float2 lds[];
  __shared__ double red[16 * 1];
  __shared__ bool amlast;
  if (ctl->done) return;
  const int z = blockIdx.y;
  const int y0 = blockIdx.x * R;
  const int np = (R + 1) >> 1;
  const int Px = P.Px, nx = P.nx, ny = P.ny, N = P.ncell;
  const int plane = nx * ny;
  const double br[3] = {P.brxd, P.bryd, P.brzd};
  double facc[1] = {0.0};
  for (int c = 0; c < 3; ++c) {
    const float* yc = ys + (size_t)c * N + (size_t)z * plane;
    // load pairs (row y0+2p as real part, y0+2p+1 as imaginary part);
    // the coupling sum takes the exact FP64 products Ms_i m_i B_rms
    const int tot = np * Px;
    double fc = 0.0;
    for (int e = threadIdx.x; e < tot; e += T) {
      const int p = e / Px, x = e - p * Px;
      float2 v = make_float2(0.f, 0.f);
      if (x < nx) {
        const int ya = y0 + 2 * p, yb = ya + 1;
        if (ya < ny && 2 * p < R) {
          const int i = ya * nx + x;
          const float msv = P.ms_map ? P.ms_map[z * plane + i] : P.ms;
          const float mv = yc[i];
          v.x = msv * mv;
          fc += (double)msv * (double)mv;
        }
        if (yb < ny && 2 * p + 1 < R) {
          const int i = yb * nx + x;
          const float msv = P.ms_map ? P.ms_map[z * plane + i] : P.ms;
          const float mv = yc[i];
          v.y = msv * mv;
          fc += (double)msv * (double)mv;
        }
      }
      if (P.demag) lds[e] = v;
    }
    facc[0] += fc * br[c];
    if (!P.demag) continue;
    __syncthreads();
    fft_lds<VPT>(lds, P.logPx, np, tw, logTw, -1.f);
    // split the two real transforms and write the half spectrum
    const int H = P.Hx;
    const int totw = np * H;
    for (int e = threadIdx.x; e < totw; e += T) {
      const int k = e / np, p = e - k * np;
      const float2 z1 = lds[p * Px + k];
      const float2 z2 = lds[p * Px + ((Px - k) & (Px - 1))];
      // A = (Z[k] + conj Z[-k]) / 2 ; B = (Z[k] - conj Z[-k]) / (2i)
      const float2 A = make_float2(0.5f * (z1.x + z2.x), 0.5f * (z1.y - z2.y));
      const float2 B = make_float2(0.5f * (z1.y + z2.y), -0.5f * (z1.x - z2.x));
      const int ya = y0 + 2 * p;
      float2* row = spec + ((size_t)(k * P.nz + z) * 3 + c) * ny;
      if (ya < ny && 2 * p < R) row[ya] = A;
      if (ya + 1 < ny && 2 * p + 1 < R) row[ya + 1] = B;
    }
    __syncthreads();
  }
  block_sum<1>(facc, red);
  const unsigned int nblk = gridDim.x * gridDim.y;
  const unsigned int bid = blockIdx.y * gridDim.x + blockIdx.x;
  if (threadIdx.x == 0) partials[bid] = facc[0];
  if (last_block(&ctl->cnt_xfwd, nblk, &amlast)) {
    if (threadIdx.x == 0) {
      double F = 0.0;
      for (unsigned int i = 0; i < nblk; ++i) F += partials[i];
      if (mode == 0) {
        cavity_stage(P, ctl, stage, F);
      } else {
        // evaluate: rate at (a_s, F, t) with s = 1
        const double ts = ctl->t;
        const double eps = P.camp * drive_shape(P.ckind, P.cw, ts);
        const double ar = ctl->as_re[1], ai = ctl->as_im[1];
        ctl->rhs_dadt_re = -P.kappa * ar + P.wc * ai;
        ctl->rhs_dadt_im = -P.wc * ar - P.kappa * ai + P.vc_hbar * F - eps;
        ctl->F_last = F;
      }
      ctl->cnt_xfwd = 0;
    }
  }
}

// ================================================================= k_yspec
// grid ceil(Hx/W); LDS: W * nz * 3 * Py complex.  Kernel layout
// K[kx][ky][comp][dz] (comp: xx yy zz xy xz yz; xz, yz coefficients of -i),
// ky in [0, Py/2]; scaled by -mu0/(Px Py).
template <int T, int NZ>
__global__ __launch_bounds__(T) void k_yspec(
    Prm P, float2* __restrict__ spec, const float* __restrict__ K,
    const Ctl* __restrict__ ctl, int W, const float2* __restrict__ tw,
    int logTw) {
  extern __shared__ float2 lds[];
  if (ctl->done) return;
  const int kx0 = blockIdx.x * W;
  const int Wb = min(W, P.Hx - kx0);
  const int ny = P.ny, Py = P.Py;
  constexpr int nz = NZ;
  const int ncol = Wb * nz * 3;
  // load physical rows, zero the padding
  const int tot = ncol * Py;
  const float2* src = spec + (size_t)kx0 * nz * 3 * ny;
  for (int e = threadIdx.x; e < tot; e += T) {
    const int col = e >> P.logPy, y = e & (Py - 1);
    lds[e] = (y < ny) ? src[(size_t)col * ny + y] : make_float2(0.f, 0.f);
  }
  __syncthreads();
  fft_lds<VPT>(lds, P.logPy, ncol, tw, logTw, -1.f);
  // pointwise product: per (w, ky), all 3*nz values
  constexpr int nz3 = 3 * NZ;
  const int Hy = P.Hy;
  for (int e = threadIdx.x; e < Wb * Py; e += T) {
    const int w = e / Py, ky = e - w * Py;
    const int kx = kx0 + w;
    const bool lo = ky <= (Py >> 1);
    const int kyi = lo ? ky : Py - ky;
    const float sy = lo ? 1.f : -1.f;   // odd-in-ky components flip
    const float* Kp = K + ((size_t)kx * Hy + kyi) * 6 * nz;
    float2 M[nz3], Hf[nz3];
#pragma unroll
    for (int q = 0; q < nz3; ++q) {
      M[q] = lds[(size_t)(w * nz3 + q) * Py + ky];
      Hf[q] = make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int zt = 0; zt < nz; ++zt) {
#pragma unroll
      for (int zs = 0; zs < nz; ++zs) {
        const int d = zt - zs;
        const int ad = d < 0 ? -d : d;
        const float sz = d < 0 ? -1.f : 1.f;   // xz, yz odd in dz
        const float kxx = Kp[0 * nz + ad], kyy = Kp[1 * nz + ad];
        const float kzz = Kp[2 * nz + ad], kxy = sy * Kp[3 * nz + ad];
        const float qxz = sz * Kp[4 * nz + ad];          // K_xz = -i qxz
        const float qyz = sz * sy * Kp[5 * nz + ad];     // K_yz = -i qyz
        const float2 mx = M[zs * 3 + 0], my = M[zs * 3 + 1],
                     mz = M[zs * 3 + 2];
        // -i q * v = (q v.y, -q v.x)
        float2& hx = Hf[zt * 3 + 0];
        float2& hy = Hf[zt * 3 + 1];
        float2& hz = Hf[zt * 3 + 2];
        hx.x += kxx * mx.x + kxy * my.x + qxz * mz.y;
        hx.y += kxx * mx.y + kxy * my.y - qxz * mz.x;
        hy.x += kxy * mx.x + kyy * my.x + qyz * mz.y;
        hy.y += kxy * mx.y + kyy * my.y - qyz * mz.x;
        hz.x += qxz * mx.y + qyz * my.y + kzz * mz.x;
        hz.y += -qxz * mx.x - qyz * my.x + kzz * mz.y;
      }
    }
#pragma unroll
    for (int q = 0; q < nz3; ++q) lds[(size_t)(w * nz3 + q) * Py + ky] = Hf[q];
  }
  __syncthreads();
  fft_lds<VPT>(lds, P.logPy, ncol, tw, logTw, 1.f);
  float2* dst = spec + (size_t)kx0 * nz * 3 * ny;
  const int totw = ncol * ny;
  for (int e = threadIdx.x; e < totw; e += T) {
    const int col = e / ny, y = e - col * ny;
    dst[e] = lds[(size_t)col * Py + y];
  }
}

// ================================================================ k_xfield
// grid (ceil(ny/R), nz); LDS: 3 * (R/2) * Px complex.
template <int T>
__global__ __launch_bounds__(T) void k_xfield(
    Prm P, const float* __restrict__ ys, const float2* __restrict__ spec,
    Ctl* __restrict__ ctl, double* __restrict__ partials,
    double* __restrict__ rec, int stage, int R, Epi E,
    const float2* __restrict__ tw, int logTw) {
  extern __shared__ float2 lds[];
  __shared__ double red[16 * 3];
  __shared__ float redf[16];
  __shared__ bool amlast;
  if (ctl->done) return;
  const int z = blockIdx.y;
  const int y0 = blockIdx.x * R;
  const int np = (R + 1) >> 1;
  const int Px = P.Px, nx = P.nx, ny = P.ny, nz = P.nz, N = P.ncell;
  const int plane = nx * ny;
  if (P.demag) {
    // rebuild the two-for-one spectra: Z[k] = A[k] + i B[k],
    // Z[Px-k] = conj(A[k]) + i conj(B[k])
    const int H = P.Hx;
    const int tot = 3 * np * H;
    for (int e = threadIdx.x; e < tot; e += T) {
      const int k = e / (3 * np);
      const int r = e - k * 3 * np;
      const int c = r / np, p = r - c * np;
      const int ya = y0 + 2 * p;
      const float2* row = spec + ((size_t)(k * nz + z) * 3 + c) * ny;
      float2 A = make_float2(0.f, 0.f), B = make_float2(0.f, 0.f);
      if (ya < ny && 2 * p < R) A = row[ya];
      if (ya + 1 < ny && 2 * p + 1 < R) B = row[ya + 1];
      if (k == 0 || 2 * k == Px) { A.y = 0.f; B.y = 0.f; }
      float2* s = lds + (size_t)(c * np + p) * Px;
      s[k] = make_float2(A.x - B.y, A.y + B.x);
      if (k != 0 && 2 * k != Px)
        s[Px - k] = make_float2(A.x + B.y, -A.y + B.x);
    }
    __syncthreads();
    fft_lds<VPT>(lds, P.logPx, 3 * np, tw, logTw, 1.f);
  }
  const double dtd = ctl->dt;
  const float dt = (float)dtd;
  const double ts = ctl->t + stage_c(P, stage) * dtd;
  const float fd = (float)(P.famp * drive_shape(P.fkind, P.fw, ts));
  const float bex = P.bx + fd * P.fdx, bey = P.by + fd * P.fdy,
              bez = P.bz + fd * P.fdz;
  const float gcav = (float)(2.0 * ctl->as_re[stage]);
  const float bcx = P.brx * gcav, bcy = P.bry * gcav, bcz = P.brz * gcav;
  double acc[3] = {0.0, 0.0, 0.0};
  float emax = 0.f;
  const int ncellb = R * nx;
  for (int e = threadIdx.x; e < ncellb; e += T) {
    const int r = e / nx, x = e - r * nx;
    const int y = y0 + r;
    if (y >= ny) continue;
    const int i = (z * ny + y) * nx + x;
    const float mx = ys[i], my = ys[N + i], mz = ys[2 * N + i];
    const float msv = P.ms_map ? P.ms_map[i] : P.ms;
    float Bx = bex + bcx, By = bey + bcy, Bz = bez + bcz;
    if (P.demag) {
      const int p = r >> 1;
      const bool hi = r & 1;
      const float2 vx = lds[(size_t)(0 * np + p) * Px + x];
      const float2 vy = lds[(size_t)(1 * np + p) * Px + x];
      const float2 vz = lds[(size_t)(2 * np + p) * Px + x];
      Bx += hi ? vx.y : vx.x;
      By += hi ? vy.y : vy.x;
      Bz += hi ? vz.y : vz.x;
    }
    if (msv > 0.f) {
      // exchange: (2A/Ms) sum over existing neighbours (m_j - m_i)/d^2
      float lx = 0.f, ly = 0.f, lz = 0.f;
      if (x > 0) { lx += (ys[i - 1] - mx) * P.idx2; ly += (ys[N + i - 1] - my) * P.idx2; lz += (ys[2 * N + i - 1] - mz) * P.idx2; }
      if (x < nx - 1) { lx += (ys[i + 1] - mx) * P.idx2; ly += (ys[N + i + 1] - my) * P.idx2; lz += (ys[2 * N + i + 1] - mz) * P.idx2; }
      if (y > 0) { lx += (ys[i - nx] - mx) * P.idy2; ly += (ys[N + i - nx] - my) * P.idy2; lz += (ys[2 * N + i - nx] - mz) * P.idy2; }
      if (y < ny - 1) { lx += (ys[i + nx] - mx) * P.idy2; ly += (ys[N + i + nx] - my) * P.idy2; lz += (ys[2 * N + i + nx] - mz) * P.idy2; }
      if (z > 0) { lx += (ys[i - plane] - mx) * P.idz2; ly += (ys[N + i - plane] - my) * P.idz2; lz += (ys[2 * N + i - plane] - mz) * P.idz2; }
      if (z < nz - 1) { lx += (ys[i + plane] - mx) * P.idz2; ly += (ys[N + i + plane] - my) * P.idz2; lz += (ys[2 * N + i + plane] - mz) * P.idz2; }
      const float ce = P.aex2 / msv;
      Bx += ce * lx; By += ce * ly; Bz += ce * lz;
      // uniaxial anisotropy (2 Ku / Ms) (u.m) u
      const float kuv = P.ku_map ? 2.f * P.ku_map[i] : P.ku2;
      const float ca = kuv / msv * (P.ux * mx + P.uy * my + P.uz * mz);
      Bx += ca * P.ux; By += ca * P.uy; Bz += ca * P.uz;
    }
    // LL torque: -gamma/(1+a^2) [ m x B + a m x (m x B) ]
    const float px = my * Bz - mz * By;
    const float py = mz * Bx - mx * Bz;
    const float pz = mx * By - my * Bx;
    const float qx = my * pz - mz * py;
    const float qy = mz * px - mx * pz;
    const float qz = mx * py - my * px;
    const float kx = P.gpref * (px + P.alpha * qx);
    const float ky = P.gpref * (py + P.alpha * qy);
    const float kz = P.gpref * (pz + P.alpha * qz);
    if (E.kout) { E.kout[i] = kx; E.kout[N + i] = ky; E.kout[2 * N + i] = kz; }
    if (E.kind == 0) {
      if (E.bout) { E.bout[i] = Bx; E.bout[N + i] = By; E.bout[2 * N + i] = Bz; }
      continue;
    }
    float sx = E.cself * kx, sy = E.cself * ky, sz = E.cself * kz;
    for (int j = 0; j < E.np; ++j) {
      const float cj = E.ca[j];
      sx += cj * E.kp[j][i];
      sy += cj * E.kp[j][N + i];
      sz += cj * E.kp[j][2 * N + i];
    }
    if (E.kind == 3) {
      const float ex = dt * sx, ey = dt * sy, ez = dt * sz;
      emax = fmaxf(emax, sqrtf(ex * ex + ey * ey + ez * ez));
      continue;
    }
    float nxv = E.yn[i] + dt * sx, nyv = E.yn[N + i] + dt * sy,
          nzv = E.yn[2 * N + i] + dt * sz;
    if (E.kind == 2) {
      const float inv = 1.f / sqrtf(nxv * nxv + nyv * nyv + nzv * nzv);
      nxv *= inv; nyv *= inv; nzv *= inv;
      acc[0] += nxv; acc[1] += nyv; acc[2] += nzv;
    }
    E.ynext[i] = nxv; E.ynext[N + i] = nyv; E.ynext[2 * N + i] = nzv;
  }
  if (E.kind != 2 && E.kind != 3) return;
  const unsigned int nblk = gridDim.x * gridDim.y;
  const unsigned int bid = blockIdx.y * gridDim.x + blockIdx.x;
  if (E.kind == 2) {
    block_sum<3>(acc, red);
    if (threadIdx.x == 0) {
      partials[3 * bid + 0] = acc[0];
      partials[3 * bid + 1] = acc[1];
      partials[3 * bid + 2] = acc[2];
    }
  } else {
    emax = block_max(emax, redf);
    if (threadIdx.x == 0) partials[bid] = (double)emax;
  }
  if (!last_block(&ctl->cnt_field, nblk, &amlast)) return;
  if (threadIdx.x != 0) return;
  Ctl* c = ctl;
  if (E.kind == 2) {
    // RK4 commit and record
    c->t = c->t + c->dt;
    c->a_re = c->anext_re;
    c->a_im = c->anext_im;
    c->as_re[1] = c->a_re;
    c->as_im[1] = c->a_im;
    c->accepted += 1;
    double s0 = 0, s1 = 0, s2 = 0;
    for (unsigned int b = 0; b < nblk; ++b) {
      s0 += partials[3 * b];
      s1 += partials[3 * b + 1];
      s2 += partials[3 * b + 2];
    }
    if (!(isfinite(s0) && isfinite(s1) && isfinite(s2))) {
      c->status = ST_NONFINITE;
      c->done = 1;
    }
    if (c->rec_every > 0 && (c->accepted % c->rec_every) == 0 &&
        c->nrec < c->rec_cap) {
      double* row = rec + 6 * (size_t)c->nrec;
      row[0] = c->t;
      row[1] = s0 / N;
      row[2] = s1 / N;
      row[3] = s2 / N;
      row[4] = c->a_re;
      row[5] = c->a_im;
      c->nrec += 1;
    }
  } else {
    // Dormand-Prince step controller
    double errm = 0.0;
    for (unsigned int b = 0; b < nblk; ++b) errm = fmax(errm, partials[b]);
    double err = fmax(errm, c->err_a);
    bool bad = !isfinite(err) || !isfinite(errm);
    for (unsigned int b = 0; b < nblk && !bad; ++b)
      if (!isfinite(partials[b])) bad = true;
    const double h = c->dt;
    double fac;
    if (!bad && err <= P.tol) {
      fac = (err == 0.0) ? 5.0 : fmin(5.0, fmax(0.2, 0.9 * pow(P.tol / err, 0.2)));
      if (c->prev_rej) fac = fmin(fac, 1.0);
      c->t = c->t + h;
      c->a_re = c->as_re[7];
      c->a_im = c->as_im[7];
      c->as_re[1] = c->a_re;
      c->as_im[1] = c->a_im;
      c->ka_re[1] = c->ka_re[7];
      c->ka_im[1] = c->ka_im[7];
      c->accepted += 1;
      c->pending_accept = 1;
      c->prev_rej = 0;
    } else {
      fac = bad ? 0.2 : fmax(0.2, 0.9 * pow(P.tol / err, 0.2));
      c->prev_rej = 1;
      c->rejected += 1;
      c->pending_accept = 0;
      if (bad) c->status = ST_NONFINITE;
    }
    c->last_err = bad ? INFINITY : err;
    double dtn = fmin(P.dt_max, h * fac);
    if (c->t >= c->t_end || c->accepted >= c->max_accepted) c->done = 1;
    if (!bad) c->status = ST_OK;
    if (dtn < P.dt_min) {
      if (!bad) c->status = ST_UNDERFLOW;
      c->done = 1;
    }
    if (!c->done) dtn = fmin(dtn, c->t_end - c->t);
    c->dt = dtn;
    // second stage amplitude of the next attempt
    c->as_re[2] = c->a_re + dtn * c_dp_a[2][0] * c->ka_re[1];
    c->as_im[2] = c->a_im + dtn * c_dp_a[2][0] * c->ka_im[1];
  }
  c->cnt_field = 0;
}

// ================================================================= k_begin
// Start of a Dormand-Prince attempt: commit an accepted step (renormalise
// y7 into y_n, FSAL k7 -> k1, record), form y2 = y_n + dt a21 k1.
template <int T>
__global__ __launch_bounds__(T) void k_begin(
    Prm P, float* __restrict__ yn, float* __restrict__ k1,
    const float* __restrict__ y7, const float* __restrict__ k7,
    float* __restrict__ y2, Ctl* __restrict__ ctl,
    double* __restrict__ partials, double* __restrict__ rec) {
  __shared__ double red[16 * 3];
  __shared__ bool amlast;
  const int pend = ctl->pending_accept;
  if (ctl->done && !pend) return;
  const int N = P.ncell;
  const float c21 = (float)(ctl->dt * c_dp_a[2][0]);
  double acc[3] = {0.0, 0.0, 0.0};
  for (int i = blockIdx.x * T + threadIdx.x; i < N; i += gridDim.x * T) {
    float mx, my, mz, kx, ky, kz;
    if (pend) {
      mx = y7[i]; my = y7[N + i]; mz = y7[2 * N + i];
      const float inv = 1.f / sqrtf(mx * mx + my * my + mz * mz);
      mx *= inv; my *= inv; mz *= inv;
      yn[i] = mx; yn[N + i] = my; yn[2 * N + i] = mz;
      kx = k7[i]; ky = k7[N + i]; kz = k7[2 * N + i];
      k1[i] = kx; k1[N + i] = ky; k1[2 * N + i] = kz;
      acc[0] += mx; acc[1] += my; acc[2] += mz;
    } else {
      mx = yn[i]; my = yn[N + i]; mz = yn[2 * N + i];
      kx = k1[i]; ky = k1[N + i]; kz = k1[2 * N + i];
    }
    if (!ctl->done) {
      y2[i] = mx + c21 * kx; y2[N + i] = my + c21 * ky;
      y2[2 * N + i] = mz + c21 * kz;
    }
  }
  if (!pend) return;
  block_sum<3>(acc, red);
  if (threadIdx.x == 0) {
    partials[3 * blockIdx.x + 0] = acc[0];
    partials[3 * blockIdx.x + 1] = acc[1];
    partials[3 * blockIdx.x + 2] = acc[2];
  }
  if (!last_block(&ctl->cnt_begin, gridDim.x, &amlast)) return;
  if (threadIdx.x != 0) return;
  double s0 = 0, s1 = 0, s2 = 0;
  for (unsigned int b = 0; b < gridDim.x; ++b) {
    s0 += partials[3 * b];
    s1 += partials[3 * b + 1];
    s2 += partials[3 * b + 2];
  }
  if (ctl->rec_every > 0 && (ctl->accepted % ctl->rec_every) == 0 &&
      ctl->nrec < ctl->rec_cap) {
    double* row = rec + 6 * (size_t)ctl->nrec;
    row[0] = ctl->t;
    row[1] = s0 / N;
    row[2] = s1 / N;
    row[3] = s2 / N;
    row[4] = ctl->a_re;
    row[5] = ctl->a_im;
    ctl->nrec += 1;
  }
  ctl->pending_accept = 0;
  ctl->cnt_begin = 0;
}

// ================================================================ k_record
// Average magnetisation of `m` written as one record row (t, <m>, a).
template <int T>
__global__ __launch_bounds__(T) void k_record(
    Prm P, const float* __restrict__ m, Ctl* __restrict__ ctl,
    double* __restrict__ partials, double* __restrict__ rec) {
  __shared__ double red[16 * 3];
  __shared__ bool amlast;
  const int N = P.ncell;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int i = blockIdx.x * T + threadIdx.x; i < N; i += gridDim.x * T) {
    acc[0] += m[i];
    acc[1] += m[N + i];
    acc[2] += m[2 * N + i];
  }
  block_sum<3>(acc, red);
  if (threadIdx.x == 0) {
    partials[3 * blockIdx.x + 0] = acc[0];
    partials[3 * blockIdx.x + 1] = acc[1];
    partials[3 * blockIdx.x + 2] = acc[2];
  }
  if (!last_block(&ctl->cnt_rec, gridDim.x, &amlast)) return;
  if (threadIdx.x != 0) return;
  double s0 = 0, s1 = 0, s2 = 0;
  for (unsigned int b = 0; b < gridDim.x; ++b) {
    s0 += partials[3 * b];
    s1 += partials[3 * b + 1];
    s2 += partials[3 * b + 2];
  }
  if (ctl->nrec < ctl->rec_cap) {
    double* row = rec + 6 * (size_t)ctl->nrec;
    row[0] = ctl->t;
    row[1] = s0 / N;
    row[2] = s1 / N;
    row[3] = s2 / N;
    row[4] = ctl->a_re;
    row[5] = ctl->a_im;
    ctl->nrec += 1;
  }
  ctl->cnt_rec = 0;
}

}  // namespace llgc
