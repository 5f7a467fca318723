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
#include "llgc_wfft.hpp"

namespace llgc {

#ifndef LLGC_VPT
#define LLGC_VPT 16
#endif
#ifndef LLGC_VPTY
#define LLGC_VPTY LLGC_VPT
#endif
// complex values a thread holds in one LDS FFT pass: x-pass kernels, y pass
constexpr int VPT = LLGC_VPT;
constexpr int VPTY = LLGC_VPTY;

// Accesses through a 32-bit unsigned offset from an array's uniform base
// address: the load or store is then the base plus a 32-bit lane offset,
// with no 64-bit address arithmetic per element (every array here stays far
// below 4 GiB: at most 3 x 1024 x 1024 x 4 floats, a half spectrum of about
// 100 MB).  ldf/stf: element i of a float array; ld4/st4: 16 bytes at byte
// offset `off`.
__device__ __forceinline__ float ldf(const float* p, unsigned i) {
  return *(const float*)((const char*)p + (i << 2));
}
__device__ __forceinline__ void stf(float* p, unsigned i, float v) {
  *(float*)((char*)p + (i << 2)) = v;
}
__device__ __forceinline__ float4 ld4(const void* p, unsigned off) {
  return *(const float4*)((const char*)p + off);
}
__device__ __forceinline__ void st4(void* p, unsigned off, float4 v) {
  *(float4*)((char*)p + off) = v;
}

// The Stockham passes of an L-point transform index the twiddle table at
// k * Ltw / (Ns R) < Ltw / 2, so the first half of the table serves every
// pass.  The LDS kernels copy it into the front of their LDS once, so that
// each pass reads its twiddles from LDS rather than from global memory right
// after a barrier.  Returns the entry count (even, so that the data after it
// stays 16-byte aligned).
__host__ __device__ constexpr int lds_twiddles(int logTw) {
  return logTw > 1 ? 1 << (logTw - 1) : 2;
}
// LDS entries ahead of the spectral pass's data: per-pass twiddle tables
// for a compile-time length 2^LP, else the staged half of the plain table.
__host__ __device__ constexpr int yspec_tw_len(int LP, int logTw) {
  return LP > 0 ? fft_tt_len(LLGC_VPTY, true, LP) : lds_twiddles(logTw);
}
__device__ __forceinline__ void stage_twiddles(float2* twl,
                                               const float2* __restrict__ tw,
                                               int logTw) {
  const int n = 1 << (logTw > 0 ? logTw - 1 : 0);
  for (int i = threadIdx.x; i < n; i += blockDim.x) twl[i] = tw[i];
}

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

// ----------------------------------------------------------- thermal field
// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32 -> 64-bit
// products with the Weyl-bumped key; counter (cell, step lo, step hi, 0),
// key (seed lo, seed hi).  The four words become uniforms (w + 1/2) 2^-32
// and, by Box-Muller on (u0, u1) and (u2, u3), normals, of which three are
// Brown's field components (FP64, as the oracle draws them).
__device__ __forceinline__ void thermal_normals(const Prm& P, int cell,
                                                long long step, double& n0,
                                                double& n1, double& n2) {
  unsigned int c0 = (unsigned int)cell, c1 = (unsigned int)step,
               c2 = (unsigned int)((unsigned long long)step >> 32), c3 = 0u;
  unsigned int k0 = P.seed_lo, k1 = P.seed_hi;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const unsigned int lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
    const unsigned int lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
    const unsigned int d0 = hi1 ^ c1 ^ k0, d2 = hi0 ^ c3 ^ k1;
    c0 = d0;
    c1 = lo1;
    c2 = d2;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  const double s = 2.3283064365386963e-10;   // 2^-32
  const double u0 = ((double)c0 + 0.5) * s, u1 = ((double)c1 + 0.5) * s;
  const double u2 = ((double)c2 + 0.5) * s, u3 = ((double)c3 + 0.5) * s;
  const double r0 = sqrt(-2.0 * log(u0)), r1 = sqrt(-2.0 * log(u2));
  const double tp = 6.283185307179586;
  n0 = r0 * cos(tp * u1);
  n1 = r0 * sin(tp * u1);
  n2 = r1 * cos(tp * u3);
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


// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2).  Remap the launch index so that consecutive tiles run on the same
// XCD: neighbouring tiles share spectrum cache lines and exchange halos.
__device__ inline int xcd_tile(int bid, int nblk) {
  const int per = nblk >> 3, rem = nblk & 7;
  const int x = bid & 7, k = bid >> 3;
  return (x < rem) ? x * (per + 1) + k : rem * (per + 1) + (x - rem) * per + k;
}

// Deterministic block-wide sum of NV interleaved partials p[b*NV + k],
// b < n (fixed assignment of partials to threads and fixed tree order).
template <int NV>
__device__ inline void sum_partials(const double* p, unsigned int n,
                                    double (&out)[NV], double* red) {
  double v[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = 0.0;
  for (unsigned int b = threadIdx.x; b < n; b += blockDim.x)
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] += p[(size_t)b * NV + k];
  block_sum<NV>(v, red);
#pragma unroll
  for (int k = 0; k < NV; ++k) out[k] = v[k];
}

__device__ inline double max_partials(const double* p, unsigned int n,
                                      double* red) {
  double v = 0.0;
  bool bad = false;
  for (unsigned int b = threadIdx.x; b < n; b += blockDim.x) {
    const double q = p[b];
    if (!(q == q) || isinf(q)) bad = true;
    v = fmax(v, q);
  }
  if (bad) v = INFINITY;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = red[0];
    for (int i = 1; i < nw; ++i) a = fmax(a, red[i]);
    v = a;
  }
  return v;
}

// ------------------------------------------------------------ cavity stage
// Cavity rate at stage s and the amplitude for stage s+1 (or the end of the
// step / the embedded error).  d alpha/dt = -(i wc + kappa) alpha
// + i (V_c/hbar) F - i eps(t).
__device__ __forceinline__ void cavity_stage(const Prm& P, Ctl* c, int s,
                                             double F) {
  const double dt = c->dt;
  if (P.cmode == 1) {
    // integrated-out cavity (RK4): at the step start alpha_n = alpha^-_n +
    // i (V_c/hbar) F_n dt (no term at the first step after the state was
    // set), held over the four stages; alpha^-_{n+1} = e^{-(i wc+kappa) dt}
    // alpha_n is committed as the end-of-step amplitude
    c->ka_re[s] = 0.0;
    c->ka_im[s] = 0.0;
    c->F_last = F;
    if (s == 1) {
      const double ar = c->as_re[1];
      const double ai = c->as_im[1] + (c->mem_n > 0 ? dt * P.vc_hbar * F : 0.0);
      for (int q = 1; q <= 4; ++q) {
        c->as_re[q] = ar;
        c->as_im[q] = ai;
      }
      const double e = exp(-P.kappa * dt);
      const double cw = cos(P.wc * dt), sw = sin(P.wc * dt);
      c->anext_re = e * (ar * cw + ai * sw);
      c->anext_im = e * (ai * cw - ar * sw);
    }
    return;
  }
  const double ts = c->t + stage_c(P, s) * dt;
  const double eps = P.camp * drive_shape(P.ckind, P.cw, ts);
  const double ar = c->as_re[s], ai = c->as_im[s];
  // the earlier stage rates, loaded together (DP45 sums below)
  double kar[8], kai[8];
#pragma unroll
  for (int j = 1; j <= 7; ++j) {
    kar[j] = c->ka_re[j];
    kai[j] = c->ka_im[j];
  }
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
          (kar[1] + 2.0 * kar[2] + 2.0 * kar[3] + kr);
      c->anext_im = c->a_im + dt / 6.0 *
          (kai[1] + 2.0 * kai[2] + 2.0 * kai[3] + ki);
    }
  } else {
    if (s < 7) {
      double sr = 0.0, si = 0.0;
#pragma unroll
      for (int j = 1; j <= 6; ++j) {
        if (j > s) break;
        sr += c_dp_a[s + 1][j - 1] * (j == s ? kr : kar[j]);
        si += c_dp_a[s + 1][j - 1] * (j == s ? ki : kai[j]);
      }
      c->as_re[s + 1] = c->a_re + dt * sr;
      c->as_im[s + 1] = c->a_im + dt * si;
    } else {
      double er = 0.0, ei = 0.0;
#pragma unroll
      for (int j = 1; j <= 7; ++j) {
        er += c_dp_e[j - 1] * (j == 7 ? kr : kar[j]);
        ei += c_dp_e[j - 1] * (j == 7 ? ki : kai[j]);
      }
      const double amag = sqrt(c->as_re[7] * c->as_re[7] +
                               c->as_im[7] * c->as_im[7]);
      c->err_a = dt * sqrt(er * er + ei * ei) / fmax(1.0, amag);
    }
  }
}

// Multimode cavity (section "Ferromagnetic materials in a cavity": each mode
// of a multimode cavity follows the single-mode equation with its own
// coupling sum F_k = sum_i Ms_i m_i . B_rms,k,i): the stage rates and next
// stage amplitudes of every mode, as cavity_stage does for one.  The DP45
// amplitude error is the 2-norm over the modes relative to
// max(1, |alpha_5|_2).
// (Loops over the modes run to kMaxModes with a guard so that the register
// array F is indexed by constants.)
__device__ __forceinline__ void cavity_stage_modes(
    const Prm& P, Ctl* c, int s, const double (&F)[kMaxModes]) {
  const Modes& M = *P.modes;
  const double dt = c->dt;
  const double ts = c->t + stage_c(P, s) * dt;
#pragma unroll
  for (int k = 0; k < kMaxModes; ++k) {
    if (k >= M.n) break;
    const double eps = M.camp[k] * drive_shape(M.ckind[k], M.cw[k], ts);
    const double ar = c->mas_re[s][k], ai = c->mas_im[s][k];
    c->mka_re[s][k] = -M.kappa[k] * ar + M.wc[k] * ai;
    c->mka_im[s][k] = -M.wc[k] * ar - M.kappa[k] * ai + P.vc_hbar * F[k] - eps;
  }
  c->F_last = F[0];
  if (P.method == 0) {
    for (int k = 0; k < M.n; ++k) {
      if (s < 4) {
        const double h = (s == 3 ? 1.0 : 0.5) * dt;
        c->mas_re[s + 1][k] = c->ma_re[k] + h * c->mka_re[s][k];
        c->mas_im[s + 1][k] = c->ma_im[k] + h * c->mka_im[s][k];
      } else {
        c->manext_re[k] = c->ma_re[k] + dt / 6.0 *
            (c->mka_re[1][k] + 2.0 * c->mka_re[2][k] + 2.0 * c->mka_re[3][k] +
             c->mka_re[4][k]);
        c->manext_im[k] = c->ma_im[k] + dt / 6.0 *
            (c->mka_im[1][k] + 2.0 * c->mka_im[2][k] + 2.0 * c->mka_im[3][k] +
             c->mka_im[4][k]);
      }
    }
    return;
  }
  if (s < 7) {
    for (int k = 0; k < M.n; ++k) {
      double sr = 0.0, si = 0.0;
      for (int j = 1; j <= s; ++j) {
        sr += c_dp_a[s + 1][j - 1] * c->mka_re[j][k];
        si += c_dp_a[s + 1][j - 1] * c->mka_im[j][k];
      }
      c->mas_re[s + 1][k] = c->ma_re[k] + dt * sr;
      c->mas_im[s + 1][k] = c->ma_im[k] + dt * si;
    }
    return;
  }
  double e2 = 0.0, a2 = 0.0;
  for (int k = 0; k < M.n; ++k) {
    double er = 0.0, ei = 0.0;
    for (int j = 1; j <= 7; ++j) {
      er += c_dp_e[j - 1] * c->mka_re[j][k];
      ei += c_dp_e[j - 1] * c->mka_im[j][k];
    }
    e2 += er * er + ei * ei;
    a2 += c->mas_re[7][k] * c->mas_re[7][k] + c->mas_im[7][k] * c->mas_im[7][k];
  }
  c->err_a = dt * sqrt(e2) / fmax(1.0, sqrt(a2));
}

// Amplitude columns of a record row: Re, Im of the mode, or of each mode.
__device__ __forceinline__ void record_amplitudes(const Prm& P, const Ctl* c,
                                                  double* row) {
  if (P.modes) {
    for (int k = 0; k < P.modes->n; ++k) {
      row[4 + 2 * k] = c->ma_re[k];
      row[5 + 2 * k] = c->ma_im[k];
    }
  } else {
    row[4] = c->a_re;
    row[5] = c->a_im;
  }
}

// ================================================================== k_xfwd
// 1D grid of ceil(ny/R)*nz tiles (R even, XCD-remapped; the nz layers of one
// y range are consecutive tiles).  LDS: (R/2) * Px complex.
// mode 0: integrate (cavity stage in the last block); mode 1: evaluate.
// V4: nx % 4 == 0 and 16-byte aligned planes (vector loads).
// LP > 0: log2(Px) fixed at compile time (specialised FFT addressing).
// At most 128 VGPRs (four waves per SIMD): two 512-thread workgroups per CU.
// LDS padding of the forward x pass: 2 slots every 2^kXfPs values
constexpr int kXfPs = 4;
template <int T, bool V4, int LP = 0>
__global__ __launch_bounds__(T) __attribute__((amdgpu_waves_per_eu(4))) void k_xfwd(
    Prm P, const float* __restrict__ ys, float2* __restrict__ spec,
    Ctl* __restrict__ ctl, double* __restrict__ partials, int stage, int R,
    const float2* __restrict__ tw, int logTw, int mode) {
  extern __shared__ float2 lds_all[];
  __shared__ double red[16];
  if (ctl->done) return;
  float2* twl = lds_all;
  float2* lds = lds_all + lds_twiddles(logTw);
  if (P.demag) stage_twiddles(twl, tw, logTw);
  const int nblk = gridDim.x;
  const int tile = xcd_tile(blockIdx.x, nblk);
  const int nz = P.nz;
  const int z = tile % nz;
  const int y0 = (tile / nz) * R;
  const int np = R >> 1;
  const int Px = P.Px, nx = P.nx, ny = P.ny, nyp = P.nyp, N = P.ncell;
  const int plane = nx * ny;
  const double br[3] = {P.brxd, P.bryd, P.brzd};
  double facc[1] = {0.0};
  const float* msz = P.ms_map ? P.ms_map + (size_t)z * plane : nullptr;
  // V4: quads of 4 consecutive x; row pair p: rows y0+2p (re), y0+2p+1
  // (im); x < Px/2 only: the rest is zero padding the first pass does not
  // read.  Quad pair q of component c, and the Ms values it is weighted by:
  const int qpr = Px >> 3;               // quads per half row
  const int nq = np * qpr;
  auto load_qp = [&](int c, int q, float4& va, float4& vb) {
    const int p = q / qpr, x = (q - p * qpr) << 2;
    const int ya = y0 + 2 * p;
    const unsigned o = (unsigned)(c * N + z * plane + ya * nx + x) << 2;
    va = vb = make_float4(0.f, 0.f, 0.f, 0.f);
    if (q < nq && x < nx) {
      if (ya < ny) va = ld4(ys, o);
      if (ya + 1 < ny) vb = ld4(ys, o + ((unsigned)nx << 2));
    }
  };
  auto load_ms = [&](int q, float4& sa, float4& sb) {
    const int p = q / qpr, x = (q - p * qpr) << 2;
    const int ya = y0 + 2 * p;
    const unsigned o = (unsigned)(z * plane + ya * nx + x) << 2;
    sa = sb = make_float4(P.ms, P.ms, P.ms, P.ms);
    if (msz && q < nq && x < nx) {
      if (ya < ny) sa = ld4(P.ms_map, o);
      if (ya + 1 < ny) sb = ld4(P.ms_map, o + ((unsigned)nx << 2));
    }
  };
  // its coupling terms into fc and its products Ms m into the LDS rows
  auto put_qp = [&](int q, const float4& va, const float4& vb,
                    const float4& sa, const float4& sb, double& fc) {
    const int p = q / qpr, x = (q - p * qpr) << 2;
    fc += (double)sa.x * va.x + (double)sa.y * va.y + (double)sa.z * va.z +
          (double)sa.w * va.w + (double)sb.x * vb.x + (double)sb.y * vb.y +
          (double)sb.z * vb.z + (double)sb.w * vb.w;
    if (P.demag) {
      const int li = p * Px + x;
      *(float4*)(lds + pidx_s<kXfPs>(li)) = make_float4(sa.x * va.x, sb.x * vb.x,
                                               sa.y * va.y, sb.y * vb.y);
      *(float4*)(lds + pidx_s<kXfPs>(li + 2)) = make_float4(sa.z * va.z, sb.z * vb.z,
                                                   sa.w * va.w, sb.w * vb.w);
    }
  };
  // the thread's first quad pair of the next component is loaded while the
  // current component is transformed (registers nva, nvb)
  float4 nva, nvb;
  if (V4) load_qp(0, threadIdx.x, nva, nvb);
  for (int c = 0; c < 3; ++c) {
    const float* yc = ys + (size_t)c * N + (size_t)z * plane;
    double fc = 0.0;
    if (V4) {
      if ((int)threadIdx.x < nq) {
        float4 sa, sb;
        load_ms(threadIdx.x, sa, sb);
        put_qp(threadIdx.x, nva, nvb, sa, sb, fc);
      }
      // the remaining quad pairs, U per batch
      constexpr int U = 2;
      for (int q0 = threadIdx.x + T; q0 < nq; q0 += T * U) {
        float4 va[U], vb[U], sa[U], sb[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          load_qp(c, q0 + u * T, va[u], vb[u]);
          load_ms(q0 + u * T, sa[u], sb[u]);
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
          if (q0 + u * T < nq) put_qp(q0 + u * T, va[u], vb[u], sa[u], sb[u], fc);
      }
    } else {
      const int xl = Px > 1 ? Px >> 1 : 1;   // lower half of the row
      const int tot = np * xl;
      for (int e = threadIdx.x; e < tot; e += T) {
        const int p = e / xl, x = e - p * xl;
        float2 v = make_float2(0.f, 0.f);
        if (x < nx) {
          const int ya = y0 + 2 * p;
          if (ya < ny) {
            const float msv = msz ? msz[ya * nx + x] : P.ms;
            const float mv = yc[ya * nx + x];
            v.x = msv * mv;
            fc += (double)msv * (double)mv;
          }
          if (ya + 1 < ny) {
            const float msv = msz ? msz[(ya + 1) * nx + x] : P.ms;
            const float mv = yc[(ya + 1) * nx + x];
            v.y = msv * mv;
            fc += (double)msv * (double)mv;
          }
        }
        if (P.demag) lds[pidx_s<kXfPs>(p * Px + x)] = v;
      }
    }
    facc[0] += fc * br[c];
    if (!P.demag) {
      if (V4 && c < 2) load_qp(c + 1, threadIdx.x, nva, nvb);
      continue;
    }
    __syncthreads();
    if (V4 && c < 2) load_qp(c + 1, threadIdx.x, nva, nvb);
    // thread index through an opaque copy: the transform's address
    // arithmetic is formed per component, not held across the loop
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    fft_lds<VPT, true, LP, true, false, kXfPs>(lds, P.logPx, np, twl, logTw, -1.f,
                                        tid);
    // split the two real transforms and write the half spectrum: rows
    // (y0+2p, y0+2p+1) are adjacent -> one 16-byte store per (kx, p)
    const int H = P.Hx;
    const int totw = np * H;
    // e = k np + p advanced by T without a division per element
    const int dk = T / np, dp = T - dk * np;
    int k = threadIdx.x / np, p = threadIdx.x - k * np;
    for (int e = threadIdx.x; e < totw;
         e += T, k += dk, p += dp, (p >= np ? (p -= np, ++k) : 0)) {
      const float2 z1 = lds[pidx_s<kXfPs>(p * Px + k)];
      const float2 z2 = lds[pidx_s<kXfPs>(p * Px + ((Px - k) & (Px - 1)))];
      // A = (Z[k] + conj Z[-k]) / 2 ; B = (Z[k] - conj Z[-k]) / (2i)
      const float4 AB = make_float4(0.5f * (z1.x + z2.x), 0.5f * (z1.y - z2.y),
                                    0.5f * (z1.y + z2.y), -0.5f * (z1.x - z2.x));
      const int ya = y0 + 2 * p;
      if (ya < ny) {
        float4 v = AB;
        if (ya + 1 >= ny) { v.z = 0.f; v.w = 0.f; }   // keep the pad zero
        st4(spec, (unsigned)(((k * nz + z) * 3 + c) * nyp + ya) << 3, v);
      }
    }
    __syncthreads();
  }
  block_sum<1>(facc, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = facc[0];
}

// ================================================================= k_xfwd3
// Forward x pass of the batch plan: the 3 components x (R/2) row pairs of a
// tile are transformed together in LDS (3 (R/2) Px complex), so short rows
// still fill the workgroup; partial sums indexed by tile.
template <int T>
__device__ __forceinline__ void xfwd3_body(
    const Prm& P, const float* __restrict__ ys, float2* __restrict__ spec,
    double* __restrict__ partials, int R, const float2* __restrict__ tw,
    int logTw, int tile, int slot, float2* lds_all) {
  __shared__ double red[16];
  float2* twl = lds_all;
  float2* lds = lds_all + lds_twiddles(logTw);
  if (P.demag) stage_twiddles(twl, tw, logTw);
  const int nz = P.nz;
  const int z = tile % nz;
  const int y0 = (tile / nz) * R;
  const int np = R >> 1;
  const int Px = P.Px, nx = P.nx, ny = P.ny, nyp = P.nyp, N = P.ncell;
  const int plane = nx * ny;
  const float* msz = P.ms_map ? P.ms_map + (size_t)z * plane : nullptr;
  // rows y0+2p (real part) and y0+2p+1 (imaginary part), x < Px/2 only:
  // the rest is zero padding the first pass does not read
  const int xl = Px > 1 ? Px >> 1 : 1;
  const int per = np * xl;
  double facc[1] = {0.0};   // sum of Ms m . B_rms over the tile
  for (int e = threadIdx.x; e < 3 * per; e += T) {
    const int c = e / per;
    const int q = e - c * per;
    const int p = q / xl, x = q - p * xl;
    const double br = c == 0 ? P.brxd : (c == 1 ? P.bryd : P.brzd);
    float2 v = make_float2(0.f, 0.f);
    if (x < nx) {
      const float* yc = ys + (size_t)c * N + (size_t)z * plane;
      const int ya = y0 + 2 * p;
      if (ya < ny) {
        const float msv = msz ? msz[ya * nx + x] : P.ms;
        const float mv = yc[ya * nx + x];
        v.x = msv * mv;
        facc[0] += (double)msv * (double)mv * br;
      }
      if (ya + 1 < ny) {
        const float msv = msz ? msz[(ya + 1) * nx + x] : P.ms;
        const float mv = yc[(ya + 1) * nx + x];
        v.y = msv * mv;
        facc[0] += (double)msv * (double)mv * br;
      }
    }
    if (P.demag) lds[pidx((c * np + p) * Px + x)] = v;
  }
  if (P.demag) {
    __syncthreads();
    fft_lds<VPT, true, 0, true, false>(lds, P.logPx, 3 * np, twl, logTw,
                                        -1.f);
    // split the two real transforms, write the half spectrum: rows
    // (y0+2p, y0+2p+1) are adjacent -> one 16-byte store per (c, kx, p)
    const int H = P.Hx;
    const int totw = 3 * np * H;
    for (int e = threadIdx.x; e < totw; e += T) {
      const int cp = e % (3 * np), k = e / (3 * np);
      const int c = cp / np, p = cp - c * np;
      const int b = cp * Px;
      const float2 z1 = lds[pidx(b + k)];
      const float2 z2 = lds[pidx(b + ((Px - k) & (Px - 1)))];
      // A = (Z[k] + conj Z[-k]) / 2 ; B = (Z[k] - conj Z[-k]) / (2i)
      float4 v = make_float4(0.5f * (z1.x + z2.x), 0.5f * (z1.y - z2.y),
                             0.5f * (z1.y + z2.y), -0.5f * (z1.x - z2.x));
      const int ya = y0 + 2 * p;
      if (ya < ny) {
        if (ya + 1 >= ny) { v.z = 0.f; v.w = 0.f; }   // keep the pad zero
        float2* row = spec + ((size_t)(k * nz + z) * 3 + c) * nyp;
        *(float4*)(row + ya) = v;
      }
    }
  }
  block_sum<1>(facc, red);
  if (threadIdx.x == 0) partials[slot] = facc[0];
}

template <int T>
__global__ __launch_bounds__(T) void k_xfwd3(
    Prm P, const float* __restrict__ ys, float2* __restrict__ spec,
    Ctl* __restrict__ ctl, double* __restrict__ partials, int R,
    const float2* __restrict__ tw, int logTw) {
  extern __shared__ float2 lds_all[];
  if (ctl->done) return;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  xfwd3_body<T>(P, ys, spec, partials, R, tw, logTw, tile, tile, lds_all);
}

// =========================================================== k_clear_empty
// m = 0 in the cells outside the geometry (Ms = 0).
template <int T>
__global__ __launch_bounds__(T) void k_clear_empty(Prm P,
                                                   float* __restrict__ m) {
  const int N = P.ncell;
  for (int i = blockIdx.x * T + threadIdx.x; i < N; i += gridDim.x * T) {
    if (!(P.ms_map[i] > 0.f)) {
      m[i] = 0.f;
      m[N + i] = 0.f;
      m[2 * N + i] = 0.f;
    }
  }
}

// ========================================================== k_coupling_map
// Partial coupling sums sum Ms_i m_i . B_rms,i over the cells of one x-pass
// tile (rows y0 .. y0+R-1 of layer z) with the per-cell B_rms map, written
// to `slot` (they replace the forward pass's uniform-B_rms sums).
template <int T>
__device__ __forceinline__ void coupling_tile_body(
    const Prm& P, const float* __restrict__ ys, double* __restrict__ partials,
    int R, int tile, int slot) {
  __shared__ double red[16];
  const int nx = P.nx, ny = P.ny, nz = P.nz, N = P.ncell;
  const int z = tile % nz;
  const int y0 = (tile / nz) * R;
  const float* bm = P.brms_map;
  double f[1] = {0.0};
  for (int e = threadIdx.x; e < R * nx; e += T) {
    const int y = y0 + e / nx, x = e % nx;
    if (y >= ny) continue;
    const int i = (z * ny + y) * nx + x;
    const double msv = P.ms_map ? (double)P.ms_map[i] : (double)P.ms;
    f[0] += msv * ((double)ys[i] * bm[i] + (double)ys[N + i] * bm[N + i] +
                   (double)ys[2 * N + i] * bm[2 * N + i]);
  }
  block_sum<1>(f, red);
  if (threadIdx.x == 0) partials[slot] = f[0];
}

template <int T>
__global__ __launch_bounds__(T) void k_coupling_map(
    Prm P, const float* __restrict__ ys, Ctl* __restrict__ ctl,
    double* __restrict__ partials, int R) {
  if (ctl->done) return;
  coupling_tile_body<T>(P, ys, partials, R, blockIdx.x, blockIdx.x);
}

// ======================================================== k_coupling_modes
// Multimode cavity: the coupling sums F_k = sum_i Ms_i m_i . B_rms,k,i of
// every mode over the cells of one x-pass tile (as k_coupling_map), FP64,
// written to P.mpart[tile * kMaxModes + k].
template <int T>
__global__ __launch_bounds__(T) void k_coupling_modes(
    Prm P, const float* __restrict__ ys, Ctl* __restrict__ ctl, int R) {
  __shared__ double red[16 * kMaxModes];
  if (ctl->done) return;
  const Modes& M = *P.modes;
  const int nx = P.nx, ny = P.ny, nz = P.nz, N = P.ncell;
  const int tile = blockIdx.x;
  const int z = tile % nz;
  const int y0 = (tile / nz) * R;
  const int nm = M.n;
  double f[kMaxModes];
#pragma unroll
  for (int k = 0; k < kMaxModes; ++k) f[k] = 0.0;
  for (int e = threadIdx.x; e < R * nx; e += T) {
    const int y = y0 + e / nx, x = e % nx;
    if (y >= ny) continue;
    const int i = (z * ny + y) * nx + x;
    const double msv = P.ms_map ? (double)P.ms_map[i] : (double)P.ms;
    const double mx = msv * ys[i], my = msv * ys[N + i],
                 mz = msv * ys[2 * N + i];
#pragma unroll
    for (int k = 0; k < kMaxModes; ++k) {
      if (k >= nm) break;
      if (const float* b = M.map[k]) {
        f[k] += mx * b[i] + my * b[N + i] + mz * b[2 * N + i];
      } else {
        f[k] += mx * M.br[k][0] + my * M.br[k][1] + mz * M.br[k][2];
      }
    }
  }
  block_sum<kMaxModes>(f, red);
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < kMaxModes; ++k)
      P.mpart[(size_t)tile * kMaxModes + k] = f[k];
}

// ================================================================ k_xfwd_w
// Forward x pass with the FFT in registers (Px = 64 * NR): one wavefront per
// (component, row pair) of an R-row tile.  Lane l, register r loads x =
// l + 64 r of both rows (coalesced), the wavefront FFT leaves the spectrum in
// its bit-reversed order, a per-wavefront LDS region (Px complex) puts it
// back in natural order for the two-for-one split, and each lane writes the
// (A, B) row pair of its kx values as one 16-byte store.  Same contract and
// partial sums as k_xfwd.
template <int NR>
__device__ __forceinline__ void xfwd_w_body(
    const Prm& P, const float* __restrict__ ys, float2* __restrict__ spec,
    double* __restrict__ partials, int R, const float2* __restrict__ tw,
    int logTw, int tile, int slot, float2* zl) {
  __shared__ double red[16];
  constexpr int LNR = Log2<NR>::v;
  const int nz = P.nz;
  const int z = tile % nz;
  const int y0 = (tile / nz) * R;
  const int np = R >> 1;
  const int Px = P.Px, nx = P.nx, ny = P.ny, nyp = P.nyp, N = P.ncell;
  const int plane = nx * ny;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double fc = 0.0;
  const bool active = wv < 3 * np;
  const int c = active ? wv / np : 0, p = active ? wv - c * np : 0;
  const int ya = y0 + 2 * p;
  const bool fft = active && P.demag && ya < ny;
  float2* zw = zl + (size_t)wv * Px;
  if (active) {
    const double br = c == 0 ? P.brxd : (c == 1 ? P.bryd : P.brzd);
    const float* yc = ys + (size_t)c * N + (size_t)z * plane;
    const float* msz = P.ms_map ? P.ms_map + (size_t)z * plane : nullptr;
    float2 v[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int x = lane + 64 * r;
      float a = 0.f, b = 0.f;
      if (x < nx) {
        if (ya < ny) {
          const float ms = msz ? msz[ya * nx + x] : P.ms;
          const float mv = yc[ya * nx + x];
          a = ms * mv;
          fc += (double)ms * (double)mv;
        }
        if (ya + 1 < ny) {
          const float ms = msz ? msz[(ya + 1) * nx + x] : P.ms;
          const float mv = yc[(ya + 1) * nx + x];
          b = ms * mv;
          fc += (double)ms * (double)mv;
        }
      }
      v[r] = make_float2(a, b);
    }
    fc *= br;
    if (fft) {
      wfft_fwd<NR>(v, lane, tw, logTw);
      const int b2 = NR * brev_bits(lane, 6);
#pragma unroll
      for (int r = 0; r < NR; ++r) zw[brev_bits(r, LNR) + b2] = v[r];
    }
  }
  __syncthreads();   // natural-order spectrum of each wavefront in LDS
  if (fft) {
    const int H = P.Hx;
    for (int k = lane; k < H; k += 64) {
      const float2 z1 = zw[k];
      const float2 z2 = zw[(Px - k) & (Px - 1)];
      // A = (Z[k] + conj Z[-k]) / 2 ; B = (Z[k] - conj Z[-k]) / (2i)
      float4 AB = make_float4(0.5f * (z1.x + z2.x), 0.5f * (z1.y - z2.y),
                              0.5f * (z1.y + z2.y), -0.5f * (z1.x - z2.x));
      if (ya + 1 >= ny) { AB.z = 0.f; AB.w = 0.f; }   // keep the pad zero
      *(float4*)(spec + ((size_t)(k * nz + z) * 3 + c) * nyp + ya) = AB;
    }
  }
  double facc[1] = {fc};
  block_sum<1>(facc, red);
  if (threadIdx.x == 0) partials[slot] = facc[0];
}

template <int NR>
__global__ __launch_bounds__(NR >= 32 ? 512 : 1024) void k_xfwd_w(
    Prm P, const float* __restrict__ ys, float2* __restrict__ spec,
    Ctl* __restrict__ ctl, double* __restrict__ partials, int stage, int R,
    const float2* __restrict__ tw, int logTw, int mode) {
  extern __shared__ float2 zl[];
  if (ctl->done) return;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  xfwd_w_body<NR>(P, ys, spec, partials, R, tw, logTw, tile, tile, zl);
}

// Finishes the FP64 coupling sum of a stage from the k_xfwd partials (the
// kernel boundary makes them visible) and advances the cavity: mode 0
// integrate, mode 1 evaluate (rate at a_1, t).  Runs in one workgroup.
__device__ __forceinline__ void finish_cavity(const Prm& P, Ctl* ctl,
                                              const double* partials,
                              int nblk, int stage, int mode, double* red) {
  (void)red;
  // first wavefront only, lane l owns partials l, l+64, ...: the summation
  // order does not depend on the workgroup size
  if (threadIdx.x >= 64) return;
  double F[1] = {0.0};
  // eight loads in flight per lane, added in the same order as one by one
  for (int b0 = threadIdx.x; b0 < nblk; b0 += 64 * 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int b = b0 + 64 * u;
      v[u] = b < nblk ? partials[b] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (b0 + 64 * u < nblk) F[0] += v[u];
  }
  for (int o = 32; o > 0; o >>= 1) F[0] += __shfl_xor(F[0], o, 64);
  if (threadIdx.x != 0) return;
  if (mode == 0) {
    if (ctl->ahist && P.method == 0) {
      double* h = ctl->ahist + 2 * (5 * ctl->accepted + (stage - 1));
      h[0] = ctl->as_re[stage];
      h[1] = ctl->as_im[stage];
    }
    cavity_stage(P, ctl, stage, F[0]);
  } else {
    const double ts = ctl->t;
    const double eps = P.camp * drive_shape(P.ckind, P.cw, ts);
    const double ar = ctl->as_re[1], ai = ctl->as_im[1];
    ctl->rhs_dadt_re = -P.kappa * ar + P.wc * ai;
    ctl->rhs_dadt_im = -P.wc * ar - P.kappa * ai + P.vc_hbar * F[0] - eps;
    ctl->F_last = F[0];
  }
}

// Multimode cavity: the coupling sum of every mode from the tiles' partials
// (first wavefront, fixed order), then the modes' stage rates and next
// stage amplitudes.  Runs in its own one-workgroup kernel so that the
// spectral pass's workgroup 0 keeps only the single-mode finish.
__device__ __forceinline__ void finish_cavity_modes(const Prm& P, Ctl* ctl,
                                                    int nblk, int stage,
                                                    int mode) {
  if (threadIdx.x >= 64) return;
  const int nm = P.modes->n;
  double Fm[kMaxModes];
#pragma unroll
  for (int k = 0; k < kMaxModes; ++k) {
    double v = 0.0;
    if (k < nm) {   // uniform across the wave
      for (int b = threadIdx.x; b < nblk; b += 64)
        v += P.mpart[(size_t)b * kMaxModes + k];
      for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    }
    Fm[k] = v;
  }
  if (threadIdx.x != 0) return;
  if (mode == 0) {
    cavity_stage_modes(P, ctl, stage, Fm);
  } else {
    // evaluation: the rates of every mode at the given amplitudes
    const Modes& M = *P.modes;
#pragma unroll
    for (int k = 0; k < kMaxModes; ++k) {
      if (k >= nm) break;
      const double eps =
          M.camp[k] * drive_shape(M.ckind[k], M.cw[k], ctl->t);
      const double ar = ctl->mas_re[1][k], ai = ctl->mas_im[1][k];
      ctl->mka_re[1][k] = -M.kappa[k] * ar + M.wc[k] * ai;
      ctl->mka_im[1][k] =
          -M.wc[k] * ar - M.kappa[k] * ai + P.vc_hbar * Fm[k] - eps;
    }
    ctl->rhs_dadt_re = ctl->mka_re[1][0];
    ctl->rhs_dadt_im = ctl->mka_im[1][0];
    ctl->F_last = Fm[0];
  }
}

template <int T>
__global__ __launch_bounds__(T) void k_finish_modes(Prm P,
                                                    Ctl* __restrict__ ctl,
                                                    int nblk, int stage,
                                                    int mode) {
  if (ctl->done) return;
  finish_cavity_modes(P, ctl, nblk, stage, mode);
}

// Stand-alone stage finish (used when there is no spectral pass).
template <int T>
__global__ __launch_bounds__(T) void k_finish_stage(
    Prm P, Ctl* __restrict__ ctl, const double* __restrict__ partials,
    int nblk, int stage, int mode) {
  __shared__ double red[16];
  if (ctl->done) return;
  finish_cavity(P, ctl, partials, nblk, stage, mode, red);
}

// ================================================================= k_yspec
// grid ceil(Hx/W); LDS: W * nz * 3 * Py complex.  Kernel layout
// K[kx][ky][kslot(comp, dz)] (comp: xx yy zz xy xz yz; xz, yz coefficients
// of -i, absent at dz = 0), ky in [0, Py/2]; scaled by -mu0/(Px Py).  Spectrum rows have nyp (even)
// entries; entries at y >= ny are zero and stay zero.
// 3x3 demag-kernel product at one (kx, ky) for all nz layers.  kk holds
// K[kx][|ky|] as kk[comp NZ + dz] (kernel_load); sy = -1 on the mirrored half
// (xy and yz are odd in ky); xz, yz are odd in the z offset.
template <int NZ>
__device__ __forceinline__ void kernel_product_k(const float (&kk)[6 * NZ],
                                                 float sy,
                                                 const float2 (&M)[3 * NZ],
                                                 float2 (&Hf)[3 * NZ]) {
#pragma unroll
  for (int q = 0; q < 3 * NZ; ++q) Hf[q] = make_float2(0.f, 0.f);
#pragma unroll
  for (int zt = 0; zt < NZ; ++zt) {
#pragma unroll
    for (int zs = 0; zs < NZ; ++zs) {
      const int d = zt - zs;
      const int ad = d < 0 ? -d : d;
      const float sz = d < 0 ? -1.f : 1.f;
      const float kxx = kk[0 * NZ + ad], kyy = kk[1 * NZ + ad];
      const float kzz = kk[2 * NZ + ad], kxy = sy * kk[3 * NZ + ad];
      const float qxz = sz * kk[4 * NZ + ad];          // K_xz = -i qxz
      const float qyz = sz * sy * kk[5 * NZ + ad];     // K_yz = -i qyz
      const float2 mx = M[zs * 3 + 0], my = M[zs * 3 + 1], mz = M[zs * 3 + 2];
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
}

// The entry at Kp (kentry(NZ) floats) into kk[comp NZ + dz], the vanishing
// xz and yz coefficients at dz = 0 as zeros.
template <int NZ>
__device__ __forceinline__ void kernel_load(const float* __restrict__ Kp,
                                            float (&kk)[6 * NZ]) {
#pragma unroll
  for (int q = 0; q < 4 * NZ; ++q) kk[q] = Kp[q];
  kk[4 * NZ] = kk[5 * NZ] = 0.f;
#pragma unroll
  for (int dz = 1; dz < NZ; ++dz) {
    kk[4 * NZ + dz] = Kp[kslot(4, dz, NZ)];
    kk[5 * NZ + dz] = Kp[kslot(5, dz, NZ)];
  }
}

template <int NZ>
__device__ __forceinline__ void kernel_product(const float* __restrict__ Kp,
                                               float sy,
                                               const float2 (&M)[3 * NZ],
                                               float2 (&Hf)[3 * NZ]) {
  float kk[6 * NZ];
  kernel_load<NZ>(Kp, kk);
  kernel_product_k<NZ>(kk, sy, M, Hf);
}

// Spectral pass of column blocks blk0, blk0 + bstride, ... < nblk (a
// workgroup of T threads; LDS `lds_all` as sized by the plan; block blk0
// only unless yspec_steps(T, NZ)).  With more than one block per workgroup, the input of the
// next block is loaded into registers before the inverse transform of the
// current one, so that its latency overlaps that transform and the stores
// (the host steps through blocks only where a block's lower half fits kPf
// float4 per thread).  LP > 0: log2(Py) fixed at compile time (specialised
// FFT addressing).
constexpr int kPf = 4;
// Workgroup sizes and layer counts whose spectral pass steps through blocks
// (elsewhere the prefetch registers would cost occupancy or spill).
__host__ __device__ constexpr bool yspec_steps(int T, int NZ) {
  return NZ <= 2 && T == 1024;
}
template <int T, int NZ, int LP = 0>
__device__ __forceinline__ void yspec_l_body(
    const Prm& P, float2* __restrict__ spec, const float* __restrict__ K,
    Ctl* __restrict__ ctl, int W, const float2* __restrict__ tw,
    int logTw, const double* __restrict__ partials, int nblk_f, int stage,
    int mode, int blk0, int nblk, int bstride, float2* lds_all) {
  __shared__ double red[16];
  // compile-time lengths read per-pass twiddle tables (fewer VALU
  // operations); otherwise the first half of the plain table is staged
  constexpr bool TT = LP > 0;
  float2* twl = lds_all;
  float2* lds = lds_all + yspec_tw_len(LP, logTw);
  if constexpr (TT) fft_tt_build<VPTY, true, LP>(twl, tw, logTw);
  else stage_twiddles(twl, tw, logTw);
  // workgroup 0 also finishes the coupling sum of this stage
  if (blk0 == 0 && !P.modes) {
    finish_cavity(P, ctl, partials, nblk_f, stage, mode, red);
    __syncthreads();
  }
  constexpr int nz3 = 3 * NZ;
  const int lpy = LP > 0 ? LP : P.logPy;
  const int ny = P.ny, nyp = P.nyp, Py = 1 << lpy;
  // Column slots: slot s >= 1 is kx = s; slot 0 carries the two real
  // columns kx = 0 (real part) and kx = Px/2 (imaginary part) as one complex
  // sequence (Px >= 2), so the Px/2 + 1 columns fill exactly Px/2 slots.
  const bool pair = P.Px >= 2;
  const int hxn = P.Px >> 1;
  const int nslot = pair ? hxn : P.Hx;
  const float2* srcn = spec + (size_t)hxn * nz3 * nyp;
  // lower halves, as pairs of rows (y, y+1) per 16-byte load: rows >= Py/2
  // are zero padding and the first pass does not read them
  const int hp = Py >> 2;
  // Blocks are stepped through with prefetch where yspec_steps allows, one
  // block per workgroup otherwise.  `blk`: the block; `tid`: the thread
  // index; `nb`: the next block of this workgroup (>= nblk: none); `pf`: its
  // input registers.
  constexpr bool PF = yspec_steps(T, NZ);
  float4 pf[kPf];
  auto block = [&](const int blk, const int tid, const int nb) {
    const int kx0 = blk * W;
    const int Wb = min(W, nslot - kx0);
    const bool has_pair = pair && blk == 0;   // slot 0 in this block
    const int ncol = Wb * nz3;
    const float2* src = spec + (size_t)kx0 * nz3 * nyp;
    if (PF && Py >= 4 && blk != blk0) {
      // this block's input, loaded during the previous block
      const int tot = ncol * hp;
#pragma unroll
      for (int u = 0; u < kPf; ++u) {
        const int e = tid + u * T;
        const int col = e >> (lpy - 2), y = (e & (hp - 1)) << 1;
        if (e < tot) *(float4*)(lds + pidx(col * Py + y)) = pf[u];
      }
    } else if (Py >= 4) {
      const int tot = ncol * hp;
      constexpr int U = 8;
      for (int e0 = tid; e0 < tot; e0 += T * U) {
        float4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int e = e0 + u * T;
          const int col = e >> (lpy - 2), y = (e & (hp - 1)) << 1;
          v[u] = make_float4(0.f, 0.f, 0.f, 0.f);
          if (e < tot && y < ny) {
            v[u] = ld4(spec, (unsigned)((kx0 * nz3 + col) * nyp + y) << 3);
            if (has_pair && col < nz3) {
              const float4 n =
                  ld4(spec, (unsigned)((hxn * nz3 + col) * nyp + y) << 3);
              v[u] = make_float4(v[u].x, n.x, v[u].z, n.z);
            }
          }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int e = e0 + u * T;
          const int col = e >> (lpy - 2), y = (e & (hp - 1)) << 1;
          if (e < tot) *(float4*)(lds + pidx(col * Py + y)) = v[u];
        }
      }
    } else {
      // Py = 1 or 2: row 0 is the only data row
      for (int e = tid; e < ncol; e += T) {
        float2 v = src[(size_t)e * nyp];
        if (has_pair && e < nz3) v.y = srcn[(size_t)e * nyp].x;
        lds[pidx(e * Py)] = v;
      }
    }
    __syncthreads();
    fft_lds<VPTY, true, LP, true, false, 4, TT>(lds, P.logPy, ncol, twl,
                                               logTw, -1.f, tid);
    // pointwise product, all 3*nz values at a (w, ky).  A thread takes the
    // mirrored pair ky = kh, Py - kh (kh in 1 .. Py/2 - 1), which share the
    // kernel row |ky| = kh (odd-in-ky parts flip), or for kh = 0 the two
    // self-mirrored rows ky = 0 and Py/2.
    const int Hy = P.Hy;
    // (Py = 1: the single row ky = 0 only)
    const int Ph = Py >> 1, nkh = Py >= 2 ? Ph : 1;
    const int lph = Py >= 2 ? lpy - 1 : 0, nself = Py >= 2 ? 2 : 1;
    for (int e = tid; e < Wb * nkh; e += T) {
      const int w = e >> lph, kh = e & (nkh - 1);
      float2 M[nz3], Hf[nz3];
      if (has_pair && w == 0) {
        // slot 0: split Z = X0 + i XN at (ky, -ky), apply each column's
        // kernel, recombine; the results are real sequences, so
        // W[-ky] = conj(Y0[ky]) + i conj(YN[ky]).  One pass per mirrored
        // pair: ky = kh, and for kh = 0 also ky = Py/2.
        // (Y0 is parked in LDS while YN is formed: fewer live registers)
#pragma unroll 1
        for (int r = 0; r < (kh == 0 ? nself : 1); ++r) {
          const int ky = r == 0 ? kh : Ph;
          const int km = (Py - ky) & (Py - 1);
          float2 XN[nz3];
#pragma unroll
          for (int q = 0; q < nz3; ++q) {
            const float2 z = lds[pidx(q * Py + ky)];
            const float2 zm = lds[pidx(q * Py + km)];
            M[q] = make_float2(0.5f * (z.x + zm.x), 0.5f * (z.y - zm.y));
            XN[q] = make_float2(0.5f * (z.y + zm.y), -0.5f * (z.x - zm.x));
          }
          kernel_product<NZ>(K + (size_t)ky * kentry(NZ), 1.f, M, Hf);
#pragma unroll
          for (int q = 0; q < nz3; ++q) lds[pidx(q * Py + ky)] = Hf[q];
          kernel_product<NZ>(K + ((size_t)hxn * Hy + ky) * kentry(NZ), 1.f, XN,
                             Hf);
#pragma unroll
          for (int q = 0; q < nz3; ++q) {
            const float2 y0 = lds[pidx(q * Py + ky)];
            lds[pidx(q * Py + ky)] = make_float2(y0.x - Hf[q].y,
                                                 y0.y + Hf[q].x);
            if (km != ky)
              lds[pidx(q * Py + km)] = make_float2(y0.x + Hf[q].y,
                                                   -y0.y + Hf[q].x);
          }
        }
        continue;
      }
      const int kx = kx0 + w;
      const int base = w * nz3 * Py;
      float kk[6 * NZ];
      if (kh == 0) {
        // ky = 0 and ky = Py/2: each its own mirror, even parts only
#pragma unroll 1
        for (int r = 0; r < nself; ++r) {
          const int ky = r * Ph;
          kernel_load<NZ>(K + ((size_t)kx * Hy + ky) * kentry(NZ), kk);
#pragma unroll
          for (int q = 0; q < nz3; ++q) M[q] = lds[pidx(base + q * Py + ky)];
          kernel_product_k<NZ>(kk, 1.f, M, Hf);
#pragma unroll
          for (int q = 0; q < nz3; ++q) lds[pidx(base + q * Py + ky)] = Hf[q];
        }
        continue;
      }
      kernel_load<NZ>(K + ((size_t)kx * Hy + kh) * kentry(NZ), kk);
#pragma unroll
      for (int q = 0; q < nz3; ++q) M[q] = lds[pidx(base + q * Py + kh)];
      kernel_product_k<NZ>(kk, 1.f, M, Hf);
#pragma unroll
      for (int q = 0; q < nz3; ++q) lds[pidx(base + q * Py + kh)] = Hf[q];
      const int km = Py - kh;
#pragma unroll
      for (int q = 0; q < nz3; ++q) M[q] = lds[pidx(base + q * Py + km)];
      kernel_product_k<NZ>(kk, -1.f, M, Hf);   // odd-in-ky parts flip
#pragma unroll
      for (int q = 0; q < nz3; ++q) lds[pidx(base + q * Py + km)] = Hf[q];
    }
    __syncthreads();
    // next block's input (it never holds slot 0: blk + bstride > 0)
    if (PF && Py >= 4 && nb < nblk) {
      const int totn = min(W, nslot - nb * W) * nz3 * hp;
      const int c0 = nb * W * nz3;
#pragma unroll
      for (int u = 0; u < kPf; ++u) {
        const int e = tid + u * T;
        const int col = e >> (lpy - 2), y = (e & (hp - 1)) << 1;
        pf[u] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (e < totn && y < ny)
          pf[u] = ld4(spec, (unsigned)((c0 + col) * nyp + y) << 3);
      }
    }
    fft_lds<VPTY, true, LP, false, true, 4, TT>(lds, P.logPy, ncol, twl,
                                               logTw, 1.f, tid);
    float2* dst = spec + (size_t)kx0 * nz3 * nyp;
    float2* dstn = spec + (size_t)hxn * nz3 * nyp;
    if (Py >= 4) {
      // row pairs of the lower half; those at y >= nyp are not stored
      const int hq = Py >> 2;
      const int tot = ncol * hq;
      for (int e = tid; e < tot; e += T) {
        const int col = e >> (lpy - 2), y = (e & (hq - 1)) << 1;
        if (y >= nyp) continue;
        float4 v = *(const float4*)(lds + pidx(col * Py + y));
        if (y + 1 >= ny) { v.z = 0.f; v.w = 0.f; }   // keep the pad zero
        if (has_pair && col < nz3) {
          st4(spec, (unsigned)((hxn * nz3 + col) * nyp + y) << 3,
              make_float4(v.y, 0.f, v.w, 0.f));
          v = make_float4(v.x, 0.f, v.z, 0.f);
        }
        st4(spec, (unsigned)((kx0 * nz3 + col) * nyp + y) << 3, v);
      }
    } else {
      // Py = 1 or 2: row 0 is the only data row (the pad row stays zero)
      for (int e = tid; e < ncol; e += T) {
        const float2 v = lds[pidx(e * Py)];
        if (has_pair && e < nz3) {
          dstn[(size_t)e * nyp] = make_float2(v.y, 0.f);
          dst[(size_t)e * nyp] = make_float2(v.x, 0.f);
        } else {
          dst[(size_t)e * nyp] = v;
        }
      }
    }
  };
  if constexpr (PF) {
    for (int blk = blk0; blk < nblk; blk += bstride) {
      // thread index through an opaque copy: the address arithmetic of a
      // block is formed where it is used, not held in registers across
      // blocks
      int tid = threadIdx.x;
      asm volatile("" : "+v"(tid));
      block(blk, tid, blk + bstride);
      if (blk + bstride < nblk) __syncthreads();   // the LDS is refilled next
    }
  } else {
    block(blk0, (int)threadIdx.x, nblk);
  }
}

// Grid: nblk workgroups (one block each), or fewer that step through the
// blocks with stride gridDim.x.
template <int T, int NZ, int LP = 0>
__global__ __launch_bounds__(T) void k_yspec(
    Prm P, float2* __restrict__ spec, const float* __restrict__ K,
    Ctl* __restrict__ ctl, int W, const float2* __restrict__ tw,
    int logTw, const double* __restrict__ partials, int nblk_f, int stage,
    int mode, int nblk) {
  extern __shared__ float2 lds_all[];
  if (ctl->done) return;
  yspec_l_body<T, NZ, LP>(P, spec, K, ctl, W, tw, logTw, partials, nblk_f,
                          stage, mode, blockIdx.x, nblk, gridDim.x, lds_all);
}


// ============================================================== k_yspec_z
// Spectral pass for two layers (nz = 2) and one kx slot per block, with
// half the LDS of k_yspec: the three columns of layer 1 are transformed
// first and their spectrum moves into registers (each thread keeps the rows
// ky = kh, Py - kh of the mirrored pairs it multiplies later), then layer 0
// is transformed in the same LDS; the 3x3 product with the z-offset sum
// reads layer 0 from LDS and layer 1 from registers, writes H(layer 0) back
// to LDS and keeps H(layer 1) in registers; layer 0 is inverse transformed
// and stored, then layer 1 from the registers.  Two 512-thread workgroups
// share a CU, so one can run its VALU-bound butterflies while the other
// waits on LDS or memory.  Arithmetic per element as k_yspec's.  Grid: one
// workgroup per kx slot (nblk of them).
constexpr int kYzT = 512;
// LDS padding of the two-layer pass: 2 slots every 2^kYzPs values
constexpr int kYzPs = 5;
template <int LP>
__global__ __launch_bounds__(kYzT) __attribute__((amdgpu_waves_per_eu(4))) void k_yspec_z(
    Prm P, float2* __restrict__ spec, const float* __restrict__ K,
    Ctl* __restrict__ ctl, const float2* __restrict__ tw, int logTw,
    const double* __restrict__ partials, int nblk_f, int stage, int mode,
    int nblk) {
  constexpr int T = kYzT, NZ = 2, nz3 = 6, Py = 1 << LP, Ph = Py >> 1;
  constexpr int hp = Py >> 2;          // row pairs of a column's lower half
  constexpr int NKH = Ph / T;          // mirrored pairs per thread (>= 1)
  static_assert(NKH >= 1, "Py >= 2 T");
  extern __shared__ float2 lds_all[];
  __shared__ double red[16];
  if (ctl->done) return;
  float2* twl = lds_all;
  float2* lds = lds_all + yspec_tw_len(LP, logTw);
  fft_tt_build<VPTY, true, LP>(twl, tw, logTw);
  const int blk0 = blockIdx.x;
  if (blk0 == 0 && !P.modes) {
    finish_cavity(P, ctl, partials, nblk_f, stage, mode, red);
    __syncthreads();
  }
  const int ny = P.ny, nyp = P.nyp, Hy = P.Hy;
  const int hxn = P.Px >> 1;   // slot 0 pairs kx = 0 and Px/2 (Px >= 2)
  // layer-1 rows ky, km of the thread's mirrored pairs (kh = tid + i T):
  // spectrum after the forward transform, then the product's output
  float2 r1[NKH][2][3];
  {
    const int blk = blk0;
    (void)nblk;
    const int tid = threadIdx.x;
    const bool has_pair = blk == 0;
    const int kx = blk;   // one slot per block; slot 0 = (0, Px/2)
    // lower halves of layer z's three columns into LDS (column c at c Py)
    auto load_layer = [&](int z) {
      for (int e = tid; e < 3 * hp; e += T) {
        const int c = e / hp, y = (e - c * hp) << 1;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (y < ny) {
          const int q = z * 3 + c;
          v = ld4(spec, (unsigned)((kx * nz3 + q) * nyp + y) << 3);
          if (has_pair) {
            const float4 n = ld4(spec, (unsigned)((hxn * nz3 + q) * nyp + y)
                                           << 3);
            v = make_float4(v.x, n.x, v.z, n.z);
          }
        }
        *(float4*)(lds + pidx_s<kYzPs>(c * Py + y)) = v;
      }
    };
    // rows (ky, km) of mirrored pair kh; kh = 0: the self-mirrored rows 0
    // and Py/2
    auto rows = [&](int kh, int& ky, int& km) {
      ky = kh;
      km = kh == 0 ? Ph : Py - kh;
    };
    auto store_layer = [&](int z) {
      for (int e = tid; e < 3 * hp; e += T) {
        const int c = e / hp, y = (e - c * hp) << 1;
        if (y >= nyp) continue;
        float4 v = *(const float4*)(lds + pidx_s<kYzPs>(c * Py + y));
        if (y + 1 >= ny) { v.z = 0.f; v.w = 0.f; }   // keep the pad zero
        const int q = z * 3 + c;
        if (has_pair) {
          st4(spec, (unsigned)((hxn * nz3 + q) * nyp + y) << 3,
              make_float4(v.y, 0.f, v.w, 0.f));
          v = make_float4(v.x, 0.f, v.z, 0.f);
        }
        st4(spec, (unsigned)((kx * nz3 + q) * nyp + y) << 3, v);
      }
    };
    // ---- layer 1: forward transform, spectrum into registers
    load_layer(1);
    __syncthreads();
    fft_lds<VPTY, true, LP, true, false, kYzPs, true>(lds, LP, 3, twl, logTw,
                                                 -1.f, tid);
#pragma unroll
    for (int i = 0; i < NKH; ++i) {
      int ky, km;
      rows(tid + i * T, ky, km);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        r1[i][0][c] = lds[pidx_s<kYzPs>(c * Py + ky)];
        r1[i][1][c] = lds[pidx_s<kYzPs>(c * Py + km)];
      }
    }
    __syncthreads();
    // ---- layer 0: forward transform in the same LDS
    load_layer(0);
    __syncthreads();
    fft_lds<VPTY, true, LP, true, false, kYzPs, true>(lds, LP, 3, twl, logTw,
                                                 -1.f, tid);
    // ---- product at (ky, km) of each of the thread's pairs; layer-0
    // results go straight back to LDS, layer-1 results to registers
#pragma unroll
    for (int i = 0; i < NKH; ++i) {
      const int kh = tid + i * T;
      int ky, km;
      rows(kh, ky, km);
      float2 Ma[nz3], Mb[nz3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        Ma[c] = lds[pidx_s<kYzPs>(c * Py + ky)];
        Mb[c] = lds[pidx_s<kYzPs>(c * Py + km)];
        Ma[3 + c] = r1[i][0][c];
        Mb[3 + c] = r1[i][1][c];
      }
      // result H at row y (j = 0: ky, j = 1: km)
      auto put = [&](const float2 (&H)[nz3], int y, int j) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          lds[pidx_s<kYzPs>(c * Py + y)] = H[c];
          r1[i][j][c] = H[3 + c];
        }
      };
      if (has_pair) {
        // slot 0: Z = X0 + i XN; X0[ky] = (Z[ky] + conj Z[-ky]) / 2,
        // XN[ky] = (Z[ky] - conj Z[-ky]) / (2i); each column's own kernel
        // at |ky|, then W[ky] = Y0[ky] + i YN[ky], W[-ky] = conj Y0[ky] +
        // i conj YN[ky] (real results)
        for (int r = 0; r < (kh == 0 ? 2 : 1); ++r) {
          const int y1 = r == 0 ? ky : km;
          float2 X0[nz3], XN[nz3], Y0[nz3], YN[nz3];
#pragma unroll
          for (int q = 0; q < nz3; ++q) {
            const float2 z = r == 0 ? Ma[q] : Mb[q];   // at y1
            const float2 zm = kh == 0 ? z : Mb[q];     // at -y1
            X0[q] = make_float2(0.5f * (z.x + zm.x), 0.5f * (z.y - zm.y));
            XN[q] = make_float2(0.5f * (z.y + zm.y), -0.5f * (z.x - zm.x));
          }
          kernel_product<NZ>(K + (size_t)y1 * kentry(NZ), 1.f, X0, Y0);
          kernel_product<NZ>(K + ((size_t)hxn * Hy + y1) * kentry(NZ), 1.f,
                             XN, YN);
          float2 W[nz3];
#pragma unroll
          for (int q = 0; q < nz3; ++q)
            W[q] = make_float2(Y0[q].x - YN[q].y, Y0[q].y + YN[q].x);
          put(W, y1, r);
          if (kh != 0) {
#pragma unroll
            for (int q = 0; q < nz3; ++q)
              W[q] = make_float2(Y0[q].x + YN[q].y, -Y0[q].y + YN[q].x);
            put(W, km, 1);
          }
        }
      } else {
        float kk[6 * NZ];
        float2 H[nz3];
        // kh = 0: rows 0 and Py/2, each its own mirror (even parts only)
        kernel_load<NZ>(K + ((size_t)kx * Hy + ky) * kentry(NZ), kk);
        kernel_product_k<NZ>(kk, 1.f, Ma, H);
        put(H, ky, 0);
        if (kh == 0)
          kernel_load<NZ>(K + ((size_t)kx * Hy + km) * kentry(NZ), kk);
        kernel_product_k<NZ>(kk, kh == 0 ? 1.f : -1.f, Mb, H);
        put(H, km, 1);   // odd-in-ky parts flip on the mirrored row
      }
    }
    __syncthreads();
    // ---- layer 0: inverse transform and store
    fft_lds<VPTY, true, LP, false, true, kYzPs, true>(lds, LP, 3, twl, logTw,
                                                 1.f, tid);
    store_layer(0);
    __syncthreads();
    // ---- layer 1: its product rows back into LDS, inverse, store
#pragma unroll
    for (int i = 0; i < NKH; ++i) {
      int ky, km;
      rows(tid + i * T, ky, km);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        lds[pidx_s<kYzPs>(c * Py + ky)] = r1[i][0][c];
        lds[pidx_s<kYzPs>(c * Py + km)] = r1[i][1][c];
      }
    }
    __syncthreads();
    fft_lds<VPTY, true, LP, false, true, kYzPs, true>(lds, LP, 3, twl, logTw,
                                                 1.f, tid);
    store_layer(1);
  }
}

// ============================================================== k_yspec_h
// Spectral pass split by ky parity.  A y column is zero beyond Py/2, so its
// Py-point DFT splits exactly into the even-ky half (the Py/2-point DFT of
// x[n]) and the odd-ky half (the Py/2-point DFT of x[n] w^n, w = exp(-2 pi
// i / Py)); on the rows kept, y < Py/2, the inverse is
//     y[n] = IDFT(Y_even)[n] + w^-n IDFT(Y_odd)[n]   (both unnormalised).
// The halves run one after the other through an LDS buffer half the size of
// k_yspec's, so two workgroups share a CU; the even result is parked in the
// output rows and completed by the same thread in the odd half.  Thread t
// owns elements e = t + i T (i < EPT) of the W * 3nz columns; the host
// guarantees W * 3nz * Py/2 <= EPT * T.  Same contract as k_yspec.
template <int T, int NZ, int EPT>
__global__ __launch_bounds__(T, 4) void k_yspec_h(
    Prm P, float2* __restrict__ spec, const float* __restrict__ K,
    Ctl* __restrict__ ctl, int W, const float2* __restrict__ tw,
    int logTw, const double* __restrict__ partials, int nblk_f, int stage,
    int mode) {
  extern __shared__ float2 lds_all[];
  __shared__ double red[16];
  if (ctl->done) return;
  float2* twl = lds_all;
  float2* lds = lds_all + lds_twiddles(logTw);
  stage_twiddles(twl, tw, logTw);
  if (blockIdx.x == 0 && !P.modes) {
    finish_cavity(P, ctl, partials, nblk_f, stage, mode, red);
    __syncthreads();
  }
  constexpr int nz3 = 3 * NZ;
  const int kx0 = blockIdx.x * W;
  const int Wb = min(W, P.Hx - kx0);
  const int ny = P.ny, nyp = P.nyp;
  const int logPh = P.logPy - 1, Ph = 1 << logPh;
  const int tot = (Wb * nz3) << logPh;
  const int sh = logTw - P.logPy;       // table stride of exp(-2 pi i n / Py)
  float2* col0 = spec + (size_t)kx0 * nz3 * nyp;
  float2 xin[EPT];
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = threadIdx.x + i * T;
    const int c = e >> logPh, n = e & (Ph - 1);
    xin[i] = (e < tot && n < ny) ? col0[(size_t)c * nyp + n]
                                 : make_float2(0.f, 0.f);
  }
#pragma unroll 1
  for (int h = 0; h < 2; ++h) {
    // opaque copy of the transform length: keeps the FFT index arithmetic
    // inside each half instead of live across both (register pressure)
    int lph = logPh;
    asm volatile("" : "+s"(lph));
    const int phl = 1 << lph;
    const int totl = (Wb * nz3) << lph;
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int e = threadIdx.x + i * T;
      if (e < totl) {
        float2 v = xin[i];
        if (h) v = cmul(v, twl[(e & (phl - 1)) << sh]);
        lds[pidx(e)] = v;
      }
    }
    __syncthreads();
    fft_lds<VPTY, true>(lds, lph, Wb * nz3, twl, logTw, -1.f);
    for (int e = threadIdx.x; e < (Wb << lph); e += T) {
      const int w = e >> lph, k = e & (phl - 1);
      const int ky = 2 * k + h;
      const bool lo = ky <= phl;
      const int kyi = lo ? ky : 2 * phl - ky;
      float2 M[nz3], Hf[nz3];
#pragma unroll
      for (int q = 0; q < nz3; ++q)
        M[q] = lds[pidx(((w * nz3 + q) << lph) + k)];
      kernel_product<NZ>(K + ((size_t)(kx0 + w) * P.Hy + kyi) * kentry(NZ),
                         lo ? 1.f : -1.f, M, Hf);
#pragma unroll
      for (int q = 0; q < nz3; ++q)
        lds[pidx(((w * nz3 + q) << lph) + k)] = Hf[q];
    }
    __syncthreads();
    fft_lds<VPTY, true>(lds, lph, Wb * nz3, twl, logTw, 1.f);
    // (same elements as the thread loaded; not unrolled, to bound the
    // number of loads in flight)
#pragma unroll 1
    for (int e = threadIdx.x; e < totl; e += T) {
      const int c = e >> lph, n = e & (phl - 1);
      if (n < nyp) {
        float2* o = col0 + (size_t)c * nyp + n;
        const float2 v = lds[pidx(e)];
        if (h == 0) {
          if (n < ny) *o = v;
        } else {
          *o = (n < ny) ? cadd(*o, wmulc(v, twl[n << sh]))
                        : make_float2(0.f, 0.f);   // pad stays zero
        }
      }
    }
    __syncthreads();   // the LDS buffer is refilled by the next half
  }
}


// ============================================================== k_yspec_w
// Kernel product of one chunk of G registers (all columns of the workgroup
// at the same ky), staged through LDS.  The chunk start G0 is a template
// parameter so that the register array is only ever indexed statically.
template <int NZ, int NR, int G, int G0>
__device__ __forceinline__ void yprod_chunks(
    float2 (&v)[NR], float2* lds, int Py, int Hy, const float* __restrict__ K,
    int kx0, int Wb, int wv, int lane, bool active) {
  constexpr int nz3 = 3 * NZ;
  constexpr int LNR = Log2<NR>::v;
  __syncthreads();
  if (active) {
#pragma unroll
    for (int rr = 0; rr < G; ++rr) lds[(wv * G + rr) * 64 + lane] = v[G0 + rr];
  }
  __syncthreads();
  const int nslot = Wb * G * 64;
  for (int s = threadIdx.x; s < nslot; s += blockDim.x) {
    const int w = s / (G * 64);
    const int rem = s - w * (G * 64);
    const int rr = rem >> 6, ln = rem & 63;
    const int ky = brev_bits(G0 + rr, LNR) + NR * brev_bits(ln, 6);
    const int kx = kx0 + w;
    const bool lo = ky <= (Py >> 1);
    const int kyi = lo ? ky : Py - ky;
    const float sy = lo ? 1.f : -1.f;
    const float* Kp = K + ((size_t)kx * Hy + kyi) * kentry(NZ);
    float kk[6 * NZ];
    kernel_load<NZ>(Kp, kk);
    float2 M[nz3], Hf[nz3];
#pragma unroll
    for (int q = 0; q < nz3; ++q) {
      M[q] = lds[((w * nz3 + q) * G + rr) * 64 + ln];
      Hf[q] = make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int zt = 0; zt < NZ; ++zt) {
#pragma unroll
      for (int zs = 0; zs < NZ; ++zs) {
        const int d = zt - zs;
        const int ad = d < 0 ? -d : d;
        const float sz = d < 0 ? -1.f : 1.f;
        const float kxx = kk[0 * NZ + ad], kyy = kk[1 * NZ + ad];
        const float kzz = kk[2 * NZ + ad], kxy = sy * kk[3 * NZ + ad];
        const float qxz = sz * kk[4 * NZ + ad];          // K_xz = -i qxz
        const float qyz = sz * sy * kk[5 * NZ + ad];     // K_yz = -i qyz
        const float2 mx = M[zs * 3 + 0], my = M[zs * 3 + 1],
                     mz = M[zs * 3 + 2];
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
    for (int q = 0; q < nz3; ++q) lds[((w * nz3 + q) * G + rr) * 64 + ln] = Hf[q];
  }
  __syncthreads();
  if (active) {
#pragma unroll
    for (int rr = 0; rr < G; ++rr) v[G0 + rr] = lds[(wv * G + rr) * 64 + lane];
  }
  if constexpr (G0 + G < NR)
    yprod_chunks<NZ, NR, G, G0 + G>(v, lds, Py, Hy, K, kx0, Wb, wv, lane,
                                    active);
}

// Spectral pass with one wavefront per column (kx, z, c) and the y FFT held
// in registers (Py = 64 * NR): the 3*nz columns of W consecutive kx form a
// workgroup; only the kernel product goes through LDS, G registers at a
// time (the product needs all columns at one ky).  Same contract as k_yspec.
template <int NZ, int NR>
__device__ __forceinline__ void yspec_w_body(
    const Prm& P, float2* __restrict__ spec, const float* __restrict__ K,
    Ctl* __restrict__ ctl, int W, const float2* __restrict__ tw,
    int logTw, const double* __restrict__ partials, int nblk_f, int stage,
    int mode, int blk, float2* lds) {
  __shared__ double red[16];
  if (blk == 0 && !P.modes) {
    finish_cavity(P, ctl, partials, nblk_f, stage, mode, red);
    __syncthreads();
  }
  constexpr int nz3 = 3 * NZ;
  constexpr int G = NR < 8 ? NR : 8;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int kx0 = blk * W;
  const int Wb = min(W, P.Hx - kx0);
  const bool active = wv < Wb * nz3;
  const int ny = P.ny, nyp = P.nyp;
  float2* col = spec + ((size_t)kx0 * nz3 + wv) * nyp;
  float2 v[NR];
  if (active) {
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int y = lane + 64 * r;
      v[r] = (y < ny) ? col[y] : make_float2(0.f, 0.f);
    }
    wfft_fwd<NR>(v, lane, tw, logTw);
  }
  yprod_chunks<NZ, NR, G, 0>(v, lds, P.Py, P.Hy, K, kx0, Wb, wv, lane, active);
  if (active) {
    wfft_inv<NR>(v, lane, tw, logTw);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int y = lane + 64 * r;
      if (y < ny) col[y] = v[r];
      else if (y < nyp) col[y] = make_float2(0.f, 0.f);   // pad stays zero
    }
  }
}

template <int NZ, int NR>
__global__ __launch_bounds__(NR >= 32 ? 512 : 1024) void k_yspec_w(
    Prm P, float2* __restrict__ spec, const float* __restrict__ K,
    Ctl* __restrict__ ctl, int W, const float2* __restrict__ tw,
    int logTw, const double* __restrict__ partials, int nblk_f, int stage,
    int mode) {
  extern __shared__ float2 lds[];
  if (ctl->done) return;
  yspec_w_body<NZ, NR>(P, spec, K, ctl, W, tw, logTw, partials, nblk_f, stage,
                       mode, blockIdx.x, lds);
}

// Local fields, LL torque and Runge-Kutta epilogue for the R rows of one
// tile (cells (x, y0 + r, z)), given B_demag through `bd(r, x)`; writes the
// stage outputs and the workgroup's partial sums (RK4 final: <m> sums,
// DP45 error stage: max error).  Any block size.
template <bool GEN, class BD>
__device__ __forceinline__ void field_cells_t(const Prm& P,
                                            const float* __restrict__ ys,
                                            const Ctl* __restrict__ ctl,
                                            double* __restrict__ partials,
                                            int stage, int R, const Epi& E,
                                            int z, int y0, BD bd,
                                            int slot) {
  __shared__ double red[16 * 3];
  __shared__ float redf[16];
  const int nx = P.nx, ny = P.ny, nz = P.nz, N = P.ncell;
  const int plane = nx * ny;
  const double dtd = ctl->dt;
  const float dt = (float)dtd;
  const double ts = ctl->t + stage_c(P, stage) * dtd;
  const float fd = (float)(P.famp * drive_shape(P.fkind, P.fw, ts));
  const float bex = P.bx + fd * P.fdx, bey = P.by + fd * P.fdy,
              bez = P.bz + fd * P.fdz;
  const float gcav = (float)(2.0 * ctl->as_re[stage]);
  float bcx = P.brx * gcav, bcy = P.bry * gcav, bcz = P.brz * gcav;
  const float* bmap = GEN ? P.brms_map : nullptr;
  // multimode cavity: sum_k B_rms,k 2 Re alpha_k (uniform vectors), or per
  // cell over the modes' maps
  float gk[kMaxModes];
  int nmodes = 0;
  bool mmap = false;
  if (GEN && P.modes) {
    const Modes& M = *P.modes;
    nmodes = M.n;
    mmap = M.any_map != 0;
    double sx = 0.0, sy = 0.0, sz = 0.0;
#pragma unroll
    for (int k = 0; k < kMaxModes; ++k) {
      const double g = k < nmodes ? 2.0 * ctl->mas_re[stage][k] : 0.0;
      gk[k] = (float)g;
      if (k < nmodes && !M.map[k]) {   // uniform modes: one vector
        sx += M.br[k][0] * g;
        sy += M.br[k][1] * g;
        sz += M.br[k][2] * g;
      }
    }
    bcx = (float)sx;
    bcy = (float)sy;
    bcz = (float)sz;
  }
  double acc[3] = {0.0, 0.0, 0.0};
  float emax = 0.f;
  const int ncellb = R * nx;
  // (r, x) of element e advanced incrementally (no division per cell)
  const int sr = blockDim.x / nx, sx = blockDim.x - sr * nx;
  int ri = threadIdx.x / nx, xi = threadIdx.x - ri * nx;
  for (int e = threadIdx.x; e < ncellb; e += blockDim.x) {
    const int r = ri, x = xi;
    xi += sx;
    ri += sr;
    if (xi >= nx) { xi -= nx; ++ri; }
    const int y = y0 + r;
    if (y >= ny) continue;
    const unsigned i = (unsigned)((z * ny + y) * nx + x);
    const unsigned Nu = (unsigned)N, N2 = 2u * Nu;
    // Every global load of the cell is issued before the first use of any:
    // a missing neighbour's index falls back to the cell itself (its
    // difference is then zero and its weight below is 0), and the earlier
    // k's sit behind uniform guards, so no load waits behind a per-lane
    // branch or behind another load's use.
    const bool hn[6] = {x > 0, x < nx - 1, y > 0, y < ny - 1, z > 0,
                        z < nz - 1};
    const int off[6] = {-1, 1, -nx, nx, -plane, plane};
    unsigned jn[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) jn[q] = hn[q] ? i + (unsigned)off[q] : i;
    const float mx = ldf(ys, i), my = ldf(ys, Nu + i), mz = ldf(ys, N2 + i);
    float nbx[6], nby[6], nbz[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      nbx[q] = ldf(ys, jn[q]);
      nby[q] = ldf(ys, Nu + jn[q]);
      nbz[q] = ldf(ys, N2 + jn[q]);
    }
    const float msv = P.ms_map ? ldf(P.ms_map, i) : P.ms;
    // Ku of the cell (2 Ku below; halving the uniform value is exact)
    const float kum = P.ku_map ? ldf(P.ku_map, i) : 0.5f * P.ku2;
    // neighbours outside the geometry (Ms = 0) are omitted like those
    // outside the grid
    const float* g = (GEN && P.masked) ? P.ms_map : nullptr;
    float gn[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) gn[q] = g ? ldf(g, jn[q]) : 1.f;
    float kpx[6], kpy[6], kpz[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      kpx[j] = kpy[j] = kpz[j] = 0.f;
      if (j < E.np) {
        kpx[j] = ldf(E.kp[j], i);
        kpy[j] = ldf(E.kp[j], Nu + i);
        kpz[j] = ldf(E.kp[j], N2 + i);
      }
    }
    float ynx = 0.f, yny = 0.f, ynz = 0.f;
    if (E.kind == 1 || E.kind == 2) {
      ynx = ldf(E.yn, i);
      yny = ldf(E.yn, Nu + i);
      ynz = ldf(E.yn, N2 + i);
    }
    if (E.commit) {
      stf(E.commit, i, mx); stf(E.commit, Nu + i, my); stf(E.commit, N2 + i, mz);
    }
    float Bx = bex + bcx, By = bey + bcy, Bz = bez + bcz;
    if (bmap) {   // per-cell vacuum field of the mode
      Bx = bex + ldf(bmap, i) * gcav;
      By = bey + ldf(bmap, Nu + i) * gcav;
      Bz = bez + ldf(bmap, N2 + i) * gcav;
    }
    if (GEN && mmap) {   // per-cell fields of the modes that have maps
#pragma unroll
      for (int k = 0; k < kMaxModes; ++k) {
        if (k >= nmodes) break;
        if (const float* b = P.modes->map[k]) {
          Bx += ldf(b, i) * gk[k];
          By += ldf(b, Nu + i) * gk[k];
          Bz += ldf(b, N2 + i) * gk[k];
        }
      }
    }
    if (GEN && P.fdrive_map) {   // field drive shaped per cell
      Bx += fd * ldf(P.fdrive_map, i);
      By += fd * ldf(P.fdrive_map, Nu + i);
      Bz += fd * ldf(P.fdrive_map, N2 + i);
    }
    if (P.demag) {
      const float3 b = bd(r, x);
      Bx += b.x;
      By += b.y;
      Bz += b.z;
    }
    if (msv > 0.f) {
      // neighbour j exists (inside the grid and the geometry)
      bool w[6];
#pragma unroll
      for (int q = 0; q < 6; ++q) w[q] = hn[q] && gn[q] > 0.f;
      // exchange: (2A/Ms) sum over existing neighbours (m_j - m_i)/d^2
      float lx = 0.f, ly = 0.f, lz = 0.f;
      const float id2[3] = {P.idx2, P.idy2, P.idz2};
#pragma unroll
      for (int q = 0; q < 6; ++q) {
        const float dx = w[q] ? nbx[q] - mx : 0.f;
        const float dy = w[q] ? nby[q] - my : 0.f;
        const float dz = w[q] ? nbz[q] - mz : 0.f;
        lx += dx * id2[q >> 1];
        ly += dy * id2[q >> 1];
        lz += dz * id2[q >> 1];
      }
      // 1/Ms: one division per cell only where Ms is a map
      const float ims = P.ms_map ? 1.f / msv : P.ims;
      const float ce = P.aex2 * ims;
      Bx += ce * lx; By += ce * ly; Bz += ce * lz;
      if (GEN && (P.dmi_i != 0.f || P.dmi_b != 0.f)) {
        // Dzyaloshinskii-Moriya: over the bonds to existing magnetic
        // neighbours j, B += (1/Ms) sum_j c_ij x m_j with
        // c_ij = D_int (z x e_ij)/d - D_bulk e_ij/d; per axis the two
        // neighbours enter as c x (m_{i+e} - m_{i-e}), a missing one omitted
        float ax = 0.f, ay = 0.f, az = 0.f;   // x bonds
        float bx = 0.f, by = 0.f, bz = 0.f;   // y bonds
        float cx = 0.f, cy = 0.f, cz = 0.f;   // z bonds
        if (w[1]) { ax += nbx[1]; ay += nby[1]; az += nbz[1]; }
        if (w[0]) { ax -= nbx[0]; ay -= nby[0]; az -= nbz[0]; }
        if (w[3]) { bx += nbx[3]; by += nby[3]; bz += nbz[3]; }
        if (w[2]) { bx -= nbx[2]; by -= nby[2]; bz -= nbz[2]; }
        if (w[5]) { cx += nbx[5]; cy += nby[5]; cz += nbz[5]; }
        if (w[4]) { cx -= nbx[4]; cy -= nby[4]; cz -= nbz[4]; }
        const float di = P.dmi_i * ims, db = P.dmi_b * ims;
        // x bonds: c = (-D_bulk, D_int, 0)/dx
        const float x0 = -db * P.idx1, x1 = di * P.idx1;
        Bx += x1 * az; By -= x0 * az; Bz += x0 * ay - x1 * ax;
        // y bonds: c = (-D_int, -D_bulk, 0)/dy
        const float y0c = -di * P.idy1, y1c = -db * P.idy1;
        Bx += y1c * bz; By -= y0c * bz; Bz += y0c * by - y1c * bx;
        // z bonds: c = (0, 0, -D_bulk)/dz
        const float z2 = -db * P.idz1;
        Bx -= z2 * cy; By += z2 * cx;
      }
      // uniaxial anisotropy (2 Ku / Ms) (u.m) u
      const float kuv = 2.f * kum;
      const float um = P.ux * mx + P.uy * my + P.uz * mz;
      const float ca =
          GEN ? (kuv * um + P.ku4 * um * um * um) * ims : (kuv * um) * ims;
      Bx += ca * P.ux; By += ca * P.uy; Bz += ca * P.uz;
      if (GEN && P.therm > 0.0) {
        // Brown's field of this step, held over its stages: variance
        // 2 alpha kB T / (gamma Ms V_c dt) per component
        double n0, n1, n2;
        thermal_normals(P, i, ctl->noise_n, n0, n1, n2);
        const double sg = sqrt(P.therm / (ctl->dt * (double)msv));
        Bx += (float)(sg * n0); By += (float)(sg * n1); Bz += (float)(sg * n2);
      }
    }
    // LL torque: -gamma/(1+a^2) [ m x B + a m x (m x B) ]
    const float px = my * Bz - mz * By;
    const float py = mz * Bx - mx * Bz;
    const float pz = mx * By - my * Bx;
    const float qx = my * pz - mz * py;
    const float qy = mz * px - mx * pz;
    const float qz = mx * py - my * px;
    const float pf = GEN ? P.prec : 1.f;
    const float kx = P.gpref * (pf * px + P.alpha * qx);
    const float ky = P.gpref * (pf * py + P.alpha * qy);
    const float kz = P.gpref * (pf * pz + P.alpha * qz);
    if (E.kout) { stf(E.kout, i, kx); stf(E.kout, Nu + i, ky); stf(E.kout, N2 + i, kz); }
    if (E.bout) { stf(E.bout, i, Bx); stf(E.bout, Nu + i, By); stf(E.bout, N2 + i, Bz); }
    if (E.kind == 0) continue;
    float sx = E.cself * kx, sy = E.cself * ky, sz = E.cself * kz;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      if (j < E.np) {
        const float cj = E.ca[j];
        sx += cj * kpx[j];
        sy += cj * kpy[j];
        sz += cj * kpz[j];
      }
    }
    if (E.kind == 3) {
      const float ex = dt * sx, ey = dt * sy, ez = dt * sz;
      const float en = sqrtf(ex * ex + ey * ey + ez * ez);
      emax = (en == en) ? fmaxf(emax, en) : INFINITY;   // NaN -> reject
      continue;
    }
    float nxv = ynx + dt * sx, nyv = yny + dt * sy, nzv = ynz + dt * sz;
    if (E.kind == 2) {
      const float nrm = sqrtf(nxv * nxv + nyv * nyv + nzv * nzv);
      if (E.nout) stf(E.nout, i, nrm);
      const float inv = nrm > 0.f ? 1.f / nrm : 0.f;   // empty cells stay 0
      nxv *= inv; nyv *= inv; nzv *= inv;
      acc[0] += nxv; acc[1] += nyv; acc[2] += nzv;
    }
    stf(E.ynext, i, nxv); stf(E.ynext, Nu + i, nyv); stf(E.ynext, N2 + i, nzv);
  }
  if (E.kind != 2 && E.kind != 3) return;
  if (E.kind == 2) {
    block_sum<3>(acc, red);
    if (threadIdx.x == 0) {
      partials[3 * slot + 0] = acc[0];
      partials[3 * slot + 1] = acc[1];
      partials[3 * slot + 2] = acc[2];
    }
  } else {
    emax = block_max(emax, redf);
    if (threadIdx.x == 0) {
      partials[slot] = (double)emax;
      // non-negative floats (and +inf) order as their bit patterns
      if (E.emax) atomicMax(E.emax, __float_as_uint(emax));
    }
  }
}


// The cell loop with the per-cell options (B_rms map, geometry, Ku2,
// precession switch) compiled in only where a problem uses one of them.
template <class BD>
__device__ __forceinline__ void field_cells(const Prm& P,
                                            const float* __restrict__ ys,
                                            const Ctl* __restrict__ ctl,
                                            double* __restrict__ partials,
                                            int stage, int R, const Epi& E,
                                            int z, int y0, BD bd, int slot) {
  if (P.plain)
    field_cells_t<false>(P, ys, ctl, partials, stage, R, E, z, y0, bd, slot);
  else
    field_cells_t<true>(P, ys, ctl, partials, stage, R, E, z, y0, bd, slot);
}


// ================================================================ k_xfield
// 1D grid of ceil(ny/R)*nz tiles (as k_xfwd); LDS: 3 * (R/2) * Px complex.
// LP > 0: log2(Px) fixed at compile time (specialised FFT addressing).
// Field pass of tile `tile` (partial sums into slot `slot`); LDS `lds`
// holds the 3 (R/2) transforms only, padded with 2 slots every 2^kPsField
// values; twiddles are read from global memory.  (The cell loop's registers
// allow two 512-thread workgroups per CU, so the LDS is padded for fewer
// bank conflicts rather than for a third workgroup.)
constexpr int kPsField = 4;
template <int T, int LP = 0>
__device__ __forceinline__ void xfield_l_body(
    const Prm& P, const float* __restrict__ ys,
    const float2* __restrict__ spec, const Ctl* __restrict__ ctl,
    double* __restrict__ partials, int stage, int R, const Epi& E,
    const float2* __restrict__ tw, int logTw, int tile, int slot,
    float2* lds) {
  constexpr int PS = kPsField;
  const int nz = P.nz;
  const int z = tile % nz;
  const int y0 = (tile / nz) * R;
  const int np = R >> 1;
  const int Px = P.Px, ny = P.ny, nyp = P.nyp;
  if (P.demag) {
    // rebuild the two-for-one spectra: Z[k] = A[k] + i B[k],
    // Z[Px-k] = conj(A[k]) + i conj(B[k]); (A, B) adjacent rows -> 16 B
    const int H = P.Hx;
    const int per = 3 * np;
    const int tot = per * H;
    constexpr int U = 4;
    // element e = k per + c np + p (column k, component c, row pair p),
    // advanced by T per step without an integer division per element
    const int dk = T / per, dr = T - dk * per;
    int ki = threadIdx.x / per, ri = threadIdx.x - ki * per;
    for (int e0 = threadIdx.x; e0 < tot; e0 += T * U) {
      float4 v[U];
      int kk[U], cc[U], pp[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = e0 + u * T;
        const int k = ki, r = ri;
        ki += dk;
        ri += dr;
        if (ri >= per) { ri -= per; ++ki; }
        const int c = (r >= np) + (r >= 2 * np), p = r - c * np;
        kk[u] = k;
        cc[u] = c;
        pp[u] = p;
        const int ya = y0 + 2 * p;
        v[u] = (e < tot && ya < ny)
                   ? ld4(spec, (unsigned)(((k * nz + z) * 3 + c) * nyp + ya)
                                   << 3)
                   : make_float4(0.f, 0.f, 0.f, 0.f);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = e0 + u * T;
        if (e >= tot) continue;
        const int k = kk[u], c = cc[u], p = pp[u];
        float2 A = make_float2(v[u].x, v[u].y), B = make_float2(v[u].z, v[u].w);
        if (k == 0 || 2 * k == Px) { A.y = 0.f; B.y = 0.f; }
        const int sp = (c * np + p) * Px;
        lds[pidx_s<PS>(sp + k)] = make_float2(A.x - B.y, A.y + B.x);
        if (k != 0 && 2 * k != Px)
          lds[pidx_s<PS>(sp + Px - k)] = make_float2(A.x + B.y, -A.y + B.x);
      }
    }
    __syncthreads();
    fft_lds<VPT, true, LP, false, true, PS>(lds, P.logPx, 3 * np, tw, logTw,
                                             1.f);
  }
  field_cells(P, ys, ctl, partials, stage, R, E, z, y0,
              [&](int r, int x) {
                const int p = r >> 1;
                const bool hi = r & 1;
                const float2 vx = lds[pidx_s<PS>((0 * np + p) * Px + x)];
                const float2 vy = lds[pidx_s<PS>((1 * np + p) * Px + x)];
                const float2 vz = lds[pidx_s<PS>((2 * np + p) * Px + x)];
                return hi ? make_float3(vx.y, vy.y, vz.y)
                          : make_float3(vx.x, vy.x, vz.x);
              }, slot);
}

template <int T, int LP = 0>
__global__ __launch_bounds__(T) void k_xfield(
    Prm P, const float* __restrict__ ys, const float2* __restrict__ spec,
    Ctl* __restrict__ ctl, double* __restrict__ partials,
    double* __restrict__ rec, int stage, int R, Epi E,
    const float2* __restrict__ tw, int logTw) {
  extern __shared__ float2 lds[];
  if (ctl->done) return;
  xfield_l_body<T, LP>(P, ys, spec, ctl, partials, stage, R, E, tw, logTw,
                       xcd_tile(blockIdx.x, gridDim.x), blockIdx.x, lds);
}

// ============================================= fused field + forward pass
// Forward x pass of one tile with the transform length fixed (LP = log2 Px)
// and the three components transformed together: Ms * y for rows y0 ..
// y0+R-1 of layer z, two rows per complex transform, into LDS laid out as
// the field pass lays out its inverse (padding kPsField, twiddles from
// global memory), so the field pass's LDS serves both; then the half
// spectrum (16-byte stores of row pairs) and the tile's FP64 coupling sum
// into partials[slot].  The arithmetic is k_xfwd's (the same radix passes).
template <int T, int LP>
__device__ __forceinline__ void xfwd3_fixed_body(
    const Prm& P, const float* __restrict__ ys, float2* __restrict__ spec,
    double* __restrict__ partials, int R, const float2* __restrict__ tw,
    int logTw, int tile, int slot, float2* lds) {
  constexpr int PS = kPsField;
  constexpr int Px = 1 << LP, xl = Px >> 1, lxl = LP - 1;
  __shared__ double red[16];
  const int nz = P.nz;
  const int z = tile % nz;
  const int y0 = (tile / nz) * R;
  const int np = R >> 1;
  const int nx = P.nx, ny = P.ny, nyp = P.nyp, N = P.ncell;
  const int plane = nx * ny;
  const float* msz = P.ms_map ? P.ms_map + (size_t)z * plane : nullptr;
  const double br[3] = {P.brxd, P.bryd, P.brzd};
  double facc[1] = {0.0};
  const int per = np << lxl;   // lower half-rows of one component
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const float* yc = ys + (size_t)c * N + (size_t)z * plane;
    double fc = 0.0;
    for (int q = threadIdx.x; q < per; q += T) {
      const int p = q >> lxl, x = q & (xl - 1);
      float2 v = make_float2(0.f, 0.f);
      if (x < nx) {
        const int ya = y0 + 2 * p;
        if (ya < ny) {
          const float msv = msz ? msz[ya * nx + x] : P.ms;
          const float mv = yc[ya * nx + x];
          v.x = msv * mv;
          fc += (double)msv * (double)mv;
        }
        if (ya + 1 < ny) {
          const float msv = msz ? msz[(ya + 1) * nx + x] : P.ms;
          const float mv = yc[(ya + 1) * nx + x];
          v.y = msv * mv;
          fc += (double)msv * (double)mv;
        }
      }
      lds[pidx_s<PS>((c * np + p) * Px + x)] = v;
    }
    facc[0] += fc * br[c];
  }
  __syncthreads();
  fft_lds<VPT, true, LP, true, false, PS>(lds, LP, 3 * np, tw, logTw, -1.f);
  constexpr int H = xl + 1;
  const int totw = np * H;
  const int dk = T / np, dp = T - dk * np;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    int k = threadIdx.x / np, p = threadIdx.x - k * np;
    for (int e = threadIdx.x; e < totw;
         e += T, k += dk, p += dp, (p >= np ? (p -= np, ++k) : 0)) {
      const int b = (c * np + p) * Px;
      const float2 z1 = lds[pidx_s<PS>(b + k)];
      const float2 z2 = lds[pidx_s<PS>(b + ((Px - k) & (Px - 1)))];
      // A = (Z[k] + conj Z[-k]) / 2 ; B = (Z[k] - conj Z[-k]) / (2i)
      float4 v = make_float4(0.5f * (z1.x + z2.x), 0.5f * (z1.y - z2.y),
                             0.5f * (z1.y + z2.y), -0.5f * (z1.x - z2.x));
      const int ya = y0 + 2 * p;
      if (ya < ny) {
        if (ya + 1 >= ny) { v.z = 0.f; v.w = 0.f; }   // keep the pad zero
        float2* row = spec + ((size_t)(k * nz + z) * 3 + c) * nyp;
        *(float4*)(row + ya) = v;
      }
    }
  }
  block_sum<1>(facc, red);
  if (threadIdx.x == 0) partials[slot] = facc[0];
}

// Stand-alone forward pass with the fused pass's tiling (the first stage of
// an attempt, whose input comes from elsewhere).
template <int T, int LP>
__global__ __launch_bounds__(T) void k_xfwd_fx(
    Prm P, const float* __restrict__ ys, float2* __restrict__ spec,
    Ctl* __restrict__ ctl, double* __restrict__ partials, int R,
    const float2* __restrict__ tw, int logTw) {
  extern __shared__ float2 lds[];
  if (ctl->done) return;
  xfwd3_fixed_body<T, LP>(P, ys, spec, partials, R, tw, logTw,
                          xcd_tile(blockIdx.x, gridDim.x), blockIdx.x, lds);
}

// Field pass of stage s fused with the forward x pass of stage s+1: the
// tile's next stage input y_{s+1} (written by the field epilogue, read back
// by the same workgroup after a barrier) is transformed into the half
// spectrum rows of this tile, which no other tile reads or writes, and the
// tile's coupling sum for stage s+1 goes to partials[blockIdx.x].  Saves
// the separate forward launch and its read of y_{s+1} from HBM.
template <int T, int LP>
__global__ __launch_bounds__(T) void k_xfield_fwd(
    Prm P, const float* __restrict__ ys, float2* __restrict__ spec,
    Ctl* __restrict__ ctl, double* __restrict__ partials,
    double* __restrict__ rec, int stage, int R, Epi E,
    const float2* __restrict__ tw, int logTw) {
  extern __shared__ float2 lds[];
  if (ctl->done) return;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  xfield_l_body<T, LP>(P, ys, spec, ctl, partials, stage, R, E, tw, logTw,
                       tile, blockIdx.x, lds);
  __syncthreads();
  xfwd3_fixed_body<T, LP>(P, E.ynext, spec, partials, R, tw, logTw, tile,
                          blockIdx.x, lds);
}

// The field pass of the batch plan: partial sums indexed by tile (as the
// batched kernels index them), so that both sum in the same order.
template <int T>
__global__ __launch_bounds__(T) void k_xfield_b(
    Prm P, const float* __restrict__ ys, const float2* __restrict__ spec,
    Ctl* __restrict__ ctl, double* __restrict__ partials,
    double* __restrict__ rec, int stage, int R, Epi E,
    const float2* __restrict__ tw, int logTw) {
  extern __shared__ float2 lds[];
  if (ctl->done) return;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  xfield_l_body<T, 0>(P, ys, spec, ctl, partials, stage, R, E, tw, logTw,
                      tile, tile, lds);
}

// ============================================================== k_xfield_w
// Field kernel with the x inverse FFT in registers (Px = 64 * NR): one
// wavefront per (component, row pair) of an R-row tile gathers its
// two-for-one spectrum straight from the half spectrum in the wavefront-FFT
// input order, transforms, and leaves B_demag of its two rows in LDS
// (3 * R * nx floats); then all threads run the cell loop.
template <int NR>
__device__ __forceinline__ void xfield_w_body(
    const Prm& P, const float* __restrict__ ys,
    const float2* __restrict__ spec, const Ctl* __restrict__ ctl,
    double* __restrict__ partials, int stage, int R, const Epi& E,
    const float2* __restrict__ tw, int logTw, int tile, int slot,
    float* bdl) {
  constexpr int LNR = Log2<NR>::v;
  const int nz = P.nz;
  const int z = tile % nz;
  const int y0 = (tile / nz) * R;
  const int np = R >> 1;
  const int Px = P.Px, nx = P.nx, ny = P.ny, nyp = P.nyp;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (P.demag && wv < 3 * np) {
    const int c = wv / np, p = wv - c * np;
    const int ya = y0 + 2 * p;
    float2 v[NR];
    if (ya < ny) {
      const int b2 = NR * brev_bits(lane, 6);
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const int k = brev_bits(r, LNR) + b2;
        const bool lo = 2 * k <= Px;
        const int kk = lo ? k : Px - k;
        const float4 ab = *(const float4*)(spec +
                                           ((size_t)(kk * nz + z) * 3 + c) * nyp + ya);
        float2 A = make_float2(ab.x, ab.y), B = make_float2(ab.z, ab.w);
        if (kk == 0 || 2 * kk == Px) { A.y = 0.f; B.y = 0.f; }
        v[r] = lo ? make_float2(A.x - B.y, A.y + B.x)
                  : make_float2(A.x + B.y, -A.y + B.x);
      }
    } else {
#pragma unroll
      for (int r = 0; r < NR; ++r) v[r] = make_float2(0.f, 0.f);
    }
    wfft_inv<NR>(v, lane, tw, logTw);
    float* b0 = bdl + (size_t)(c * R + 2 * p) * nx;
    float* b1 = b0 + nx;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int x = lane + 64 * r;
      if (x < nx) { b0[x] = v[r].x; b1[x] = v[r].y; }
    }
  }
  __syncthreads();
  field_cells(P, ys, ctl, partials, stage, R, E, z, y0,
              [&](int r, int x) {
                return make_float3(bdl[(0 * R + r) * nx + x],
                                   bdl[(1 * R + r) * nx + x],
                                   bdl[(2 * R + r) * nx + x]);
              }, slot);
}

template <int NR>
__global__ __launch_bounds__(NR >= 32 ? 512 : 1024) void k_xfield_w(
    Prm P, const float* __restrict__ ys, const float2* __restrict__ spec,
    Ctl* __restrict__ ctl, double* __restrict__ partials,
    double* __restrict__ rec, int stage, int R, Epi E,
    const float2* __restrict__ tw, int logTw) {
  extern __shared__ float bdl[];
  if (ctl->done) return;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  xfield_w_body<NR>(P, ys, spec, ctl, partials, stage, R, E, tw, logTw,
                    tile, tile, bdl);
}

// Dormand-Prince step controller: the decision on an attempt from the
// largest per-cell error (errm) and the control block as the attempt left
// it (dp_decide reads only), and its application (dp_commit writes).
struct DpDecision {
  bool accept, bad, done;
  double err, t, dt;   // err of the attempt; t and next dt after it
  int status;
};
__device__ inline void dp_decide(const Prm& P, const Ctl* c, double errm,
                                 DpDecision& d) {
  const double err = fmax(errm, c->err_a);
  d.bad = !isfinite(err);
  d.err = err;
  const double h = c->dt;
  double fac;
  d.accept = !d.bad && err <= P.tol;
  int acc = c->accepted;
  d.t = c->t;
  if (d.accept) {
    fac = (err == 0.0) ? 5.0 : fmin(5.0, fmax(0.2, 0.9 * pow(P.tol / err, 0.2)));
    if (c->prev_rej) fac = fmin(fac, 1.0);
    d.t = c->t + h;
    acc += 1;
  } else {
    fac = d.bad ? 0.2 : fmax(0.2, 0.9 * pow(P.tol / err, 0.2));
  }
  double dtn = fmin(P.dt_max, h * fac);
  d.done = c->done || d.t >= c->t_end || acc >= c->max_accepted;
  d.status = d.bad ? ST_NONFINITE : ST_OK;
  if (dtn < P.dt_min) {
    if (!d.bad) d.status = ST_UNDERFLOW;
    d.done = true;
  }
  if (!d.done) dtn = fmin(dtn, c->t_end - d.t);
  d.dt = dtn;
}
__device__ inline void dp_commit(const Prm& P, Ctl* c, const DpDecision& d) {
  if (d.accept) {
    c->t = d.t;
    c->a_re = c->as_re[7];
    c->a_im = c->as_im[7];
    c->as_re[1] = c->a_re;
    c->as_im[1] = c->a_im;
    c->ka_re[1] = c->ka_re[7];
    c->ka_im[1] = c->ka_im[7];
    if (P.modes)
      for (int k = 0; k < P.modes->n; ++k) {
        c->ma_re[k] = c->mas_re[1][k] = c->mas_re[7][k];
        c->ma_im[k] = c->mas_im[1][k] = c->mas_im[7][k];
        c->mka_re[1][k] = c->mka_re[7][k];
        c->mka_im[1][k] = c->mka_im[7][k];
      }
    c->accepted += 1;
    c->pending_accept = 1;
    c->prev_rej = 0;
  } else {
    c->prev_rej = 1;
    c->rejected += 1;
    c->pending_accept = 0;
  }
  c->last_err = d.bad ? INFINITY : d.err;
  if (d.done) c->done = 1;
  c->status = d.status;
  const double dtn = d.dt;
  c->dt = dtn;
  // second stage amplitude of the next attempt
  c->as_re[2] = c->a_re + dtn * c_dp_a[2][0] * c->ka_re[1];
  c->as_im[2] = c->a_im + dtn * c_dp_a[2][0] * c->ka_im[1];
  if (P.modes)
    for (int k = 0; k < P.modes->n; ++k) {
      c->mas_re[2][k] = c->ma_re[k] + dtn * c_dp_a[2][0] * c->mka_re[1][k];
      c->mas_im[2][k] = c->ma_im[k] + dtn * c_dp_a[2][0] * c->mka_im[1][k];
    }
}

// End of a step, one workgroup: RK4 commit and record (kind 2) or the
// Dormand-Prince step controller (kind 3), from the k_xfield partials.
// `ndone` (optional) counts the runs this call finishes.
__device__ __forceinline__ void finish_step_body(
    const Prm& P, Ctl* __restrict__ ctl, const double* __restrict__ partials,
    int nblk, int kind, double* __restrict__ rec, int* __restrict__ ndone) {
  __shared__ double red[16 * 3];
  const int N = P.ncell;
  double S[3] = {0.0, 0.0, 0.0};
  double errm = 0.0;
  if (kind == 2) sum_partials<3>(partials, nblk, S, red);
  else errm = max_partials(partials, nblk, red);
  if (threadIdx.x != 0) return;
  Ctl* c = ctl;
  if (kind == 2) {
    // RK4: the new state (in a scratch register) and amplitude are committed
    // only when finite; otherwise the run stops with y_n, t and alpha those
    // of the last accepted step
    const double s0 = S[0], s1 = S[1], s2 = S[2];
    bool fin = isfinite(s0) && isfinite(s1) && isfinite(s2) &&
               isfinite(c->anext_re) && isfinite(c->anext_im);
    if (P.modes)
      for (int k = 0; k < P.modes->n; ++k)
        fin = fin && isfinite(c->manext_re[k]) && isfinite(c->manext_im[k]);
    if (!fin) {
      c->status = ST_NONFINITE;
      c->done = 1;
      if (ndone) atomicAdd(ndone, 1);
      return;
    }
    c->t = c->t + c->dt;
    c->a_re = c->anext_re;
    c->a_im = c->anext_im;
    if (P.modes)
      for (int k = 0; k < P.modes->n; ++k) {
        c->ma_re[k] = c->mas_re[1][k] = c->manext_re[k];
        c->ma_im[k] = c->mas_im[1][k] = c->manext_im[k];
      }
    c->mem_n += 1;
    c->noise_n += 1;
    c->as_re[1] = c->a_re;
    c->as_im[1] = c->a_im;
    if (c->ahist) {
      double* h = c->ahist + 2 * (5 * c->accepted + 4);
      h[0] = c->a_re;
      h[1] = c->a_im;
    }
    c->accepted += 1;
    if (c->accepted >= c->loss_n0 && c->accepted <= c->loss_n1)
      c->loss_acc += c->a_re * c->a_re + c->a_im * c->a_im;
    if (c->max_accepted > 0 && c->accepted >= c->max_accepted) c->done = 1;
    if (c->rec_every > 0 && (c->accepted % c->rec_every) == 0 &&
        c->nrec < c->rec_cap) {
      double* row = rec + (size_t)P.recw * c->nrec;
      row[0] = c->t;
      row[1] = s0 / P.nmag;
      row[2] = s1 / P.nmag;
      row[3] = s2 / P.nmag;
      record_amplitudes(P, c, row);
      c->nrec += 1;
    }
  } else {
    DpDecision d;
    dp_decide(P, c, errm, d);
    dp_commit(P, c, d);
  }
  if (ndone && c->done) atomicAdd(ndone, 1);
}

template <int T>
__global__ __launch_bounds__(T) void k_finish_step(
    Prm P, Ctl* __restrict__ ctl, const double* __restrict__ partials,
    int nblk, int kind, double* __restrict__ rec) {
  if (ctl->done) return;
  finish_step_body(P, ctl, partials, nblk, kind, rec, nullptr);
}

// ================================================================= k_begin
// Start of a Dormand-Prince attempt: commit an accepted step (renormalise
// y7 into y_n, FSAL k7 -> k1, record), form y2 = y_n + dt a21 k1.
// Requires N % 4 == 0 for the vector path (scalar tail otherwise).
// Workgroup `blk` of `nblk` (grid-stride over the cells of one run).
// The cell work of an attempt's start: with `pend` (an accepted step) y_n =
// y7 renormalised and k1 = k7 (FSAL), summing y_n into acc; unless `done`,
// y2 = y_n + c21 k1.  Workgroup `blk` of `nblk`.
template <int T>
__device__ __forceinline__ void begin_cells(
    const Prm& P, float* __restrict__ yn, float* __restrict__ k1,
    const float* __restrict__ y7, const float* __restrict__ k7,
    float* __restrict__ y2, bool pend, bool done, float c21, int blk,
    int nblk, double (&acc)[3]) {
  const int N = P.ncell;
  const int n4 = N >> 2;
  const int stride = nblk * T;
  // component planes as float4 (N % 4 == 0 checked by the host; the
  // remainder loop below covers the rest)
  const int nvec = (N % 4 == 0) ? n4 : 0;
  for (int q = blk * T + threadIdx.x; q < nvec; q += stride) {
    float4 m[3], k[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const unsigned o = (unsigned)(c * N + 4 * q) << 2;
      if (pend) {
        m[c] = ld4(y7, o);
        k[c] = ld4(k7, o);
      } else {
        m[c] = ld4(yn, o);
        k[c] = ld4(k1, o);
      }
    }
    if (pend) {
      float* mx = &m[0].x; float* my = &m[1].x; float* mz = &m[2].x;
#pragma unroll
      for (int l = 0; l < 4; ++l) {
        const float n2 = mx[l] * mx[l] + my[l] * my[l] + mz[l] * mz[l];
        const float inv = n2 > 0.f ? 1.f / sqrtf(n2) : 0.f;
        mx[l] *= inv; my[l] *= inv; mz[l] *= inv;
        acc[0] += mx[l]; acc[1] += my[l]; acc[2] += mz[l];
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const unsigned o = (unsigned)(c * N + 4 * q) << 2;
        st4(yn, o, m[c]);
        st4(k1, o, k[c]);
      }
    }
    if (!done) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        float4 o;
        o.x = m[c].x + c21 * k[c].x; o.y = m[c].y + c21 * k[c].y;
        o.z = m[c].z + c21 * k[c].z; o.w = m[c].w + c21 * k[c].w;
        st4(y2, (unsigned)(c * N + 4 * q) << 2, o);
      }
    }
  }
  for (int i = 4 * nvec + blk * T + threadIdx.x; i < N; i += stride) {
    float mx, my, mz, kx, ky, kz;
    if (pend) {
      mx = y7[i]; my = y7[N + i]; mz = y7[2 * N + i];
      const float n2 = mx * mx + my * my + mz * mz;
      const float inv = n2 > 0.f ? 1.f / sqrtf(n2) : 0.f;
      mx *= inv; my *= inv; mz *= inv;
      yn[i] = mx; yn[N + i] = my; yn[2 * N + i] = mz;
      kx = k7[i]; ky = k7[N + i]; kz = k7[2 * N + i];
      k1[i] = kx; k1[N + i] = ky; k1[2 * N + i] = kz;
      acc[0] += mx; acc[1] += my; acc[2] += mz;
    } else {
      mx = yn[i]; my = yn[N + i]; mz = yn[2 * N + i];
      kx = k1[i]; ky = k1[N + i]; kz = k1[2 * N + i];
    }
    if (!done) {
      y2[i] = mx + c21 * kx; y2[N + i] = my + c21 * ky;
      y2[2 * N + i] = mz + c21 * kz;
    }
  }
}

template <int T>
__device__ __forceinline__ void begin_body(
    const Prm& P, float* __restrict__ yn, float* __restrict__ k1,
    const float* __restrict__ y7, const float* __restrict__ k7,
    float* __restrict__ y2, Ctl* __restrict__ ctl,
    double* __restrict__ partials, double* __restrict__ rec, int blk,
    int nblk) {
  __shared__ double red[16 * 3];
  __shared__ bool amlast;
  const int pend = ctl->pending_accept;
  const int done = ctl->done;
  if (done && !pend) return;
  // the average is reduced only when this accepted step is recorded
  const bool rec_due = pend && ctl->rec_every > 0 && ctl->nrec < ctl->rec_cap &&
                       (ctl->accepted % ctl->rec_every) == 0;
  const float c21 = (float)(ctl->dt * c_dp_a[2][0]);
  double acc[3] = {0.0, 0.0, 0.0};
  begin_cells<T>(P, yn, k1, y7, k7, y2, pend, done, c21, blk, nblk, acc);
  if (!pend) return;
  if (!rec_due) {
    // every block saw pend = 1; clear it from the last one to arrive, once
    // every wave of this block is past its read of the flag
    __syncthreads();
    if (threadIdx.x == 0) {
      const unsigned int prev = atomicAdd(&ctl->cnt_begin, 1u);
      if (prev == nblk - 1) {
        ctl->pending_accept = 0;
        ctl->cnt_begin = 0;
      }
    }
    return;
  }
  block_sum<3>(acc, red);
  if (threadIdx.x == 0) {
    partials[3 * blk + 0] = acc[0];
    partials[3 * blk + 1] = acc[1];
    partials[3 * blk + 2] = acc[2];
  }
  if (!last_block(&ctl->cnt_begin, nblk, &amlast)) return;
  double S[3];
  sum_partials<3>(partials, nblk, S, red);
  if (threadIdx.x != 0) return;
  {
    double* row = rec + (size_t)P.recw * ctl->nrec;
    row[0] = ctl->t;
    row[1] = S[0] / P.nmag;
    row[2] = S[1] / P.nmag;
    row[3] = S[2] / P.nmag;
    record_amplitudes(P, ctl, row);
    ctl->nrec += 1;
  }
  ctl->pending_accept = 0;
  ctl->cnt_begin = 0;
}

template <int T>
__global__ __launch_bounds__(T) void k_begin(
    Prm P, float* __restrict__ yn, float* __restrict__ k1,
    const float* __restrict__ y7, const float* __restrict__ k7,
    float* __restrict__ y2, Ctl* __restrict__ ctl,
    double* __restrict__ partials, double* __restrict__ rec) {
  begin_body<T>(P, yn, k1, y7, k7, y2, ctl, partials, rec, blockIdx.x,
                gridDim.x);
}

// End of a Dormand-Prince attempt and start of the next in one launch (one
// run): every workgroup takes the step controller's decision from the
// attempt's largest error (the field pass's atomic maximum in the control
// block) and the control block as the attempt left it, then does the
// start's cell work with it.  The last workgroup to arrive -- every other
// one is past its reads of the control block by then -- commits the
// decision, clears the maximum and writes the record row.
template <int T>
__global__ __launch_bounds__(T) void k_step_begin(
    Prm P, float* __restrict__ yn, float* __restrict__ k1,
    const float* __restrict__ y7, const float* __restrict__ k7,
    float* __restrict__ y2, Ctl* __restrict__ ctl,
    double* __restrict__ partials, double* __restrict__ rec) {
  __shared__ double red[16 * 3];
  __shared__ bool amlast;
  __shared__ int sflag[3];
  __shared__ float sc21;
  if (ctl->done) return;
  const int blk = blockIdx.x, nblk = gridDim.x;
  DpDecision d;
  if (threadIdx.x == 0) {
    dp_decide(P, ctl, (double)__uint_as_float(ctl->emax_bits), d);
    sflag[0] = d.accept;
    sflag[1] = d.done;
    sflag[2] = d.accept && ctl->rec_every > 0 && ctl->nrec < ctl->rec_cap &&
               ((ctl->accepted + 1) % ctl->rec_every) == 0;
    sc21 = (float)(d.dt * c_dp_a[2][0]);
  }
  __syncthreads();
  // wave-uniform (scalar) copies, so that the cell loops branch as k_begin's
  const bool pend = __builtin_amdgcn_readfirstlane(sflag[0]) != 0;
  const bool done = __builtin_amdgcn_readfirstlane(sflag[1]) != 0;
  const bool rec_due = __builtin_amdgcn_readfirstlane(sflag[2]) != 0;
  const float c21 = __int_as_float(
      __builtin_amdgcn_readfirstlane(__float_as_int(sc21)));
  double acc[3] = {0.0, 0.0, 0.0};
  if (pend || !done)
    begin_cells<T>(P, yn, k1, y7, k7, y2, pend, done, c21, blk, nblk, acc);
  double S[3] = {0.0, 0.0, 0.0};
  if (rec_due) {
    // the record's sums are published to the last workgroup (fenced)
    block_sum<3>(acc, red);
    if (threadIdx.x == 0) {
      partials[3 * blk + 0] = acc[0];
      partials[3 * blk + 1] = acc[1];
      partials[3 * blk + 2] = acc[2];
    }
    if (!last_block(&ctl->cnt_begin, nblk, &amlast)) return;
    sum_partials<3>(partials, nblk, S, red);
    if (threadIdx.x != 0) return;
  } else {
    // nothing to publish: every wave of this workgroup read the control
    // block before the barrier above, so a bare count suffers no device
    // fence (which would write back this XCD's L2)
    if (threadIdx.x != 0) return;
    if (atomicAdd(&ctl->cnt_begin, 1u) != (unsigned int)nblk - 1) return;
  }
  dp_commit(P, ctl, d);
  ctl->pending_accept = 0;
  ctl->emax_bits = 0u;
  if (rec_due) {
    double* row = rec + (size_t)P.recw * ctl->nrec;
    row[0] = ctl->t;
    row[1] = S[0] / P.nmag;
    row[2] = S[1] / P.nmag;
    row[3] = S[2] / P.nmag;
    record_amplitudes(P, ctl, row);
    ctl->nrec += 1;
  }
  ctl->cnt_begin = 0;
}

// ========================================================== k_torque_stats
// Per-workgroup sum and maximum of |k_i|^2 over the magnetic cells of a
// 3N-float field k (relax's stopping rule), to part[2 b], part[2 b + 1].
template <int T>
__global__ __launch_bounds__(T) void k_torque_stats(
    Prm P, const float* __restrict__ k, double* __restrict__ part) {
  __shared__ double red[16];
  __shared__ double redm[16];
  const int N = P.ncell;
  double s2 = 0.0, mx = 0.0;
  for (int i = blockIdx.x * T + threadIdx.x; i < N; i += gridDim.x * T) {
    if (P.ms_map && !(P.ms_map[i] > 0.f)) continue;
    const double a = k[i], b = k[N + i], c = k[2 * N + i];
    const double n2 = a * a + b * b + c * c;
    s2 += n2;
    mx = fmax(mx, n2);
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int o = 32; o > 0; o >>= 1) {
    s2 += __shfl_xor(s2, o, 64);
    mx = fmax(mx, __shfl_xor(mx, o, 64));
  }
  if (lane == 0) {
    red[w] = s2;
    redm[w] = mx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0;
    for (int j = 0; j < T / 64; ++j) {
      a += red[j];
      b = fmax(b, redm[j]);
    }
    part[2 * blockIdx.x] = a;
    part[2 * blockIdx.x + 1] = b;
  }
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
  double S[3];
  sum_partials<3>(partials, gridDim.x, S, red);
  if (threadIdx.x != 0) return;
  if (ctl->nrec < ctl->rec_cap) {
    double* row = rec + (size_t)P.recw * ctl->nrec;
    row[0] = ctl->t;
    row[1] = S[0] / P.nmag;
    row[2] = S[1] / P.nmag;
    row[3] = S[2] / P.nmag;
    record_amplitudes(P, ctl, row);
    ctl->nrec += 1;
  }
  ctl->cnt_rec = 0;
}

}  // namespace llgc
