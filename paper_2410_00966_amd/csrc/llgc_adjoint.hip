// Discrete adjoint of the RK4 cavity-LLG step (gfx950).
//
// Reverse-mode differentiation of the forward map of one RK4 step
//   Y1 = (m_n, a_n); K_s = f(Y_s, t_s); Y2 = Y1 + dt/2 K1; Y3 = Y1 + dt/2 K2;
//   Y4 = Y1 + dt K3; m^ = m_n + dt/6 (K1 + 2K2 + 2K3 + K4);
//   m_{n+1} = m^/|m^|; a_{n+1} = a_n + dt/6 (...)
// given lam = dL/d(m_{n+1}, a_{n+1}):
//   lam^ = (I - m m^T) lam_m / |m^|  (cavity part unchanged),
//   lamK4 = dt/6 lam^,           lamY4 = J(Y4)^T lamK4,
//   lamK3 = dt/3 lam^ + dt lamY4, lamY3 = J(Y3)^T lamK3,
//   lamK2 = dt/3 lam^ + dt/2 lamY3, ...,  lamK1 = dt/6 lam^ + dt/2 lamY2,
//   lam_n = lam^ + lamY1 + lamY2 + lamY3 + lamY4,
// where J(Y)^T v is the vector-Jacobian product of the right-hand side:
//   torque: with p = -gamma/(1+alpha^2), t = p (m x B + alpha m x (m x B)),
//     dL/dB = p (v x m + alpha (m (m.v) - v |m|^2)),
//     dL/dm = p (B x v + alpha (v (m.B) + B (m.v) - 2 m (B.v)));
//   anisotropy B_a = (2Ku/Ms)(u.m)u, exchange B_ex = (2A/Ms) L m (L the
//   symmetric open-boundary Laplacian: transpose = L applied to
//   2A lamB/Ms), demag B_d = -mu0 N*(Ms m) (symmetric, even kernel: the
//   convolution is self-adjoint), cavity field B_rms 2 Re a;
//   cavity rate -(i wc + kappa) a + i (V/hbar) sum Ms m.B_rms - i eps0 f(t).
// Parameter gradients (Ms map, Ku map, B_rms, eps0) accumulate in FP64.
#include <hip/hip_runtime.h>

namespace llgc {

// Adjoint scalar state (device).
struct AdjCtl {
  double lam_re, lam_im;     // adjoint of alpha at the current step end
  double hat_re, hat_im;     // lam^ cavity part (= lam, no renormalisation)
  double acc_re, acc_im;     // running lam_n (cavity)
  double lk_re, lk_im;       // lamK (cavity) of the stage being processed
  double g_brms[3];
  double g_eps0;
  double loss_scale;         // 1/|W|
};

// Renormalisation VJP and start of the step's reverse sweep.
// m_end = m_{n+1}, nrm = |m^|; lam (in) -> hat; acc = hat; lamK = dt/6 hat.
__global__ __launch_bounds__(256) void k_adj_begin(
    int N, const float* __restrict__ m_end, const float* __restrict__ nrm,
    const float* __restrict__ lam, float* __restrict__ hat,
    float* __restrict__ acc, float* __restrict__ lamK, float c4) {
  for (int i = blockIdx.x * 256 + threadIdx.x; i < N; i += gridDim.x * 256) {
    const float mx = m_end[i], my = m_end[N + i], mz = m_end[2 * N + i];
    const float lx = lam[i], ly = lam[N + i], lz = lam[2 * N + i];
    const float dot = mx * lx + my * ly + mz * lz;
    const float inv = 1.f / nrm[i];
    const float hx = (lx - mx * dot) * inv, hy = (ly - my * dot) * inv,
                hz = (lz - mz * dot) * inv;
    hat[i] = hx; hat[N + i] = hy; hat[2 * N + i] = hz;
    acc[i] = hx; acc[N + i] = hy; acc[2 * N + i] = hz;
    lamK[i] = c4 * hx; lamK[N + i] = c4 * hy; lamK[2 * N + i] = c4 * hz;
  }
}

// Cavity part of the step start: loss term, hat, acc, lamK = dt/6 hat.
__global__ void k_adj_begin_scalar(AdjCtl* __restrict__ A,
                                   const double* __restrict__ a_end,
                                   int in_window, double c4) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double lr = A->lam_re, li = A->lam_im;
  if (in_window) {
    lr += 2.0 * A->loss_scale * a_end[0];
    li += 2.0 * A->loss_scale * a_end[1];
  }
  A->hat_re = lr; A->hat_im = li;
  A->acc_re = lr; A->acc_im = li;
  A->lk_re = c4 * lr; A->lk_im = c4 * li;
}

// Local part of J(Y_s)^T lamK: torque, anisotropy, cavity coupling.
// Writes lamB (field adjoint) and lamM (local m adjoint); FP64 partial sums
// per workgroup: [0] sum B_rms.lamB, [1..3] sum lamB, [4..6] sum Ms m.
// Gradient contributions of the anisotropy to g_ku, g_ms.
__global__ __launch_bounds__(256) void k_vjp_local(
    Prm P, const float* __restrict__ Y, const float* __restrict__ B,
    const float* __restrict__ lamK, const AdjCtl* __restrict__ A,
    float* __restrict__ lamB, float* __restrict__ lamM,
    double* __restrict__ g_ms, double* __restrict__ g_ku,
    double* __restrict__ partials) {
  __shared__ double red[16 * 7];
  const int N = P.ncell;
  // lam_F = (V/hbar) * Im(lamK_a): adjoint of the coupling sum F
  const double lamF = P.vc_hbar * A->lk_im;
  const float lamFf = (float)lamF;
  double s[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int i = blockIdx.x * 256 + threadIdx.x; i < N; i += gridDim.x * 256) {
    const float mx = Y[i], my = Y[N + i], mz = Y[2 * N + i];
    const float Bx = B[i], By = B[N + i], Bz = B[2 * N + i];
    const float vx = lamK[i], vy = lamK[N + i], vz = lamK[2 * N + i];
    const float p = P.gpref, al = P.alpha;
    const float mv = mx * vx + my * vy + mz * vz;
    const float mB = mx * Bx + my * By + mz * Bz;
    const float Bv = Bx * vx + By * vy + Bz * vz;
    const float mm = mx * mx + my * my + mz * mz;
    // dL/dB = p (v x m + alpha (m (m.v) - v |m|^2))
    const float bx = p * ((vy * mz - vz * my) + al * (mx * mv - vx * mm));
    const float by = p * ((vz * mx - vx * mz) + al * (my * mv - vy * mm));
    const float bz = p * ((vx * my - vy * mx) + al * (mz * mv - vz * mm));
    // dL/dm (torque) = p (B x v + alpha (v (m.B) + B (m.v) - 2 m (B.v)))
    float lx = p * ((By * vz - Bz * vy) + al * (vx * mB + Bx * mv - 2.f * mx * Bv));
    float ly = p * ((Bz * vx - Bx * vz) + al * (vy * mB + By * mv - 2.f * my * Bv));
    float lz = p * ((Bx * vy - By * vx) + al * (vz * mB + Bz * mv - 2.f * mz * Bv));
    const float msv = P.ms_map ? P.ms_map[i] : P.ms;
    if (msv > 0.f) {
      const float kuv = P.ku_map ? P.ku_map[i] : 0.5f * P.ku2;
      const float um = P.ux * mx + P.uy * my + P.uz * mz;
      const float ub = P.ux * bx + P.uy * by + P.uz * bz;
      const float ca = 2.f * kuv / msv * ub;
      lx += ca * P.ux; ly += ca * P.uy; lz += ca * P.uz;
      g_ku[i] += (double)(2.f / msv * um * ub);
      g_ms[i] += (double)(-2.f * kuv / (msv * msv) * um * ub);
    }
    // coupling sum F = sum Ms m.B_rms
    lx += lamFf * msv * P.brx; ly += lamFf * msv * P.bry;
    lz += lamFf * msv * P.brz;
    g_ms[i] += lamF * (double)(mx * P.brx + my * P.bry + mz * P.brz);
    lamB[i] = bx; lamB[N + i] = by; lamB[2 * N + i] = bz;
    lamM[i] = lx; lamM[N + i] = ly; lamM[2 * N + i] = lz;
    s[0] += (double)(P.brx * bx + P.bry * by + P.brz * bz);
    s[1] += bx; s[2] += by; s[3] += bz;
    s[4] += (double)msv * mx; s[5] += (double)msv * my; s[6] += (double)msv * mz;
  }
  block_sum<7>(s, red);
  if (threadIdx.x == 0)
    for (int k = 0; k < 7; ++k) partials[7 * blockIdx.x + k] = s[k];
}

// Non-local part: demag adjoint (C lamB from the spectral pipeline, in LDS
// after the x inverse FFT), exchange transpose, Ms gradients; then the RK4
// reverse combination: acc += lamY; lamK = cK * hat + cY * lamY (if cY != 0).
template <int NR>
__global__ __launch_bounds__(NR >= 32 ? 512 : 1024) void k_vjp_field_w(
    Prm P, const float* __restrict__ Y, const float2* __restrict__ spec,
    const float* __restrict__ lamB, const float* __restrict__ lamM,
    double* __restrict__ g_ms, float* __restrict__ acc,
    const float* __restrict__ hat, float* __restrict__ lamK, float cK,
    float cY, int R, const float2* __restrict__ tw, int logTw) {
  extern __shared__ float bdl[];
  constexpr int LNR = Log2<NR>::v;
  const int nblk = gridDim.x;
  const int nz = P.nz;
  const int tile = xcd_tile(blockIdx.x, nblk);
  const int z = tile % nz;
  const int y0 = (tile / nz) * R;
  const int np = R >> 1;
  const int Px = P.Px, nx = P.nx, ny = P.ny, nyp = P.nyp, N = P.ncell;
  const int plane = nx * ny;
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
        float2 Aq = make_float2(ab.x, ab.y), Bq = make_float2(ab.z, ab.w);
        if (kk == 0 || 2 * kk == Px) { Aq.y = 0.f; Bq.y = 0.f; }
        v[r] = lo ? make_float2(Aq.x - Bq.y, Aq.y + Bq.x)
                  : make_float2(Aq.x + Bq.y, -Aq.y + Bq.x);
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
  const int ncellb = R * nx;
  for (int e = threadIdx.x; e < ncellb; e += blockDim.x) {
    const int r = e / nx, x = e - r * nx;
    const int y = y0 + r;
    if (y >= ny) continue;
    const int i = (z * ny + y) * nx + x;
    const float msv = P.ms_map ? P.ms_map[i] : P.ms;
    float lx = lamM[i], ly = lamM[N + i], lz = lamM[2 * N + i];
    if (msv > 0.f) {
      float cx = 0.f, cy = 0.f, cz = 0.f;
      if (P.demag) {
        cx = bdl[(0 * R + r) * nx + x];
        cy = bdl[(1 * R + r) * nx + x];
        cz = bdl[(2 * R + r) * nx + x];
      }
      const float mx = Y[i], my = Y[N + i], mz = Y[2 * N + i];
      lx += msv * cx; ly += msv * cy; lz += msv * cz;
      // exchange transpose: sum_nb (2A/d^2) (lamB_j/Ms_j - lamB_i/Ms_i),
      // and g_ms from B_ex,i = (2A/Ms_i) sum_nb (m_j - m_i)/d^2
      const float bix = lamB[i], biy = lamB[N + i], biz = lamB[2 * N + i];
      const float wi = P.aex2 / msv;
      float tx = 0.f, ty = 0.f, tz = 0.f;
      float ex = 0.f, ey = 0.f, ez = 0.f;
      auto nb = [&](int j, float id2) {
        const float msj = P.ms_map ? P.ms_map[j] : P.ms;
        const float wj = msj > 0.f ? P.aex2 / msj : 0.f;
        tx += id2 * (wj * lamB[j] - wi * bix);
        ty += id2 * (wj * lamB[N + j] - wi * biy);
        tz += id2 * (wj * lamB[2 * N + j] - wi * biz);
        ex += id2 * (Y[j] - mx);
        ey += id2 * (Y[N + j] - my);
        ez += id2 * (Y[2 * N + j] - mz);
      };
      if (x > 0) nb(i - 1, P.idx2);
      if (x < nx - 1) nb(i + 1, P.idx2);
      if (y > 0) nb(i - nx, P.idy2);
      if (y < ny - 1) nb(i + nx, P.idy2);
      if (z > 0) nb(i - plane, P.idz2);
      if (z < nz - 1) nb(i + plane, P.idz2);
      lx += tx; ly += ty; lz += tz;
      // dB_ex,i/dMs_i = -B_ex,i/Ms_i ; dB_d/dMs enters through M = Ms m
      const float bex = wi * (bix * ex + biy * ey + biz * ez);
      g_ms[i] += (double)(mx * cx + my * cy + mz * cz) - (double)(bex / msv);
    }
    acc[i] += lx; acc[N + i] += ly; acc[2 * N + i] += lz;
    if (cY != 0.f) {
      lamK[i] = cK * hat[i] + cY * lx;
      lamK[N + i] = cK * hat[N + i] + cY * ly;
      lamK[2 * N + i] = cK * hat[2 * N + i] + cY * lz;
    }
  }
}

// Cavity part of one stage's VJP, one workgroup: finishes the sums of
// k_vjp_local; lamY_a = adjoint of a_s, accumulates acc_a and gradients,
// and forms the cavity lamK of the previous stage.
__global__ __launch_bounds__(256) void k_vjp_scalar(
    Prm P, AdjCtl* __restrict__ A, const double* __restrict__ partials,
    int nblk, const double* __restrict__ a_stage, double t_s, double cK,
    double cY) {
  __shared__ double red[16 * 7];
  double S[7];
  sum_partials<7>(partials, nblk, S, red);
  if (threadIdx.x != 0) return;
  const double vr = A->lk_re, vi = A->lk_im;
  // Re f = -kappa ar + wc ai ; Im f = -wc ar - kappa ai + (V/hbar) F - eps
  double yr = -P.kappa * vr - P.wc * vi + 2.0 * S[0];  // B_cav = Brms 2 Re a
  double yi = P.wc * vr - P.kappa * vi;
  const double lamF = P.vc_hbar * vi;
  const double two_ar = 2.0 * a_stage[0];
  A->g_brms[0] += two_ar * S[1] + lamF * S[4];
  A->g_brms[1] += two_ar * S[2] + lamF * S[5];
  A->g_brms[2] += two_ar * S[3] + lamF * S[6];
  A->g_eps0 += -vi * drive_shape(P.ckind, P.cw, t_s);
  A->acc_re += yr;
  A->acc_im += yi;
  if (cY != 0.0) {
    A->lk_re = cK * A->hat_re + cY * yr;
    A->lk_im = cK * A->hat_im + cY * yi;
  }
}

// End of the step's reverse sweep: lam <- acc (cavity part).
__global__ void k_adj_end_scalar(AdjCtl* __restrict__ A) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  A->lam_re = A->acc_re;
  A->lam_im = A->acc_im;
}

}  // namespace llgc
