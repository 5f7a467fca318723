// Register-resident complex FFT: one transform of length L = 64 * NR per
// wavefront (gfx950, 64 lanes), NR a power of two <= 32.
//
// Layout: lane l, register r holds element n = l + 64 r.
// Forward: radix-2 decimation in frequency over the registers (an NR-point
// DFT on r with compile-time twiddles), the inter-step twiddle
// exp(-2 pi i l k1 / L), then radix-2 decimation in frequency across the
// lanes (a 64-point DFT on l, partners exchanged with lane shuffles).  The
// result X[k] sits at lane l, register r with
//     k = bitrev_NR(r) + NR * bitrev_64(l).
// Inverse: the mirror image (decimation in time across lanes, conjugate
// twiddle, decimation in time over registers), taking that layout back to
// natural order; unnormalised.  No LDS is used.
#pragma once
#include <hip/hip_runtime.h>

namespace llgc {

// exp(-2 pi i m / 32), m < 16
__constant__ float2 c_w32[16] = {
    {1.000000000e+00f, -0.000000000e+00f},
    {9.807852804e-01f, -1.950903220e-01f},
    {9.238795325e-01f, -3.826834324e-01f},
    {8.314696123e-01f, -5.555702330e-01f},
    {7.071067812e-01f, -7.071067812e-01f},
    {5.555702330e-01f, -8.314696123e-01f},
    {3.826834324e-01f, -9.238795325e-01f},
    {1.950903220e-01f, -9.807852804e-01f},
    {0.000000000e+00f, -1.000000000e+00f},
    {-1.950903220e-01f, -9.807852804e-01f},
    {-3.826834324e-01f, -9.238795325e-01f},
    {-5.555702330e-01f, -8.314696123e-01f},
    {-7.071067812e-01f, -7.071067812e-01f},
    {-8.314696123e-01f, -5.555702330e-01f},
    {-9.238795325e-01f, -3.826834324e-01f},
    {-9.807852804e-01f, -1.950903220e-01f}};

__device__ __forceinline__ float2 wmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 wmulc(float2 a, float2 b) {  // a * conj(b)
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}

template <int N>
struct Log2 {
  static constexpr int v = 1 + Log2<N / 2>::v;
};
template <>
struct Log2<1> {
  static constexpr int v = 0;
};

__device__ __forceinline__ int brev_bits(int x, int nb) {
  return nb == 0 ? 0 : (int)(__builtin_bitreverse32((unsigned)x) >> (32 - nb));
}

__device__ __forceinline__ float2 shfl_xor2(float2 v, int m) {
  return make_float2(__shfl_xor(v.x, m, 64), __shfl_xor(v.y, m, 64));
}

// tw: table of exp(-2 pi i m / Ltw), m < Ltw (Ltw = 2^logTw >= L).
template <int NR>
__device__ __forceinline__ void wfft_fwd(float2 (&v)[NR], int lane,
                                         const float2* __restrict__ tw,
                                         int logTw) {
  constexpr int LNR = Log2<NR>::v;
  const int logL = 6 + LNR;
  const int sh = logTw - logL;               // table stride for length L
  const int tmask = (1 << logTw) - 1;
  // step A: DIF over registers (linear stage counter so the loops unroll)
#pragma unroll
  for (int st = 0; st < LNR; ++st) {
    const int h = NR >> (st + 1);
#pragma unroll
    for (int r0 = 0; r0 < NR; r0 += 2 * h) {
#pragma unroll
      for (int i = 0; i < h; ++i) {
        const float2 u = v[r0 + i], w = v[r0 + i + h];
        v[r0 + i] = make_float2(u.x + w.x, u.y + w.y);
        const float2 d = make_float2(u.x - w.x, u.y - w.y);
        v[r0 + i + h] = (i == 0) ? d : wmul(d, c_w32[i * (16 / h)]);
      }
    }
  }
  // step B: exp(-2 pi i l k1 / L), k1 = bitrev(r); twiddles fetched in
  // groups of 8 to bound register use
#pragma unroll
  for (int r0 = 0; r0 < NR; r0 += 8) {
    constexpr int GB = NR < 8 ? NR : 8;
    float2 t[GB];
#pragma unroll
    for (int q = 0; q < GB; ++q) {
      const int k1 = brev_bits(r0 + q, LNR);
      t[q] = tw[((lane * k1) << sh) & tmask];
    }
#pragma unroll
    for (int q = 0; q < GB; ++q) v[r0 + q] = wmul(v[r0 + q], t[q]);
  }
  // step C: DIF across lanes
#pragma unroll
  for (int st = 0; st < 6; ++st) {
    const int h = 32 >> st;
    const bool up = (lane & h) != 0;
    // exp(-2 pi i (l mod h) / (2h))
    const float2 tl = tw[((lane & (h - 1)) << (logTw - 1)) / h];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const float2 p = shfl_xor2(v[r], h);
      if (up) {
        v[r] = wmul(make_float2(p.x - v[r].x, p.y - v[r].y), tl);
      } else {
        v[r] = make_float2(v[r].x + p.x, v[r].y + p.y);
      }
    }
  }
}

template <int NR>
__device__ __forceinline__ void wfft_inv(float2 (&v)[NR], int lane,
                                         const float2* __restrict__ tw,
                                         int logTw) {
  constexpr int LNR = Log2<NR>::v;
  const int logL = 6 + LNR;
  const int sh = logTw - logL;
  const int tmask = (1 << logTw) - 1;
  // inverse of step C: DIT across lanes, bit-reversed in, natural out
#pragma unroll
  for (int st = 0; st < 6; ++st) {
    const int h = 1 << st;
    const bool up = (lane & h) != 0;
    const float2 tl = tw[((lane & (h - 1)) << (logTw - 1)) / h];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const float2 p = shfl_xor2(v[r], h);
      if (up) {
        const float2 q = wmulc(v[r], tl);
        v[r] = make_float2(p.x - q.x, p.y - q.y);
      } else {
        const float2 q = wmulc(p, tl);
        v[r] = make_float2(v[r].x + q.x, v[r].y + q.y);
      }
    }
  }
  // inverse of step B
#pragma unroll
  for (int r0 = 0; r0 < NR; r0 += 8) {
    constexpr int GB = NR < 8 ? NR : 8;
    float2 t[GB];
#pragma unroll
    for (int q = 0; q < GB; ++q) {
      const int k1 = brev_bits(r0 + q, LNR);
      t[q] = tw[((lane * k1) << sh) & tmask];
    }
#pragma unroll
    for (int q = 0; q < GB; ++q) v[r0 + q] = wmulc(v[r0 + q], t[q]);
  }
  // inverse of step A: DIT over registers
#pragma unroll
  for (int st = 0; st < LNR; ++st) {
    const int h = 1 << st;
#pragma unroll
    for (int r0 = 0; r0 < NR; r0 += 2 * h) {
#pragma unroll
      for (int i = 0; i < h; ++i) {
        const float2 u = v[r0 + i];
        const float2 w = (i == 0) ? v[r0 + i + h]
                                  : wmulc(v[r0 + i + h], c_w32[i * (16 / h)]);
        v[r0 + i] = make_float2(u.x + w.x, u.y + w.y);
        v[r0 + i + h] = make_float2(u.x - w.x, u.y - w.y);
      }
    }
  }
}

}  // namespace llgc
