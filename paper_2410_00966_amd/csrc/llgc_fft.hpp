// Batched in-LDS complex FFT for power-of-two lengths (gfx950).
//
// Stockham auto-sort, radix 16/8/4/2, in place in one LDS buffer: each pass
// loads a thread's butterflies into registers, barriers, computes and
// stores to the auto-sorted positions, barriers.  All threads of the
// workgroup cooperate on a batch of `batch` transforms of length L stored
// contiguously (transform t at logical s + t*L, stored at pidx()).  Twiddles come from a table of
// exp(-2 pi i m / Ltw) for m < Ltw (Ltw a power of two >= L).
#pragma once
#include <hip/hip_runtime.h>

namespace llgc {

// LDS index with 2 padding slots every 16 complex values: spreads the
// strided Stockham stores over the banks and keeps even indices 16-byte
// aligned (pairs 2i, 2i+1 never straddle a gap).
__host__ __device__ __forceinline__ int pidx(int i) { return i + ((i >> 4) << 1); }
// The same with 2 slots every 2^PS values (PS = 4 is pidx): less LDS for
// kernels whose occupancy is bound by it, at more bank conflicts.
template <int PS>
__host__ __device__ __forceinline__ int pidx_s(int i) {
  return i + ((i >> PS) << 1);
}
template <int PS>
__host__ __device__ __forceinline__ size_t padded_len_s(size_t n) {
  return n + ((n >> PS) << 1) + 2;
}
__host__ __device__ __forceinline__ size_t padded_len(size_t n) {
  return n + ((n >> 4) << 1) + 2;
}

__device__ __forceinline__ float2 cadd(float2 a, float2 b) {
  return make_float2(a.x + b.x, a.y + b.y);
}
__device__ __forceinline__ float2 csub(float2 a, float2 b) {
  return make_float2(a.x - b.x, a.y - b.y);
}
// Complex product with its two fused multiply-adds written out, so that
// every kernel the transforms are inlined into rounds them alike (left to
// the compiler, which product of a.x b.x - a.y b.y is fused can differ from
// one kernel to another).
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -(a.y * b.y)), fmaf(a.x, b.y, a.y * b.x));
}
// multiply by s*i with s = +-1
__device__ __forceinline__ float2 cmul_si(float2 a, float s) {
  return make_float2(-s * a.y, s * a.x);
}
// multiply by (c h, s h), h = 1/sqrt(2), c, s = +-1 (the odd eighth roots of
// unity): two additions and two products instead of a general product
__device__ __forceinline__ float2 cmul_h(float2 a, float c, float s) {
  const float h = 0.70710678118654752f;
  return make_float2((c * a.x - s * a.y) * h, (c * a.y + s * a.x) * h);
}

template <int R>
struct RadixTag {
  static constexpr int value = R;
};
template <int R>
struct Log2C {
  static constexpr int v = R == 2 ? 1 : R == 4 ? 2 : R == 8 ? 3 : 4;
};

// R-point DFT in registers: X_p = sum_q v_q exp(s 2 pi i p q / R),
// s = -1 forward, +1 inverse.
template <int R>
__device__ __forceinline__ void dft_small(float2* v, float s);

template <>
__device__ __forceinline__ void dft_small<2>(float2* v, float) {
  float2 a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}

template <>
__device__ __forceinline__ void dft_small<4>(float2* v, float s) {
  float2 t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
  float2 t2 = cadd(v[1], v[3]), t3 = cmul_si(csub(v[1], v[3]), s);
  v[0] = cadd(t0, t2);
  v[2] = csub(t0, t2);
  v[1] = cadd(t1, t3);
  v[3] = csub(t1, t3);
}

template <>
__device__ __forceinline__ void dft_small<8>(float2* v, float s) {
  float2 e[4] = {v[0], v[2], v[4], v[6]};
  float2 o[4] = {v[1], v[3], v[5], v[7]};
  dft_small<4>(e, s);
  dft_small<4>(o, s);
  // w8^p = exp(s i pi p / 4): (h, s h), s i, (-h, s h)
  float2 o1 = cmul_h(o[1], 1.f, s), o2 = cmul_si(o[2], s),
         o3 = cmul_h(o[3], -1.f, s);
  v[0] = cadd(e[0], o[0]);
  v[4] = csub(e[0], o[0]);
  v[1] = cadd(e[1], o1);
  v[5] = csub(e[1], o1);
  v[2] = cadd(e[2], o2);
  v[6] = csub(e[2], o2);
  v[3] = cadd(e[3], o3);
  v[7] = csub(e[3], o3);
}

template <>
__device__ __forceinline__ void dft_small<16>(float2* v, float s) {
  float2 e[8] = {v[0], v[2], v[4], v[6], v[8], v[10], v[12], v[14]};
  float2 o[8] = {v[1], v[3], v[5], v[7], v[9], v[11], v[13], v[15]};
  dft_small<8>(e, s);
  dft_small<8>(o, s);
  // w16^p = exp(s i pi p / 8)
  const float c1 = 0.92387953251128676f, s1 = 0.38268343236508977f;
  const float h = 0.70710678118654752f;
  const float2 w[8] = {make_float2(1.f, 0.f),   make_float2(c1, s * s1),
                       make_float2(h, s * h),    make_float2(s1, s * c1),
                       make_float2(0.f, s),      make_float2(-s1, s * c1),
                       make_float2(-h, s * h),   make_float2(-c1, s * s1)};
#pragma unroll
  for (int p = 0; p < 8; ++p) {
    // p = 2, 4, 6 are eighth roots of unity: cheaper products
    const float2 t = (p == 0)   ? o[0]
                     : (p == 4) ? cmul_si(o[4], s)
                     : (p == 2) ? cmul_h(o[2], 1.f, s)
                     : (p == 6) ? cmul_h(o[6], -1.f, s)
                                : cmul(o[p], w[p]);
    v[p] = cadd(e[p], t);
    v[p + 8] = csub(e[p], t);
  }
}

// R-point DFT whose inputs v[R/2..R-1] are zero (not read): the even
// outputs are the R/2-point DFT of v[0..R/2-1], the odd ones that of
// v[q] w_R^q.  Outputs in v[0..R-1].
template <int R>
__device__ __forceinline__ void dft_in_half(float2* v, float s) {
  if constexpr (R == 2) {
    v[1] = v[0];
  } else {
    constexpr int H = R / 2;
    float2 e[H], o[H];
#pragma unroll
    for (int q = 0; q < H; ++q) e[q] = v[q];
    // w_R^q = exp(s i 2 pi q / R), q < R/2
    const float c1 = 0.92387953251128676f, s1 = 0.38268343236508977f;
    const float h = 0.70710678118654752f;
    o[0] = v[0];
    if constexpr (R == 4) {
      o[1] = cmul_si(v[1], s);
    } else if constexpr (R == 8) {
      o[1] = cmul_h(v[1], 1.f, s);
      o[2] = cmul_si(v[2], s);
      o[3] = cmul_h(v[3], -1.f, s);
    } else {
      static_assert(R == 16, "radix 2, 4, 8 or 16");
      const float2 w[8] = {make_float2(1.f, 0.f),  make_float2(c1, s * s1),
                           make_float2(h, s * h),   make_float2(s1, s * c1),
                           make_float2(0.f, s),     make_float2(-s1, s * c1),
                           make_float2(-h, s * h),  make_float2(-c1, s * s1)};
#pragma unroll
      for (int q = 1; q < H; ++q)
        o[q] = (q == 4)   ? cmul_si(v[4], s)
               : (q == 2) ? cmul_h(v[2], 1.f, s)
               : (q == 6) ? cmul_h(v[6], -1.f, s)
                          : cmul(v[q], w[q]);
    }
    dft_small<H>(e, s);
    dft_small<H>(o, s);
#pragma unroll
    for (int m = 0; m < H; ++m) {
      v[2 * m] = e[m];
      v[2 * m + 1] = o[m];
    }
  }
}

// One Stockham pass of radix R over `batch` transforms of length L = 2^logL
// held in LDS.  Ns = 2^logNs is the length of the sub-transforms already
// done.  NB is the number of butterflies a thread holds in registers; the
// caller guarantees batch * L / R <= NB * blockDim.x.
// PIN (first pass only, Ns = 1): inputs at positions >= L/2 are zero and
// are not read.  POUT (last pass only, Ns = L/R): outputs at positions
// >= L/2 are not needed and are not written.
// TT: `tw` is this pass's twiddle table, tw[(q-1) Ns + k] = exp(-2 pi i k q
// / (Ns R)) (q = 1..R-1), read per power instead of forming the powers of
// the base twiddle by repeated products (fewer VALU operations).
template <int R, int NB, bool PIN = false, bool POUT = false, int PS = 4,
          bool TT = false>
__device__ __forceinline__ void fft_pass(float2* s, int logL, int logNs,
                                         int batch, const float2* tw,
                                         int logTw, float dir, int tid) {
  constexpr int logR = (R == 2) ? 1 : (R == 4) ? 2 : (R == 8) ? 3 : 4;
  const int logLr = logL - logR;
  const int Lr = 1 << logLr;
  const int nbf = batch << logLr;
  const int Ns = 1 << logNs;
  const int twshift = logTw - logNs - logR;   // k * Ltw / (Ns R)
  const int twmask = (1 << logTw) - 1;
  float2 v[NB][R];
  float2 w1[NB];
  // Loads of the butterfly inputs and of its base twiddle w = exp(-/+ i 2 pi
  // k / (Ns R)) are issued before the barrier so their latency overlaps;
  // the powers w^q are formed in registers afterwards.
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int b = tid + i * blockDim.x;
    w1[i] = make_float2(1.f, 0.f);
    if (b < nbf) {
      const int t = b >> logLr, j = b & (Lr - 1);
      const int base = t << logL;
#pragma unroll
      for (int q = 0; q < (PIN ? R / 2 : R); ++q)
        v[i][q] = s[pidx_s<PS>(base + j + q * Lr)];
      const int k = j & (Ns - 1);
      if (!TT && logNs > 0) w1[i] = tw[(k << twshift) & twmask];
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int b = tid + i * blockDim.x;
    if (b < nbf) {
      const int t = b >> logLr, j = b & (Lr - 1);
      const int k = j & (Ns - 1);
      // Twiddles in every pass after the first (Ns > 1; a uniform branch).
      // Lanes with k = 0 multiply by exactly 1 + 0i: no per-lane branch,
      // whose merge would cost a register move per value.
      if (TT && logNs > 0) {
#pragma unroll
        for (int q = 1; q < R; ++q) {
          float2 wq = tw[(q - 1) * Ns + k];
          wq.y *= -dir;   // table holds exp(-i ...); inverse conjugates
          v[i][q] = cmul(v[i][q], wq);
        }
      } else if (!TT && logNs > 0) {
        float2 w = w1[i];
        w.y *= -dir;   // table holds exp(-i ...); inverse conjugates
        float2 wq = w;
#pragma unroll
        for (int q = 1; q < R; ++q) {
          v[i][q] = cmul(v[i][q], wq);
          if (q + 1 < R) wq = cmul(wq, w);
        }
      }
      if constexpr (PIN) dft_in_half<R>(v[i], dir);
      else dft_small<R>(v[i], dir);
      const int out0 = (t << logL) + ((j - k) << logR) + k;
#pragma unroll
      for (int q = 0; q < (POUT ? R / 2 : R); ++q)
        s[pidx_s<PS>(out0 + q * Ns)] = v[i][q];
    }
  }
  __syncthreads();
}

// Full transform: dir = -1 forward (exp(-i...)), +1 inverse (unnormalised).
// VPT = complex values a thread may hold (register budget per pass); R16
// allows radix-16 passes (fewer LDS round trips, more registers).
// LOGL > 0 fixes the length at compile time (logL must then equal it): the
// pass loops unroll and every stride and padded LDS offset becomes an
// immediate, which removes most of the per-element address arithmetic.
// PIN: the input is zero from position L/2 on (zero padding; the first
// pass does not read it).  POUT: only outputs below L/2 are used (the last
// pass does not write the rest).
// Radix plan of a length-2^logL transform: 16s (R16 and a thread may hold
// 16 values), then the remainder as one 8, one 4, two 4s, 8 + 4 in place of
// one 16, or one 2; passes run in that order.
struct FftPlan {
  int n16, n8, n4, n2;
};
__host__ __device__ constexpr FftPlan fft_plan(int VPT, bool R16, int logL) {
  int n16 = (R16 && VPT >= 16) ? logL / 4 : 0;
  const int rem = logL - 4 * n16;
  int n8 = rem / 3, n4 = 0, n2 = 0;
  const int tail = rem % 3;
  if (tail == 2) n4 = 1;
  if (tail == 1) {
    if (n8 > 0) { n8 -= 1; n4 = 2; }
    else if (n16 > 0) { n16 -= 1; n8 = 1; n4 = 1; }
    else { n2 = 1; }
  }
  return FftPlan{n16, n8, n4, n2};
}

// Entries of the per-pass twiddle tables of that plan: (R-1) Ns for every
// pass after the first.
__host__ __device__ constexpr int fft_tt_len(int VPT, bool R16, int logL) {
  const FftPlan pl = fft_plan(VPT, R16, logL);
  int logNs = 0, n = 0;
  auto add = [&](int logR, int count) {
    for (int q = 0; q < count; ++q) {
      if (logNs > 0) n += ((1 << logR) - 1) << logNs;
      logNs += logR;
    }
  };
  add(4, pl.n16);
  add(3, pl.n8);
  add(2, pl.n4);
  add(1, pl.n2);
  return n;
}

// Fills the per-pass twiddle tables (fft_tt_len entries at `tt`) from the
// table tw[m] = exp(-2 pi i m / 2^logTw) in global memory; the caller
// synchronises before the first transform.
template <int VPT, bool R16, int LOGL>
__device__ __forceinline__ void fft_tt_build(float2* tt,
                                             const float2* __restrict__ tw,
                                             int logTw) {
  constexpr FftPlan pl = fft_plan(VPT, R16, LOGL);
  int logNs = 0, off = 0;
  const int mask = (1 << logTw) - 1;
  auto fill = [&](int logR, int count) {
    for (int c = 0; c < count; ++c) {
      if (logNs > 0) {
        const int Ns = 1 << logNs, n = ((1 << logR) - 1) << logNs;
        const int sh = logTw - logNs - logR;
        for (int e = threadIdx.x; e < n; e += blockDim.x) {
          const int q = 1 + (e >> logNs), k = e & (Ns - 1);
          tt[off + e] = tw[((k * q) << sh) & mask];
        }
        off += n;
      }
      logNs += logR;
    }
  };
  fill(4, pl.n16);
  fill(3, pl.n8);
  fill(2, pl.n4);
  fill(1, pl.n2);
}

// TT (with LOGL > 0): `tw` holds the per-pass twiddle tables of
// fft_tt_build instead of the plain table.  `tid`: the thread's index in
// the workgroup (threadIdx.x if negative); a caller that loops over blocks
// passes it through an opaque copy, so that the passes' address arithmetic
// is formed where it is used rather than held across the loop.
template <int VPT, bool R16 = false, int LOGL = 0, bool PIN = false,
          bool POUT = false, int PS = 4, bool TT = false>
__device__ __forceinline__ void fft_lds(float2* s, int logL, int batch,
                                        const float2* tw,
                        int logTw, float dir, int tid = -1) {
  if (tid < 0) tid = threadIdx.x;
  static_assert(!TT || LOGL > 0, "twiddle tables need a fixed length");
  if constexpr (LOGL > 0) logL = LOGL;
  if (logL == 0) return;
  int logNs = 0;
  const FftPlan pl = fft_plan(VPT, R16, logL);
  const int n16 = pl.n16, n8 = pl.n8, n4 = pl.n4, n2 = pl.n2;
  const int npass = n16 + n8 + n4 + n2;
  int p = 0;
  int toff = 0;   // this pass's table offset (TT)
  // pass p of radix R; the first honours PIN, the last POUT
  auto pass = [&](auto rtag) {
    constexpr int R = decltype(rtag)::value;
    constexpr int NB = VPT / R;
    const bool first = p == 0, last = p == npass - 1;
    const float2* twp = TT ? tw + toff : tw;
    if (PIN && first && POUT && last)
      fft_pass<R, NB, PIN, POUT, PS, TT>(s, logL, logNs, batch, twp, logTw,
                                         dir, tid);
    else if (PIN && first)
      fft_pass<R, NB, PIN, false, PS, TT>(s, logL, logNs, batch, twp, logTw,
                                          dir, tid);
    else if (POUT && last)
      fft_pass<R, NB, false, POUT, PS, TT>(s, logL, logNs, batch, twp,
                                           logTw, dir, tid);
    else
      fft_pass<R, NB, false, false, PS, TT>(s, logL, logNs, batch, twp,
                                            logTw, dir, tid);
    if (logNs > 0) toff += (R - 1) << logNs;
    logNs += Log2C<R>::v;
    ++p;
  };
  if constexpr (R16 && VPT >= 16) {
#pragma unroll
    for (int q = 0; q < n16; ++q) pass(RadixTag<16>{});
  }
#pragma unroll
  for (int q = 0; q < n8; ++q) pass(RadixTag<8>{});
#pragma unroll
  for (int q = 0; q < n4; ++q) pass(RadixTag<4>{});
#pragma unroll
  for (int q = 0; q < n2; ++q) pass(RadixTag<2>{});
}

}  // namespace llgc
