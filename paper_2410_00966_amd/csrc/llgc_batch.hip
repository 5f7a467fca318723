// Batched engine kernels: one launch per kernel type and stage advances
// every active instance of a batch.  Each workgroup reads a work item
// (instance, tile) and runs the same device body as the single-instance
// kernel of that tile, on that instance's buffers, parameters, control
// block and Runge-Kutta epilogue, so a batched instance performs exactly the
// arithmetic of a context created with the batch plan.
#pragma once
#include "llgc_common.hpp"

namespace llgc {

constexpr int kBXT = 512;   // x pass / field: LDS FFT of 3 (R/2) rows
constexpr int kBYT = 512;   // spectral pass: 8 wavefronts (LDS FFT)
constexpr int kBPT = 256;   // pointwise (k_begin) threads

// Device-resident description of one instance.
struct BInst {
  Prm P;
  Ctl* ctl;
  const float2* tw;
  int logTw;
  int R;                // rows per x-pass / field tile
  int W;                // column slots per spectral workgroup
  int nf;               // x-pass / field tiles
  int nbeg;             // k_begin workgroups
  float *yn, *k1, *y7, *k7, *y2;   // operands of the attempt start
  float2* spec;
  const float* K;
  double* partials;
  double* rec;
  const float* ys[kMaxStages];     // stage inputs
  Epi E[kMaxStages];               // stage epilogues
};

// Work items: .x = instance, .y = tile (or workgroup) within the instance;
// consecutive items run on one XCD.
__device__ __forceinline__ int2 bitem(const int2* __restrict__ it) {
  return it[xcd_tile(blockIdx.x, gridDim.x)];
}

__global__ __launch_bounds__(kBXT) void kb_xfwd(const BInst* __restrict__ I,
                                                const int2* __restrict__ it,
                                                int stage) {
  extern __shared__ float2 zl[];
  const int2 w = bitem(it);
  const BInst& B = I[w.x];
  if (B.ctl->done) return;
  xfwd3_body<kBXT>(B.P, B.ys[stage], B.spec, B.partials, B.R, B.tw, B.logTw,
                   w.y, w.y, zl);
}

__global__ __launch_bounds__(kBYT, 4) void kb_yspec(const BInst* __restrict__ I,
                                                 const int2* __restrict__ it,
                                                 int stage, int mode) {
  extern __shared__ float2 lds[];
  __shared__ double red[16];
  const int2 w = bitem(it);
  const BInst& B = I[w.x];
  if (B.ctl->done) return;
  if (!B.P.demag) {
    // no spectral pass: only the cavity stage (one item per instance)
    finish_cavity(B.P, B.ctl, B.partials, B.nf, stage, mode, red);
    return;
  }
#define LLGC_BY_ARGS B.P, B.spec, B.K, B.ctl, B.W, B.tw, B.logTw, \
                     B.partials, B.nf, stage, mode, w.y, w.y + 1, 1, lds
  switch (B.P.nz) {
    case 1: yspec_l_body<kBYT, 1, 0>(LLGC_BY_ARGS); break;
    case 2: yspec_l_body<kBYT, 2, 0>(LLGC_BY_ARGS); break;
    case 3: yspec_l_body<kBYT, 3, 0>(LLGC_BY_ARGS); break;
    default: yspec_l_body<kBYT, 4, 0>(LLGC_BY_ARGS); break;
  }
#undef LLGC_BY_ARGS
}

__global__ __launch_bounds__(kBXT) void kb_xfield(const BInst* __restrict__ I,
                                                  const int2* __restrict__ it,
                                                  int stage) {
  extern __shared__ float2 lds[];
  const int2 w = bitem(it);
  const BInst& B = I[w.x];
  if (B.ctl->done) return;
  xfield_l_body<kBXT, 0>(B.P, B.ys[stage], B.spec, B.ctl, B.partials, stage,
                         B.R, B.E[stage], B.tw, B.logTw, w.y, w.y, lds);
}

// Coupling sums with a per-cell B_rms map, tile for tile after kb_xfwd
// (instances without a map return at once).
__global__ __launch_bounds__(256) void kb_coupling(const BInst* __restrict__ I,
                                                   const int2* __restrict__ it,
                                                   int stage) {
  const int2 w = bitem(it);
  const BInst& B = I[w.x];
  if (B.ctl->done || !B.P.brms_map) return;
  coupling_tile_body<256>(B.P, B.ys[stage], B.partials, B.R, w.y, w.y);
}

// One workgroup per active instance (`act` lists them).
__global__ __launch_bounds__(256) void kb_finish_step(
    const BInst* __restrict__ I, const int* __restrict__ act, int kind,
    int* __restrict__ ndone) {
  const BInst& B = I[act[blockIdx.x]];
  if (B.ctl->done) return;
  finish_step_body(B.P, B.ctl, B.partials, B.nf, kind, B.rec, ndone);
}

__global__ __launch_bounds__(kBPT) void kb_begin(const BInst* __restrict__ I,
                                                 const int2* __restrict__ it) {
  const int2 w = bitem(it);
  const BInst& B = I[w.x];
  begin_body<kBPT>(B.P, B.yn, B.k1, B.y7, B.k7, B.y2, B.ctl, B.partials,
                   B.rec, w.y, B.nbeg);
}

// done flag of every instance
__global__ void kb_done_flags(const BInst* __restrict__ I, int n,
                              int* __restrict__ out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) out[k] = I[k].ctl->done;
}

}  // namespace llgc
