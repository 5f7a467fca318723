// Batched engine kernels: one launch per kernel type and stage advances
// every active instance of a batch.  Each workgroup reads a work item
// (instance, tile) and runs the same device body as the single-instance
// kernel of that tile, on that instance's buffers, parameters, control
// block and Runge-Kutta epilogue, so a batched instance performs exactly the
// arithmetic of a context created with the batch plan.
#pragma once
#include "llgc_common.hpp"

namespace llgc {

constexpr int kBXT = 384;   // x pass / field: 6 wavefronts (4-row tiles)
constexpr int kBYT = 768;   // spectral pass: 12 wavefronts
constexpr int kBPT = 256;   // pointwise (k_begin) threads

// Device-resident description of one instance.
struct BInst {
  Prm P;
  Ctl* ctl;
  const float2* tw;
  int logTw;
  int nrx, nry;         // Px / 64, Py / 64 (1, 2 or 4)
  int Ww;               // kx columns per spectral workgroup
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
  const float* ys = B.ys[stage];
  switch (B.nrx) {
    case 1: xfwd_w_body<1>(B.P, ys, B.spec, B.partials, 4, B.tw, B.logTw, w.y, w.y, zl); break;
    case 2: xfwd_w_body<2>(B.P, ys, B.spec, B.partials, 4, B.tw, B.logTw, w.y, w.y, zl); break;
    default: xfwd_w_body<4>(B.P, ys, B.spec, B.partials, 4, B.tw, B.logTw, w.y, w.y, zl); break;
  }
}

template <int NZ>
__device__ __forceinline__ void kb_yspec_nz(const BInst& B, int stage,
                                            int mode, int blk, float2* lds) {
#define LLGC_BY_ARGS B.P, B.spec, B.K, B.ctl, B.Ww, B.tw, B.logTw, \
                     B.partials, B.nf, stage, mode, blk, lds
  switch (B.nry) {
    case 1: yspec_w_body<NZ, 1>(LLGC_BY_ARGS); break;
    case 2: yspec_w_body<NZ, 2>(LLGC_BY_ARGS); break;
    default: yspec_w_body<NZ, 4>(LLGC_BY_ARGS); break;
  }
#undef LLGC_BY_ARGS
}

__global__ __launch_bounds__(kBYT) void kb_yspec(const BInst* __restrict__ I,
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
  switch (B.P.nz) {
    case 1: kb_yspec_nz<1>(B, stage, mode, w.y, lds); break;
    case 2: kb_yspec_nz<2>(B, stage, mode, w.y, lds); break;
    case 3: kb_yspec_nz<3>(B, stage, mode, w.y, lds); break;
    default: kb_yspec_nz<4>(B, stage, mode, w.y, lds); break;
  }
}

__global__ __launch_bounds__(kBXT) void kb_xfield(const BInst* __restrict__ I,
                                                  const int2* __restrict__ it,
                                                  int stage) {
  extern __shared__ float bdl[];
  const int2 w = bitem(it);
  const BInst& B = I[w.x];
  if (B.ctl->done) return;
  const float* ys = B.ys[stage];
  const Epi& E = B.E[stage];
  switch (B.nrx) {
    case 1: xfield_w_body<1>(B.P, ys, B.spec, B.ctl, B.partials, stage, 4, E, B.tw, B.logTw, w.y, w.y, bdl); break;
    case 2: xfield_w_body<2>(B.P, ys, B.spec, B.ctl, B.partials, stage, 4, E, B.tw, B.logTw, w.y, w.y, bdl); break;
    default: xfield_w_body<4>(B.P, ys, B.spec, B.ctl, B.partials, stage, 4, E, B.tw, B.logTw, w.y, w.y, bdl); break;
  }
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
