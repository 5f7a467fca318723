// Host side of the llgc C ABI: context, FFT planning, demag-kernel setup,
// device-driven RK4 / Dormand-Prince run loops, per-kernel timing.
// Single translation unit: the device code is included below.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <string>
#include <vector>

#include "../../include/llgc.h"
#include "llgc_common.hpp"
#include "llgc_demag.hip"
#include "llgc_kernels.hip"
#include "llgc_adjoint.hip"
#include "llgc_batch.hip"

using namespace llgc;

namespace {

constexpr int kT = 256;               // pointwise / reduction threads
#ifndef LLGC_TX
#define LLGC_TX 512
#endif
#ifndef LLGC_TYMAX
#define LLGC_TYMAX 1024
#endif
constexpr int kTX = LLGC_TX;          // threads of the LDS x-pass kernels
constexpr int kTyMax = LLGC_TYMAX;    // largest LDS spectral workgroup
constexpr int kYhEpt = 12;            // split y pass: elements per thread
constexpr int kMaxLen = 2048;         // largest padded FFT length per axis
constexpr size_t kLdsCap = 120 * 1024; // LDS per workgroup this plan uses
constexpr int kBatchMaxLen = 256;     // batched plan: padded length per axis
constexpr int kBatchTy = kBYT;        // batched plan: spectral workgroup threads

struct TimerRec {
  double ms = 0.0;
  int64_t launches = 0;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
};

}  // namespace

struct llgc_ctx {
  // grid and plan
  int nx, ny, nz, N;
  double dx, dy, dz;
  int Px, Py, Hx, Hy, logPx, logPy, logTw;
  int Rf, Ri, W, Ty;
  int Ww = 1;            // kx columns per register-FFT spectral block
  bool use_wy = false;   // register (wavefront) FFT along y
  bool use_wxf = false;  // register (wavefront) FFT in the forward x pass
  bool use_wxi = false;  // register (wavefront) inverse FFT in the field pass
  bool x3 = false;       // LDS x passes over the 3 components of a tile at once
  bool batch_plan = false;  // fixed plan shared with the batched engine
  bool no_fuse = false;     // LLGC_NO_FUSE: separate forward x passes
  bool force_fuse = false;  // LLGC_FUSE: fused passes on any grid
  bool fused_run = false;   // launches of a chunk with fused passes
  bool yhalf = false;    // LDS spectral pass split by ky parity (k_yspec_h)
  bool no_ypersist = false;  // LLGC_NO_YPERSIST: one spectral block per workgroup
  // Dormand-Prince controller fused into the next attempt's start
  // (LLGC_NO_STEP_BEGIN: a separate one-workgroup k_finish_step)
  bool step_begin = true;
  bool ysplit = false;   // two-layer spectral pass with half the LDS (k_yspec_z)
  size_t lds_yz = 0;     // its dynamic LDS
  int ncu = 0;           // compute units of the device
  int Tyh = 512;         // its workgroup size
  size_t lds_yh = 0;     // its LDS bytes
  int Rw = 2;            // rows per tile of the wavefront field kernel
  int Rwf = 2;           // rows per tile of the wavefront forward x pass
  size_t lds_f, lds_i, lds_y;
  hipStream_t stream;
  int device = 0;        // HIP device current at creation
  // device buffers
  float *yn = nullptr, *yb[2] = {nullptr, nullptr}, *kb[7] = {};
  float2* spec = nullptr;
  float* K = nullptr;
  double* tensor = nullptr;
  float2* tw = nullptr;
  double* partials = nullptr;
  double* rec = nullptr;
  int64_t rec_dev_cap = 0;    // record buffer size in doubles
  Ctl* ctl = nullptr;
  Ctl* ctl_eval = nullptr;
  float *ms_map = nullptr, *ku_map = nullptr;
  float* brms_map = nullptr;   // 3 N floats
  float* fdrive_map = nullptr; // 3 N floats: field drive per cell
  // multimode cavity (llgc_set_modes): constants on the device, per-mode
  // maps, per-tile coupling partials; nmodes = 0 for the single mode
  int nmodes = 0;
  llgc_mode mode_h[kMaxModes] = {};
  Modes* modes_dev = nullptr;
  float* mode_maps = nullptr;   // nmodes * 3 N floats when any mode has one
  double* mpart = nullptr;      // kMaxModes doubles per x-pass tile
  bool masked = false;         // geometry: some cells have Ms = 0
  double nmag = 0.0;           // magnetic cells
  size_t npartials = 0;
  // host state
  llgc_params prm{};
  Prm P{};
  bool have_params = false, have_state = false, need_init = true;
  bool kernel_built = false;
  double kernel_mu0 = 0.0;
  std::string err;
  bool timing = false;
  std::string timing_only;            // time only this kernel ("" = all)
  std::vector<hipEvent_t> event_pool; // reusable timing events
  std::map<std::string, TimerRec> timers;
  // HIP graphs of the integrator's launch sequences (index 0: a chunk of
  // Dormand-Prince attempts, 1: one RK4 step), with the launch arguments
  // they were captured with
  bool graphs = true;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph[2] = {nullptr, nullptr};
  hipGraphExec_t graph_exec[2] = {nullptr, nullptr};
  std::vector<unsigned char> graph_sig[2];
};

namespace {

int fail(llgc_ctx* c, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  return code;
}

#define HIPCHK(ctx, call)                                                   \
  do {                                                                      \
    hipError_t e_ = (call);                                                 \
    if (e_ != hipSuccess)                                                   \
      return fail(ctx, LLGC_E_HIP, "%s failed: %s", #call,                  \
                  hipGetErrorString(e_));                                   \
  } while (0)

int pow2_ceil(int v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}

// Events around a launch when timing is on.
hipEvent_t pooled_event(llgc_ctx* c);

struct Timed {
  llgc_ctx* c;
  const char* name;
  bool on;
  hipEvent_t a = nullptr, b = nullptr;
  Timed(llgc_ctx* cc, const char* n)
      : c(cc), name(n),
        on(cc->timing && (cc->timing_only.empty() || cc->timing_only == n)) {
    if (on) {
      a = pooled_event(c);
      b = pooled_event(c);
      hipEventRecord(a, c->stream);
    }
  }
  ~Timed() {
    if (on) {
      hipEventRecord(b, c->stream);
      auto& t = c->timers[name];
      t.pending.emplace_back(a, b);
      t.launches += 1;
    }
  }
};

int check_launch(llgc_ctx* c, const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess)
    return fail(c, LLGC_E_HIP, "launch of %s failed: %s", what,
                hipGetErrorString(e));
  return LLGC_OK;
}

// 1D tile grid: ceil(ny/R) y-tiles for each of the nz layers
dim3 xgrid(const llgc_ctx* c, int R) {
  return dim3(((c->ny + R - 1) / R) * c->nz, 1, 1);
}

int n_pointwise_blocks(const llgc_ctx* c) {
  return std::max(1, std::min(2048, (c->N + kT - 1) / kT));
}

// ------------------------------------------------------------ stage launch
bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }

// Chunks of the integrator may fuse the forward x pass of stage s+1 into
// the field pass of stage s (k_xfield_fwd): LDS x passes on a transform
// length the kernels are specialised for, demag on, single-context plan.
// The fused passes use the field pass's tiling (Ri rows) for both.  Fusing
// pays where the grid leaves the GPU part-idle and launches dominate (the
// 512x32x4 wire: 0.256 -> 0.225 ms per DP45 step; the 256x256x2 film: RK4
// 9.1e8 -> 1.08e9 cell-steps/s); on a full GPU the separate passes are
// faster (1024x1024x2: 1.07 ms fused 1.21 ms), so only grids of at most
// 512 field tiles fuse (LLGC_FUSE forces it on, LLGC_NO_FUSE off).
bool fusable(const llgc_ctx* c) {
  if (!(c->P.demag && !c->use_wxf && !c->use_wxi && !c->x3 &&
        !c->batch_plan && !c->no_fuse && c->logPx >= 8 && c->logPx <= 11))
    return false;
  return c->force_fuse || xgrid(c, c->Ri).x <= 512;
}

// rows per tile of whichever forward x pass runs
int fwd_rows(const llgc_ctx* c) {
  if (c->fused_run) return c->Ri;
  return c->use_wxf ? c->Rwf : c->Rf;
}

int launch_xfwd(llgc_ctx* c, const float* ys, Ctl* ctl, int stage,
                int mode) {
  if (c->fused_run) {
    // the first stage of a fused chunk: the fused pass's forward body
    Timed tm(c, "k_xfwd_fx");
#define LLGC_XFX(LP)                                                        \
  hipLaunchKernelGGL((k_xfwd_fx<kTX, LP>), xgrid(c, c->Ri), dim3(kTX),       \
                     c->lds_i, c->stream, c->P, ys, c->spec, ctl,           \
                     c->partials, c->Ri, c->tw, c->logTw)
    switch (c->logPx) {
      case 8: LLGC_XFX(8); break;
      case 9: LLGC_XFX(9); break;
      case 10: LLGC_XFX(10); break;
      default: LLGC_XFX(11); break;
    }
#undef LLGC_XFX
    return check_launch(c, "k_xfwd_fx");
  }
  Timed tm(c, "k_xfwd");
  if (c->use_wxf) {
    const int R = c->Rwf;
    const size_t lds = c->P.demag ? sizeof(float2) * 3 * (R / 2) * c->Px : 0;
    dim3 g = xgrid(c, R), b(64 * 3 * (R / 2));
#define LLGC_FW_ARGS c->P, ys, c->spec, ctl, c->partials, stage, R, c->tw, \
                     c->logTw, mode
    switch (c->Px) {
      case 64: hipLaunchKernelGGL((k_xfwd_w<1>), g, b, lds, c->stream, LLGC_FW_ARGS); break;
      case 128: hipLaunchKernelGGL((k_xfwd_w<2>), g, b, lds, c->stream, LLGC_FW_ARGS); break;
      case 256: hipLaunchKernelGGL((k_xfwd_w<4>), g, b, lds, c->stream, LLGC_FW_ARGS); break;
      case 512: hipLaunchKernelGGL((k_xfwd_w<8>), g, b, lds, c->stream, LLGC_FW_ARGS); break;
      case 1024: hipLaunchKernelGGL((k_xfwd_w<16>), g, b, lds, c->stream, LLGC_FW_ARGS); break;
      default: hipLaunchKernelGGL((k_xfwd_w<32>), g, b, lds, c->stream, LLGC_FW_ARGS); break;
    }
#undef LLGC_FW_ARGS
    return check_launch(c, "k_xfwd_w");
  }
  if (c->batch_plan || c->x3) {
    hipLaunchKernelGGL((k_xfwd3<kTX>), xgrid(c, c->Rf), dim3(kTX),
                       c->P.demag ? c->lds_f : 0, c->stream, c->P, ys,
                       c->spec, ctl, c->partials, c->Rf, c->tw, c->logTw);
    return check_launch(c, "k_xfwd3");
  }
  const bool v4 = (c->nx % 4 == 0) && aligned16(ys) &&
                  (!c->ms_map || aligned16(c->ms_map));
  const size_t lds = c->P.demag ? c->lds_f : 0;
#define LLGC_XF(V, LP)                                                      \
  hipLaunchKernelGGL((k_xfwd<kTX, V, LP>), xgrid(c, c->Rf), dim3(kTX), lds,  \
                     c->stream, c->P, ys, c->spec, ctl, c->partials, stage, \
                     c->Rf, c->tw, c->logTw, mode)
  if (v4) {
    if (c->logPx == 11) LLGC_XF(true, 11);
    else if (c->logPx == 10) LLGC_XF(true, 10);
    else LLGC_XF(true, 0);
  } else {
    if (c->logPx == 11) LLGC_XF(false, 11);
    else if (c->logPx == 10) LLGC_XF(false, 10);
    else LLGC_XF(false, 0);
  }
#undef LLGC_XF
  return check_launch(c, "k_xfwd");
}

// The LDS FFT kernels are specialised on the transform length for the
// long transforms they serve (LP = log2 length; 0 = any length).
// Workgroups of `f` (T threads, `lds` bytes of dynamic LDS) resident on one
// CU at a time (cached per kernel and size).
int blocks_per_cu(const void* f, int T, size_t lds) {
  static std::map<std::pair<const void*, size_t>, int> cache;
  static std::mutex mu;
  std::lock_guard<std::mutex> lock(mu);
  auto key = std::make_pair(f, lds);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, T, lds) !=
      hipSuccess)
    nb = 0;
  (void)hipGetLastError();
  cache[key] = nb;
  return nb;
}

template <int T, int LP>
void yspec_nz_lp(llgc_ctx* c, Ctl* ctl, dim3 g, int stage, int mode) {
  const int nf = (int)xgrid(c, fwd_rows(c)).x;
  const int nblk = (int)g.x;
  // Fewer workgroups than blocks, each stepping through several and loading
  // the next block's input during the current block's inverse transform:
  // as many as are resident at once (the blocks' lower halves must fit the
  // kernel's prefetch registers).
  auto grid_for = [&](const void* f) {
    const int hp = c->Py >> 2;
    if (!yspec_steps(T, c->nz) || c->no_ypersist || c->ncu <= 0 ||
        c->Py < 4 || c->W * 3 * c->nz * hp > kPf * T)
      return g;
    const int per = blocks_per_cu(f, T, c->lds_y);
    if (per <= 0) return g;
    return dim3((unsigned)std::min(nblk, per * c->ncu));
  };
#define LLGC_YSPEC_ARGS c->P, c->spec, c->K, ctl, c->W, c->tw, c->logTw, \
                        c->partials, nf, stage, mode, nblk
#define LLGC_YS(NZ)                                                         \
  hipLaunchKernelGGL((k_yspec<T, NZ, LP>),                                  \
                     grid_for((const void*)k_yspec<T, NZ, LP>), dim3(T),    \
                     c->lds_y, c->stream, LLGC_YSPEC_ARGS)
  switch (c->nz) {
    case 1: LLGC_YS(1); break;
    case 2: LLGC_YS(2); break;
    case 3: LLGC_YS(3); break;
    default: LLGC_YS(4); break;
  }
#undef LLGC_YS
#undef LLGC_YSPEC_ARGS
}

template <int T>
void yspec_nz(llgc_ctx* c, Ctl* ctl, dim3 g, int stage, int mode) {
  switch (c->logPy) {
    case 10: yspec_nz_lp<T, 10>(c, ctl, g, stage, mode); break;
    case 11: yspec_nz_lp<T, 11>(c, ctl, g, stage, mode); break;
    default: yspec_nz_lp<T, 0>(c, ctl, g, stage, mode); break;
  }
}

// Dynamic-LDS limit of a kernel: process-wide, so it only ever grows (a
// later, smaller context must not shrink the limit an earlier one needs).
void raise_lds_limit(const void* f, size_t bytes) {
  static std::map<const void*, size_t> cur;
  static std::mutex mu;
  std::lock_guard<std::mutex> lock(mu);
  size_t& v = cur[f];
  if (bytes > v) {
    hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)bytes);
    v = bytes;
  }
}

template <int T, int LP>
void yspec_attr_lp(size_t lds) {
  raise_lds_limit((const void*)k_yspec<T, 1, LP>, lds);
  raise_lds_limit((const void*)k_yspec<T, 2, LP>, lds);
  raise_lds_limit((const void*)k_yspec<T, 3, LP>, lds);
  raise_lds_limit((const void*)k_yspec<T, 4, LP>, lds);
}

template <int T>
void yspec_attr(size_t lds) {
  yspec_attr_lp<T, 0>(lds);
  yspec_attr_lp<T, 10>(lds);
  yspec_attr_lp<T, 11>(lds);
}

// Spectral pass; its workgroup 0 also finishes the stage's coupling sum.
// Without demag a one-workgroup kernel finishes the sum instead.
template <int NZ>
void yspec_w_nr(llgc_ctx* c, Ctl* ctl, dim3 g, dim3 b, size_t lds, int stage,
                int mode) {
  const int nf = (int)xgrid(c, fwd_rows(c)).x;
#define LLGC_YW_ARGS c->P, c->spec, c->K, ctl, c->Ww, c->tw, c->logTw, \
                     c->partials, nf, stage, mode
  switch (c->Py) {
    case 64: hipLaunchKernelGGL((k_yspec_w<NZ, 1>), g, b, lds, c->stream, LLGC_YW_ARGS); break;
    case 128: hipLaunchKernelGGL((k_yspec_w<NZ, 2>), g, b, lds, c->stream, LLGC_YW_ARGS); break;
    case 256: hipLaunchKernelGGL((k_yspec_w<NZ, 4>), g, b, lds, c->stream, LLGC_YW_ARGS); break;
    case 512: hipLaunchKernelGGL((k_yspec_w<NZ, 8>), g, b, lds, c->stream, LLGC_YW_ARGS); break;
    case 1024: hipLaunchKernelGGL((k_yspec_w<NZ, 16>), g, b, lds, c->stream, LLGC_YW_ARGS); break;
    default: hipLaunchKernelGGL((k_yspec_w<NZ, 32>), g, b, lds, c->stream, LLGC_YW_ARGS); break;
  }
#undef LLGC_YW_ARGS
}

int launch_yspec(llgc_ctx* c, Ctl* ctl, int stage, int mode) {
  if (c->P.demag && c->use_wy) {
    Timed tm(c, "k_yspec");
    const int nz3 = 3 * c->nz;
    dim3 g((c->Hx + c->Ww - 1) / c->Ww), b(64 * c->Ww * nz3);
    const int G = std::min(c->Py / 64, 8);
    const size_t lds = sizeof(float2) * (size_t)c->Ww * nz3 * G * 64;
    switch (c->nz) {
      case 1: yspec_w_nr<1>(c, ctl, g, b, lds, stage, mode); break;
      case 2: yspec_w_nr<2>(c, ctl, g, b, lds, stage, mode); break;
      case 3: yspec_w_nr<3>(c, ctl, g, b, lds, stage, mode); break;
      default: yspec_w_nr<4>(c, ctl, g, b, lds, stage, mode); break;
    }
    return check_launch(c, "k_yspec_w");
  }
  if (!c->P.demag && c->P.modes) return LLGC_OK;   // k_finish_modes did it
  if (!c->P.demag) {
    Timed tm(c, "k_finish_stage");
    hipLaunchKernelGGL(k_finish_stage<kT>, dim3(1), dim3(kT), 0, c->stream,
                       c->P, ctl, c->partials, (int)xgrid(c, fwd_rows(c)).x,
                       stage, mode);
    return check_launch(c, "k_finish_stage");
  }
  Timed tm(c, "k_yspec");
  dim3 g((c->Hx + c->W - 1) / c->W);
  if (c->yhalf) {
    const int nf = (int)xgrid(c, fwd_rows(c)).x;
#define LLGC_YH_ARGS c->P, c->spec, c->K, ctl, c->W, c->tw, c->logTw, \
                     c->partials, nf, stage, mode
#define LLGC_YH(TT, EE)                                                      \
    switch (c->nz) {                                                        \
      case 1: hipLaunchKernelGGL((k_yspec_h<TT, 1, EE>), g, dim3(TT), c->lds_yh, c->stream, LLGC_YH_ARGS); break; \
      case 2: hipLaunchKernelGGL((k_yspec_h<TT, 2, EE>), g, dim3(TT), c->lds_yh, c->stream, LLGC_YH_ARGS); break; \
      default: hipLaunchKernelGGL((k_yspec_h<TT, 3, EE>), g, dim3(TT), c->lds_yh, c->stream, LLGC_YH_ARGS); break; \
    }
    if (c->nz == 4) {
      hipLaunchKernelGGL((k_yspec_h<1024, 4, kYhEpt>), g, dim3(1024),
                         c->lds_yh, c->stream, LLGC_YH_ARGS);
    } else if (c->Tyh == 1024) { LLGC_YH(1024, kYhEpt) }
    else { LLGC_YH(512, kYhEpt) }
#undef LLGC_YH
#undef LLGC_YH_ARGS
    return check_launch(c, "k_yspec_h");
  }
  // k_yspec pairs the real columns kx = 0 and Px/2 into one slot
  const int nslot = c->Px >= 2 ? c->Px / 2 : c->Hx;
  g = dim3((nslot + c->W - 1) / c->W);
  if (c->ysplit) {
    // one slot per workgroup
    const int nf = (int)xgrid(c, fwd_rows(c)).x;
    const dim3 gz((unsigned)nslot);
#define LLGC_YZ_ARGS c->P, c->spec, c->K, ctl, c->tw, c->logTw, c->partials, \
                     nf, stage, mode, nslot
    if (c->logPy == 11)
      hipLaunchKernelGGL(k_yspec_z<11>, gz, dim3(kYzT), c->lds_yz, c->stream,
                         LLGC_YZ_ARGS);
    else
      hipLaunchKernelGGL(k_yspec_z<10>, gz, dim3(kYzT), c->lds_yz, c->stream,
                         LLGC_YZ_ARGS);
#undef LLGC_YZ_ARGS
    return check_launch(c, "k_yspec_z");
  }
  if constexpr (kTyMax >= 1024) {
    if (c->Ty == 1024) yspec_nz<1024>(c, ctl, g, stage, mode);
  }
  if (c->Ty == 512) yspec_nz<512>(c, ctl, g, stage, mode);
  else if (c->Ty == 256) yspec_nz<256>(c, ctl, g, stage, mode);
  return check_launch(c, "k_yspec");
}

int launch_xfield(llgc_ctx* c, const float* ys, Ctl* ctl, int stage,
                  const Epi& E, bool fuse_fwd = false) {
  if (fuse_fwd) {
    // field pass of this stage + forward x pass of the next stage input
    Timed tm(c, "k_xfield_fwd");
#define LLGC_XFF(LP)                                                        \
  hipLaunchKernelGGL((k_xfield_fwd<kTX, LP>), xgrid(c, c->Ri), dim3(kTX),    \
                     c->lds_i, c->stream, c->P, ys, c->spec, ctl,           \
                     c->partials, c->rec, stage, c->Ri, E, c->tw, c->logTw)
    switch (c->logPx) {
      case 8: LLGC_XFF(8); break;
      case 9: LLGC_XFF(9); break;
      case 10: LLGC_XFF(10); break;
      default: LLGC_XFF(11); break;
    }
#undef LLGC_XFF
    return check_launch(c, "k_xfield_fwd");
  }
  Timed tm(c, "k_xfield");
  if (c->use_wxi) {
    const int R = c->Rw;
    const size_t lds = c->P.demag ? sizeof(float) * 3 * R * c->nx : 0;
    dim3 g = xgrid(c, R), b(64 * 3 * (R / 2));
#define LLGC_XW_ARGS c->P, ys, c->spec, ctl, c->partials, c->rec, stage, R, \
                     E, c->tw, c->logTw
    switch (c->Px) {
      case 64: hipLaunchKernelGGL((k_xfield_w<1>), g, b, lds, c->stream, LLGC_XW_ARGS); break;
      case 128: hipLaunchKernelGGL((k_xfield_w<2>), g, b, lds, c->stream, LLGC_XW_ARGS); break;
      case 256: hipLaunchKernelGGL((k_xfield_w<4>), g, b, lds, c->stream, LLGC_XW_ARGS); break;
      case 512: hipLaunchKernelGGL((k_xfield_w<8>), g, b, lds, c->stream, LLGC_XW_ARGS); break;
      case 1024: hipLaunchKernelGGL((k_xfield_w<16>), g, b, lds, c->stream, LLGC_XW_ARGS); break;
      default: hipLaunchKernelGGL((k_xfield_w<32>), g, b, lds, c->stream, LLGC_XW_ARGS); break;
    }
#undef LLGC_XW_ARGS
    return check_launch(c, "k_xfield_w");
  }
  if (c->batch_plan || c->x3) {
    hipLaunchKernelGGL((k_xfield_b<kTX>), xgrid(c, c->Ri), dim3(kTX),
                       c->P.demag ? c->lds_i : 0, c->stream, c->P, ys,
                       c->spec, ctl, c->partials, c->rec, stage, c->Ri, E,
                       c->tw, c->logTw);
    return check_launch(c, "k_xfield_b");
  }
#define LLGC_XI(LP)                                                         \
  hipLaunchKernelGGL((k_xfield<kTX, LP>), xgrid(c, c->Ri), dim3(kTX),        \
                     c->P.demag ? c->lds_i : 0, c->stream, c->P, ys,       \
                     c->spec, ctl, c->partials, c->rec, stage, c->Ri, E,   \
                     c->tw, c->logTw)
  switch (c->logPx) {
    case 8: LLGC_XI(8); break;
    case 9: LLGC_XI(9); break;
    case 10: LLGC_XI(10); break;
    case 11: LLGC_XI(11); break;
    default: LLGC_XI(0); break;
  }
#undef LLGC_XI
  return check_launch(c, "k_xfield");
}

// rows per tile of whichever field kernel runs
int field_rows(const llgc_ctx* c) { return c->use_wxi ? c->Rw : c->Ri; }

// One right-hand side.  In a fused chunk (c->fused_run) the stage's
// forward x pass was done by the previous stage's field pass unless
// `first`, and `fuse_next` lets this stage's field pass do the next one's.
// `end_in_begin`: a Dormand-Prince attempt's controller is left to the
// k_step_begin launch that follows.
int rhs_stage(llgc_ctx* c, const float* ys, Ctl* ctl, int stage,
              const Epi& E, int mode, bool first = true,
              bool fuse_next = false, bool end_in_begin = false) {
  int r;
  if (first && (r = launch_xfwd(c, ys, ctl, stage, mode))) return r;
  if (c->P.modes) {
    // multimode cavity: one coupling sum per mode and x-pass tile
    Timed tm(c, "k_coupling_modes");
    const int R = fwd_rows(c);
    hipLaunchKernelGGL(k_coupling_modes<kT>, xgrid(c, R), dim3(kT), 0,
                       c->stream, c->P, ys, ctl, R);
    if ((r = check_launch(c, "k_coupling_modes"))) return r;
    // the modes' stage rates and next amplitudes (the spectral pass then
    // skips its single-mode finish)
    hipLaunchKernelGGL(k_finish_modes<64>, dim3(1), dim3(64), 0, c->stream,
                       c->P, ctl, (int)xgrid(c, R).x, stage, mode);
    if ((r = check_launch(c, "k_finish_modes"))) return r;
  }
  if (c->P.brms_map) {
    // coupling partial sums with the per-cell B_rms (replace the forward
    // pass's uniform-B_rms sums, tile for tile)
    Timed tm(c, "k_coupling_map");
    const int R = fwd_rows(c);
    hipLaunchKernelGGL(k_coupling_map<kT>, xgrid(c, R), dim3(kT), 0,
                       c->stream, c->P, ys, ctl, c->partials, R);
    if ((r = check_launch(c, "k_coupling_map"))) return r;
  }
  if ((r = launch_yspec(c, ctl, stage, mode))) return r;
  if ((r = launch_xfield(c, ys, ctl, stage, E, fuse_next))) return r;
  if (E.kind == 2 || (E.kind == 3 && !end_in_begin)) {
    Timed tm(c, "k_finish_step");
    hipLaunchKernelGGL(k_finish_step<kT>, dim3(1), dim3(kT), 0, c->stream,
                       c->P, ctl, c->partials,
                       (int)xgrid(c, field_rows(c)).x, E.kind, c->rec);
    if ((r = check_launch(c, "k_finish_step"))) return r;
  }
  return LLGC_OK;
}

// k_begin streams 60 B per cell: two 256-thread workgroups per CU, each
// thread taking several float4 quads in turn, moved the film's 126 MB in
// 23.6 us against 32 us with one quad per thread (2048 workgroups).
int begin_blocks(const llgc_ctx* c) {
  const int per = c->ncu > 0 ? 2 * c->ncu : 512;
  return std::max(1, std::min(per, (c->N / 4 + kT - 1) / kT));
}

// The end of an attempt (controller) fused with the next one's start.
int launch_step_begin(llgc_ctx* c) {
  Timed tm(c, "k_step_begin");
  hipLaunchKernelGGL(k_step_begin<kT>, dim3(begin_blocks(c)), dim3(kT), 0,
                     c->stream, c->P, c->yn, c->kb[0], c->yb[1], c->kb[6],
                     c->yb[0], c->ctl, c->partials, c->rec);
  return check_launch(c, "k_step_begin");
}

int launch_begin(llgc_ctx* c) {
  Timed tm(c, "k_begin");
  hipLaunchKernelGGL(k_begin<kT>, dim3(begin_blocks(c)), dim3(kT), 0,
                     c->stream, c->P, c->yn, c->kb[0], c->yb[1], c->kb[6],
                     c->yb[0], c->ctl, c->partials, c->rec);
  return check_launch(c, "k_begin");
}

int launch_record(llgc_ctx* c) {
  Timed tm(c, "k_record");
  hipLaunchKernelGGL(k_record<kT>, dim3(n_pointwise_blocks(c)), dim3(kT), 0,
                     c->stream, c->P, c->yn, c->ctl, c->partials, c->rec);
  return check_launch(c, "k_record");
}

// --------------------------------------------------------- RK epilogues
Epi epi_eval(float* kout, float* bout) {
  Epi E{};
  E.kind = 0;
  E.kout = kout;
  E.bout = bout;
  return E;
}

// RK4 stage epilogues.  A run keeps y_n intact until a step is known to be
// finite: stage 4 writes the renormalised new state into the scratch
// register yb[0]; stage 1 of the next step reads it from there and copies it
// into y_n (the commit), so a non-finite step leaves y_n at the last
// accepted state.  The run copies y_n into yb[0] before its first step and
// the last accepted state back after its last (run_prepare, run_conclude).
// `inplace`: the adjoint's forward sweeps, which read and write y_n itself.
Epi epi_rk4(llgc_ctx* c, int s, bool inplace = false) {
  Epi E{};
  E.yn = c->yn;
  if (s < 4) {
    E.kind = 1;
    E.np = 0;
    E.cself = (s == 3) ? 1.f : 0.5f;
    E.ynext = c->yb[s % 2];        // stage s reads yb[(s+1)%2] (s>1)
    E.kout = c->kb[s - 1];
    if (s == 1 && !inplace) {
      E.yn = c->yb[0];
      E.commit = c->yn;
    }
  } else {
    E.kind = 2;
    E.np = 3;
    E.kp[0] = c->kb[0];
    E.kp[1] = c->kb[1];
    E.kp[2] = c->kb[2];
    E.ca[0] = (float)(1.0 / 6.0);
    E.ca[1] = (float)(1.0 / 3.0);
    E.ca[2] = (float)(1.0 / 3.0);
    E.cself = (float)(1.0 / 6.0);
    E.ynext = inplace ? c->yn : c->yb[0];
    E.kout = nullptr;
  }
  return E;
}

// Input of RK4 stage s (see epi_rk4).
const float* rk4_input(const llgc_ctx* c, int s, bool inplace = false) {
  if (s == 1) return inplace ? c->yn : c->yb[0];
  return c->yb[(s + 1) % 2];
}

static const double kDPA[8][7] = {
    {0}, {0},
    {1.0 / 5},
    {3.0 / 40, 9.0 / 40},
    {44.0 / 45, -56.0 / 15, 32.0 / 9},
    {19372.0 / 6561, -25360.0 / 2187, 64448.0 / 6561, -212.0 / 729},
    {9017.0 / 3168, -355.0 / 33, 46732.0 / 5247, 49.0 / 176,
     -5103.0 / 18656},
    {35.0 / 384, 0.0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784,
     11.0 / 84}};
static const double kDPE[7] = {
    35.0 / 384 - 5179.0 / 57600, 0.0, 500.0 / 1113 - 7571.0 / 16695,
    125.0 / 192 - 393.0 / 640, -2187.0 / 6784 + 92097.0 / 339200,
    11.0 / 84 - 187.0 / 2100, -1.0 / 40};

Epi epi_dp(llgc_ctx* c, int s) {
  Epi E{};
  E.yn = c->yn;
  E.kout = c->kb[s - 1];
  if (s < 7) {
    E.kind = 1;
    for (int j = 1; j < s; ++j) {
      double a = kDPA[s + 1][j - 1];
      if (a == 0.0) continue;
      E.kp[E.np] = c->kb[j - 1];
      E.ca[E.np] = (float)a;
      E.np++;
    }
    E.cself = (float)kDPA[s + 1][s - 1];
    E.ynext = c->yb[(s + 1) % 2];
  } else {
    E.kind = 3;
    for (int j = 1; j < 7; ++j) {
      if (kDPE[j - 1] == 0.0) continue;
      E.kp[E.np] = c->kb[j - 1];
      E.ca[E.np] = (float)kDPE[j - 1];
      E.np++;
    }
    E.cself = (float)kDPE[6];
    E.ynext = nullptr;
  }
  return E;
}

// ----------------------------------------------------------- host ctl I/O
int ctl_read(llgc_ctx* c, Ctl* h, const Ctl* d) {
  HIPCHK(c, hipMemcpyAsync(h, d, sizeof(Ctl), hipMemcpyDeviceToHost,
                           c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return LLGC_OK;
}
int ctl_write(llgc_ctx* c, Ctl* d, const Ctl* h) {
  HIPCHK(c, hipMemcpyAsync(d, h, sizeof(Ctl), hipMemcpyHostToDevice,
                           c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return LLGC_OK;
}

// Record rows: t, <m>, then Re, Im of the mode (6 doubles) or of each mode
// of a multimode cavity (4 + 2 modes).
int rec_width(const llgc_ctx* c) { return c->nmodes ? 4 + 2 * c->nmodes : 6; }

int ensure_rec(llgc_ctx* c, int64_t cap) {
  const int64_t need = (int64_t)kMaxModes * 2 + 4;   // widest row
  const int64_t n = std::max<int64_t>(cap, 16) * need;
  if (std::max<int64_t>(cap, 16) * rec_width(c) <= c->rec_dev_cap)
    return LLGC_OK;
  if (c->rec) HIPCHK(c, hipFree(c->rec));
  c->rec = nullptr;
  if (hipMalloc(&c->rec, sizeof(double) * n) != hipSuccess)
    return fail(c, LLGC_E_OOM, "record buffer of %lld rows", (long long)cap);
  c->rec_dev_cap = n;
  return LLGC_OK;
}

// ----------------------------------------------------------- demag setup
void gauss_legendre(int n, double* x, double* w) {
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      double dp = n * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) {
        // final derivative for the weight
        p0 = 1.0;
        p1 = z;
        for (int k = 2; k <= n; ++k) {
          double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
          p0 = p1;
          p1 = p2;
        }
        dp = n * (z * p1 - p0) / (z * z - 1.0);
        break;
      }
    }
    x[i] = z;
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= n; ++k) {
      double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    double dp = n * (z * p1 - p0) / (z * z - 1.0);
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

int build_demag_kernel(llgc_ctx* c, double mu0) {
  const size_t n = (size_t)c->N;
  if (!c->tensor) {
    if (hipMalloc(&c->tensor, sizeof(double) * 6 * n) != hipSuccess)
      return fail(c, LLGC_E_OOM, "demag tensor (%zu doubles)", 6 * n);
    GLRule gl;
    gauss_legendre(kGLHalf, gl.x, gl.w);
    dim3 g((c->nx + 127) / 128, c->ny, c->nz);
    hipLaunchKernelGGL(k_tensor, g, dim3(128), 0, c->stream, c->tensor,
                       c->nx, c->ny, c->nz, c->dx, c->dy, c->dz, gl);
    if (int r = check_launch(c, "k_tensor")) return r;
  }
  // twiddle tables in float64 for the separable transforms
  std::vector<double2> twx(c->Px), twy(c->Py);
  for (int m = 0; m < c->Px; ++m) {
    double a = 2.0 * M_PI * m / c->Px;
    twx[m] = make_double2(std::cos(a), std::sin(a));
  }
  for (int m = 0; m < c->Py; ++m) {
    double a = 2.0 * M_PI * m / c->Py;
    twy[m] = make_double2(std::cos(a), std::sin(a));
  }
  double2 *dtx = nullptr, *dty = nullptr;
  double* o1 = nullptr;
  size_t no1 = (size_t)6 * c->nz * c->ny * c->Hx;
  if (hipMalloc(&dtx, sizeof(double2) * c->Px) != hipSuccess ||
      hipMalloc(&dty, sizeof(double2) * c->Py) != hipSuccess ||
      hipMalloc(&o1, sizeof(double) * no1) != hipSuccess) {
    hipFree(dtx);
    hipFree(dty);
    hipFree(o1);
    return fail(c, LLGC_E_OOM, "demag transform scratch");
  }
  hipMemcpyAsync(dtx, twx.data(), sizeof(double2) * c->Px,
                 hipMemcpyHostToDevice, c->stream);
  hipMemcpyAsync(dty, twy.data(), sizeof(double2) * c->Py,
                 hipMemcpyHostToDevice, c->stream);
  hipLaunchKernelGGL(k_dct_x, dim3((c->Hx + 255) / 256, c->ny * c->nz, 6),
                     dim3(256), 0, c->stream, c->tensor, o1, c->nx, c->ny,
                     c->nz, c->Px, c->Hx, dtx);
  int r = check_launch(c, "k_dct_x");
  if (!r) {
    const double scale = -mu0 / ((double)c->Px * (double)c->Py);
    hipLaunchKernelGGL(k_dct_y, dim3((c->Hx + 255) / 256, c->Hy, 6 * c->nz),
                       dim3(256), 0, c->stream, o1, c->K, c->ny, c->nz,
                       c->Py, c->Hx, c->Hy, dty, scale);
    r = check_launch(c, "k_dct_y");
  }
  hipStreamSynchronize(c->stream);
  hipFree(dtx);
  hipFree(dty);
  hipFree(o1);
  if (r) return r;
  c->kernel_built = true;
  c->kernel_mu0 = mu0;
  return LLGC_OK;
}

void fill_prm(llgc_ctx* c) {
  const llgc_params& p = c->prm;
  Prm& P = c->P;
  P.nx = c->nx; P.ny = c->ny; P.nz = c->nz; P.ncell = c->N;
  P.nyp = c->ny + (c->ny & 1);
  P.Px = c->Px; P.Py = c->Py; P.Hx = c->Hx; P.Hy = c->Hy;
  P.logPx = c->logPx; P.logPy = c->logPy;
  P.idx2 = (float)(1.0 / (c->dx * c->dx));
  P.idy2 = (float)(1.0 / (c->dy * c->dy));
  P.idz2 = (float)(1.0 / (c->dz * c->dz));
  P.idx1 = (float)(1.0 / c->dx);
  P.idy1 = (float)(1.0 / c->dy);
  P.idz1 = (float)(1.0 / c->dz);
  P.dmi_i = (float)p.dmi_int;
  P.dmi_b = (float)p.dmi_bulk;
  P.therm = p.temperature > 0
                ? 2.0 * p.alpha * 1.380649e-23 * p.temperature /
                      ((p.gamma > 0 ? p.gamma : 1.7595e11) * c->dx * c->dy *
                       c->dz)
                : 0.0;
  P.seed_lo = (unsigned int)(p.seed & 0xFFFFFFFFull);
  P.seed_hi = (unsigned int)(p.seed >> 32);
  P.ms = (float)p.ms;
  P.ims = p.ms > 0 ? (float)(1.0 / p.ms) : 0.f;
  P.ms_map = c->ms_map;
  P.brms_map = c->brms_map;
  P.masked = c->masked ? 1 : 0;
  P.nmag = c->nmag > 0 ? c->nmag : (double)c->N;
  P.aex2 = (float)(2.0 * p.aex);
  P.ku2 = (float)(2.0 * p.ku1);
  P.ku_map = c->ku_map;
  double un = std::sqrt(p.anis_u[0] * p.anis_u[0] + p.anis_u[1] * p.anis_u[1] +
                        p.anis_u[2] * p.anis_u[2]);
  if (un == 0.0) un = 1.0;
  P.ux = (float)(p.anis_u[0] / un);
  P.uy = (float)(p.anis_u[1] / un);
  P.uz = (float)(p.anis_u[2] / un);
  P.bx = (float)p.bext[0]; P.by = (float)p.bext[1]; P.bz = (float)p.bext[2];
  P.fkind = p.fdrive_kind; P.famp = p.fdrive_amp; P.fw = p.fdrive_w;
  P.fdx = (float)p.fdrive_dir[0]; P.fdy = (float)p.fdrive_dir[1];
  P.fdz = (float)p.fdrive_dir[2];
  P.fdrive_map = c->fdrive_map;
  if (c->fdrive_map) P.fdx = P.fdy = P.fdz = 0.f;   // the map replaces it
  P.demag = p.enable_demag ? 1 : 0;
  P.brx = (float)p.brms[0]; P.bry = (float)p.brms[1]; P.brz = (float)p.brms[2];
  P.brxd = p.brms[0]; P.bryd = p.brms[1]; P.brzd = p.brms[2];
  const double hbar = p.hbar > 0 ? p.hbar : 1.05457182e-34;
  const double gamma = p.gamma > 0 ? p.gamma : 1.7595e11;
  P.wc = p.wc; P.kappa = p.kappa;
  P.vc_hbar = c->dx * c->dy * c->dz / hbar;
  P.ckind = p.cdrive_kind; P.camp = p.cdrive_amp; P.cw = p.cdrive_w;
  P.gpref = (float)(-gamma / (1.0 + p.alpha * p.alpha));
  P.alpha = (float)p.alpha;
  P.method = p.method;
  P.cmode = p.cavity_mode;
  P.ku4 = (float)(4.0 * p.ku2);
  P.prec = p.no_precession ? 0.f : 1.f;
  P.plain = (!c->masked && !c->brms_map && !c->fdrive_map &&
             p.ku2 == 0.0 && !p.no_precession && !c->nmodes &&
             p.dmi_int == 0.0 && p.dmi_bulk == 0.0 &&
             !(p.temperature > 0)) ? 1 : 0;
  P.modes = c->nmodes ? c->modes_dev : nullptr;
  P.mpart = c->mpart;
  P.recw = rec_width(c);
  if (c->nmodes) {
    // the modes replace the single mode of the parameters
    P.brms_map = nullptr;
    P.brx = P.bry = P.brz = 0.f;
    P.brxd = P.bryd = P.brzd = 0.0;
    P.wc = P.kappa = 0.0;
    P.ckind = 0;
    P.camp = 0.0;
  }
  P.tol = p.tol;
  P.dt_min = p.dt_min > 0 ? p.dt_min : 1e-20;
  P.dt_max = p.dt_max > 0 ? p.dt_max : 1e-10;
}

hipEvent_t pooled_event(llgc_ctx* c) {
  hipEvent_t e = nullptr;
  if (!c->event_pool.empty()) {
    e = c->event_pool.back();
    c->event_pool.pop_back();
  } else {
    hipEventCreate(&e);
  }
  return e;
}

int timers_collect(llgc_ctx* c) {
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (auto& kv : c->timers) {
    for (auto& pr : kv.second.pending) {
      float ms = 0.f;
      hipEventElapsedTime(&ms, pr.first, pr.second);
      kv.second.ms += ms;
      c->event_pool.push_back(pr.first);
      c->event_pool.push_back(pr.second);
    }
    kv.second.pending.clear();
  }
  return LLGC_OK;
}

// Quantities that follow from the FFT kinds in use_wy / use_wxf / use_wxi and
// the rows and columns per workgroup: the ky-split choice, LDS sizes (checked
// against the device) and the kernels' LDS limits.
int plan_derive(llgc_ctx* c) {
  const int col = 3 * c->nz * c->Py;
  const int ycap = VPTY * kTyMax;       // complex values one workgroup holds
  const int W = c->W;
  // the ky-parity split of the LDS spectral pass: half the LDS per
  // workgroup (two workgroups per CU) for long columns
  {
    const int hcol = W * 3 * c->nz * (c->Py / 2);
    // 512 or 1024 threads, up to 12 elements each (the instances that
    // compile without register spills: nz <= 3)
    c->Tyh = hcol > kYhEpt * 512 ? 1024 : 512;
    const char* s = getenv("LLGC_YHALF");
    const bool fits = !c->use_wy && c->Py >= 4 &&
                      hcol <= kYhEpt * c->Tyh && hcol <= VPTY * c->Tyh;
    // used where a whole column set exceeds one workgroup (nz = 3, 4 at
    // 2048 points); elsewhere the unsplit pass measured faster
    c->yhalf = !c->batch_plan && fits &&
               ((W * col > ycap) || (c->nz <= 3 && s && atoi(s)));
    c->lds_yh = sizeof(float2) * (lds_twiddles(c->logTw) +
                                  padded_len((size_t)hcol));
  }
  if (!c->use_wy && !c->yhalf && W * col > ycap)
    return fail(c, LLGC_E_UNSUPPORTED, "column set exceeds one workgroup");
  const size_t twb = sizeof(float2) * lds_twiddles(c->logTw);  // LDS twiddles
  const size_t fcol = (size_t)(c->Rf / 2) * c->Px;   // one forward tile
  c->lds_f = twb + sizeof(float2) * ((c->batch_plan || c->x3)
                                         ? padded_len(3 * fcol)
                                         : padded_len_s<kXfPs>(fcol));
  c->lds_i = sizeof(float2) * padded_len_s<kPsField>((size_t)3 * (c->Ri / 2) * c->Px);
  // the spectral pass is specialised on 1024 and 2048 points (yspec_nz)
  const int lpy = (c->logPy == 10 || c->logPy == 11) ? c->logPy : 0;
  c->lds_y = sizeof(float2) * (yspec_tw_len(lpy, c->logTw) +
                               padded_len((size_t)W * col));
  // two layers of 1024 or 2048 points, one kx slot per block: the split
  // pass (k_yspec_z) needs LDS for three columns only, so two workgroups
  // share a CU (film: 59.7 -> 57.0 us); LLGC_NO_YSPLIT keeps k_yspec
  c->ysplit = getenv("LLGC_NO_YSPLIT") == nullptr && c->nz == 2 && W == 1 &&
              lpy > 0 && !c->use_wy && !c->yhalf && !c->batch_plan &&
              c->Px >= 2;
  c->lds_yz = sizeof(float2) * (yspec_tw_len(lpy, c->logTw) +
                                padded_len_s<kYzPs>((size_t)3 * c->Py));
  int dev = 0, maxlds = 65536;
  hipGetDevice(&dev);
  hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock,
                        dev);
  // LDS of the kernels this plan launches
  const size_t need_y = c->use_wy ? 0 : (c->yhalf ? c->lds_yh : c->lds_y);
  size_t need = std::max(c->use_wxf ? 0 : c->lds_f,
                         std::max(c->use_wxi ? 0 : c->lds_i, need_y));
  if (need > (size_t)std::max(maxlds, 65536) && need > 65536)
    return fail(c, LLGC_E_UNSUPPORTED,
                "plan needs more LDS than the device offers");
  {
    const void* xf[] = {
        (const void*)k_xfwd<kTX, true, 0>, (const void*)k_xfwd<kTX, true, 10>,
        (const void*)k_xfwd<kTX, true, 11>, (const void*)k_xfwd<kTX, false, 0>,
        (const void*)k_xfwd<kTX, false, 10>,
        (const void*)k_xfwd<kTX, false, 11>};
    for (const void* f : xf)
      raise_lds_limit(f, c->lds_f);
    const void* xi[] = {
        (const void*)k_xfield<kTX, 0>, (const void*)k_xfield<kTX, 8>,
        (const void*)k_xfield<kTX, 9>, (const void*)k_xfield<kTX, 10>,
        (const void*)k_xfield<kTX, 11>};
    for (const void* f : xi)
      raise_lds_limit(f, c->lds_i);
    raise_lds_limit((const void*)k_xfwd3<kTX>, c->lds_f);
    const void* xff[] = {
        (const void*)k_xfield_fwd<kTX, 8>, (const void*)k_xfield_fwd<kTX, 9>,
        (const void*)k_xfield_fwd<kTX, 10>, (const void*)k_xfield_fwd<kTX, 11>,
        (const void*)k_xfwd_fx<kTX, 8>, (const void*)k_xfwd_fx<kTX, 9>,
        (const void*)k_xfwd_fx<kTX, 10>, (const void*)k_xfwd_fx<kTX, 11>};
    for (const void* f : xff)
      raise_lds_limit(f, c->lds_i);
    raise_lds_limit((const void*)k_xfield_b<kTX>, c->lds_i);
  }
  if (c->yhalf) {
    const void* fs[] = {
        (const void*)k_yspec_h<512, 1, kYhEpt>, (const void*)k_yspec_h<512, 2, kYhEpt>,
        (const void*)k_yspec_h<512, 3, kYhEpt>, (const void*)k_yspec_h<1024, 1, kYhEpt>,
        (const void*)k_yspec_h<1024, 2, kYhEpt>, (const void*)k_yspec_h<1024, 3, kYhEpt>,
        (const void*)k_yspec_h<1024, 4, kYhEpt>};
    for (const void* f : fs)
      raise_lds_limit(f, c->lds_yh);
  }
  if (!c->use_wy && !c->yhalf) {
    yspec_attr<256>(c->lds_y);
    yspec_attr<512>(c->lds_y);
    if constexpr (kTyMax >= 1024) {
      yspec_attr<1024>(c->lds_y);
      // residency of the block-stepping instances, queried here rather
      // than at a launch that may be under stream capture
      const void* fs[] = {
          (const void*)k_yspec<1024, 1, 0>, (const void*)k_yspec<1024, 2, 0>,
          (const void*)k_yspec<1024, 1, 10>, (const void*)k_yspec<1024, 2, 10>,
          (const void*)k_yspec<1024, 1, 11>, (const void*)k_yspec<1024, 2, 11>};
      for (const void* f : fs) blocks_per_cu(f, 1024, c->lds_y);
    }
  }
  if (c->ysplit) {
    raise_lds_limit((const void*)k_yspec_z<10>, c->lds_yz);
    raise_lds_limit((const void*)k_yspec_z<11>, c->lds_yz);
  }
  return LLGC_OK;
}

// ---------------------------------------------------------------- autotune
// A plan kind says which passes keep their FFT in registers: bit 0 the
// spectral (y) pass, bit 1 the forward x pass, bit 2 the field x pass; rows
// and columns per workgroup follow each kind as in the default plan.
// Bit 3: both x passes in LDS over the three components of a tile at once
// (the batch plan's x kernels; rows per tile sized to fill the workgroup).
bool plan_kind_ok(const llgc_ctx* c, int k) {
  if ((k & 1) && !(c->Py >= 64 && c->Py <= 2048 &&
                   (c->Py < 2048 || c->nz <= 2)))
    return false;
  if ((k & 6) && !(c->Px >= 64 && c->Px <= 2048)) return false;
  if ((k & 8) && ((k & 6) || c->Px < 64)) return false;
  return true;
}
int plan_kind(const llgc_ctx* c) {
  return (c->use_wy ? 1 : 0) | (c->use_wxf ? 2 : 0) | (c->use_wxi ? 4 : 0) |
         (c->x3 ? 8 : 0);
}
void plan_set_kind(llgc_ctx* c, int k) {
  c->use_wy = (k & 1) != 0;
  c->use_wxf = (k & 2) != 0;
  c->use_wxi = (k & 4) != 0;
  c->x3 = (k & 8) != 0;
}
// Rows per tile of the three-component x passes: 3 (R/2) Px fills
// VPT * kTX complex values, tiles splitting ny evenly.
int x3_rows(const llgc_ctx* c) {
  const int npmax = std::max(1, VPT * kTX / (3 * c->Px));
  const int pairs = (c->ny + 1) / 2;
  const int nty = (pairs + npmax - 1) / npmax;
  return 2 * ((pairs + nty - 1) / nty);
}

// Mean milliseconds of one right-hand-side evaluation (forward x pass,
// spectral pass, field pass) under the current plan, over `reps`
// evaluations of the current state into a scratch k register.
int time_rhs(llgc_ctx* c, int reps, double* ms) {
  Ctl h{};
  h.t_end = 1e300;
  if (int r = ctl_write(c, c->ctl_eval, &h)) return r;
  const Epi E = epi_eval(c->kb[1], nullptr);
  hipEvent_t e0, e1;
  HIPCHK(c, hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    hipEventDestroy(e0);
    return fail(c, LLGC_E_HIP, "hipEventCreate failed");
  }
  int r = rhs_stage(c, c->yn, c->ctl_eval, 1, E, 1);   // untimed first call
  if (!r && hipEventRecord(e0, c->stream) != hipSuccess)
    r = fail(c, LLGC_E_HIP, "hipEventRecord failed");
  for (int i = 0; i < reps && !r; ++i)
    r = rhs_stage(c, c->yn, c->ctl_eval, 1, E, 1);
  float t = 0.f;
  if (!r && (hipEventRecord(e1, c->stream) != hipSuccess ||
             hipEventSynchronize(e1) != hipSuccess ||
             hipEventElapsedTime(&t, e0, e1) != hipSuccess))
    r = fail(c, LLGC_E_HIP, "timing events failed");
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  *ms = (double)t / std::max(1, reps);
  return r;
}

// Tuned plan kinds per grid shape (process-wide).
// Plan shape: FFT kind plus rows per x-pass tile and kx columns per
// spectral workgroup.
struct PlanShape {
  int kind, Rf, Ri, Rw, Rwf, W;
};
PlanShape plan_get(const llgc_ctx* c) {
  return PlanShape{plan_kind(c), c->Rf, c->Ri, c->Rw, c->Rwf, c->W};
}
void plan_put(llgc_ctx* c, const PlanShape& s) {
  plan_set_kind(c, s.kind);
  c->Rf = s.Rf;
  c->Ri = s.Ri;
  c->Rw = s.Rw;
  c->Rwf = s.Rwf;
  c->W = s.W;
  const int col = 3 * c->nz * c->Py;
  c->Ty = 256;
  while (c->Ty < kTyMax && c->W * col > VPTY * c->Ty) c->Ty *= 2;
}
// Register-budget limits of the LDS kernels' tiles (as at creation): rows
// per forward / field tile, spectral column slots per workgroup.
void plan_limits(const llgc_ctx* c, int* rf_max, int* ri_max, int* w_max) {
  const int VPTT = VPT * kTX;
  *rf_max = 2 * std::max(1, std::min(8, VPTT / c->Px));
  *ri_max = 2 * std::max(1, std::min(8, VPTT / (3 * c->Px)));
  if (c->x3) *rf_max = *ri_max = 2 * std::max(1, VPTT / (3 * c->Px));
  const int col = 3 * c->nz * c->Py;
  *w_max = std::max(1, std::min(VPTY * kTyMax / col,
                                (int)(kLdsCap / (9 * col))));
}

// Tuned plan shapes per grid shape (process-wide).
std::map<std::tuple<int, int, int, int>, PlanShape> g_tuned;
std::mutex g_tuned_mu;

// ------------------------------------------------------- launch sequences
constexpr int kDpChunk = 8;   // Dormand-Prince attempts per host check

// The launches of one chunk, issued on c->stream: kind 0 = kDpChunk
// Dormand-Prince attempts (stages 2..7, then the next attempt's start),
// kind 1 = one RK4 step (stages 1..4).
int chunk_direct(llgc_ctx* c, int kind, int attempts = kDpChunk) {
  int r = LLGC_OK;
  const bool fz = fusable(c);
  c->fused_run = fz;
  if (kind == 1) {
    for (int s = 1; s <= 4 && !r; ++s) {
      r = rhs_stage(c, rk4_input(c, s), c->ctl, s, epi_rk4(c, s), 0,
                    !fz || s == 1, fz && s < 4);
    }
  } else {
    for (int b = 0; b < attempts && !r; ++b) {
      for (int s = 2; s <= 7 && !r; ++s) {
        Epi E = epi_dp(c, s);
        if (s == 7 && c->step_begin)
          E.emax = (unsigned int*)((char*)c->ctl + offsetof(Ctl, emax_bits));
        r = rhs_stage(c, c->yb[s % 2], c->ctl, s, E, 0, !fz || s == 2,
                      fz && s < 7, c->step_begin);
      }
      if (!r) r = c->step_begin ? launch_step_begin(c) : launch_begin(c);
    }
  }
  c->fused_run = false;
  return r;
}

// Everything a captured chunk depends on besides device memory contents:
// the parameters passed by value, the plan and the record buffer.
std::vector<unsigned char> chunk_signature(const llgc_ctx* c) {
  std::vector<unsigned char> v;
  auto put = [&v](const void* p, size_t n) {
    const unsigned char* b = (const unsigned char*)p;
    v.insert(v.end(), b, b + n);
  };
  put(&c->P, sizeof(Prm));
  const int plan[] = {c->use_wy, c->use_wxf, c->use_wxi, c->yhalf, c->x3,
                      c->ysplit,
                      c->Rf,     c->Ri,      c->W,       c->Ty,    c->Ww,
                      c->Rw,     c->Rwf,     c->Tyh,     (int)c->lds_f,
                      (int)c->lds_i, (int)c->lds_y, (int)c->lds_yh};
  put(plan, sizeof(plan));
  put(&c->rec, sizeof(c->rec));
  put(&c->ms_map, sizeof(c->ms_map));
  put(&c->ku_map, sizeof(c->ku_map));
  return v;
}

void graph_release(llgc_ctx* c, int kind) {
  if (c->graph_exec[kind]) hipGraphExecDestroy(c->graph_exec[kind]);
  if (c->graph[kind]) hipGraphDestroy(c->graph[kind]);
  c->graph_exec[kind] = nullptr;
  c->graph[kind] = nullptr;
  c->graph_sig[kind].clear();
}

// One chunk, replayed from a HIP graph captured on a private stream (only
// kernel nodes: no copies or memsets inside); re-captured when the
// signature changes.  Timed runs launch directly (events stay outside
// graphs).
int run_chunk(llgc_ctx* c, int kind) {
  if (!c->graphs || c->timing) return chunk_direct(c, kind);
  std::vector<unsigned char> sig = chunk_signature(c);
  if (!c->graph_exec[kind] || sig != c->graph_sig[kind]) {
    graph_release(c, kind);
    if (!c->cap_stream)
      HIPCHK(c, hipStreamCreateWithFlags(&c->cap_stream,
                                         hipStreamNonBlocking));
    // capture records the launches without running them; the graph then
    // runs on the caller's stream, after the work already queued there
    hipStream_t user = c->stream;
    c->stream = c->cap_stream;
    if (hipStreamBeginCapture(c->cap_stream,
                              hipStreamCaptureModeThreadLocal) != hipSuccess) {
      // capture unavailable (e.g. the caller is capturing this thread):
      // this context launches directly from now on
      c->stream = user;
      (void)hipGetLastError();
      c->graphs = false;
      return chunk_direct(c, kind);
    }
    int r = chunk_direct(c, kind);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
    c->stream = user;
    if (!r && e != hipSuccess)
      r = fail(c, LLGC_E_HIP, "hipStreamEndCapture: %s",
               hipGetErrorString(e));
    if (!r && hipGraphInstantiate(&c->graph_exec[kind], g, nullptr,
                                  nullptr, 0) != hipSuccess) {
      c->graph_exec[kind] = nullptr;
      r = fail(c, LLGC_E_HIP, "hipGraphInstantiate failed");
    }
    if (r) {
      if (g) hipGraphDestroy(g);
      (void)hipGetLastError();
      return r;
    }
    c->graph[kind] = g;
    c->graph_sig[kind] = std::move(sig);
  }
  HIPCHK(c, hipGraphLaunch(c->graph_exec[kind], c->stream));
  return LLGC_OK;
}

}  // namespace

// ================================================================== C ABI
extern "C" {

int llgc_create(const llgc_grid* g, void* stream, llgc_ctx** out) {
  return llgc_create_ex(g, stream, 0, out);
}

int llgc_create_ex(const llgc_grid* g, void* stream, int flags,
                   llgc_ctx** out) {
  if (!g || !out) return LLGC_E_ARG;
  *out = nullptr;
  if (g->nx < 1 || g->ny < 1 || g->nz < 1 || !(g->dx > 0) || !(g->dy > 0) ||
      !(g->dz > 0) || (flags & ~LLGC_PLAN_BATCH))
    return LLGC_E_ARG;
  if (g->nz > 4 || g->nx > kMaxLen / 2 || g->ny > kMaxLen / 2)
    return LLGC_E_UNSUPPORTED;
  const bool bplan = (flags & LLGC_PLAN_BATCH) != 0;
  if (bplan && (g->nx < 2 || g->ny < 2 || g->nx > kBatchMaxLen / 2 ||
                g->ny > kBatchMaxLen / 2))
    return LLGC_E_UNSUPPORTED;
  llgc_ctx* c = new llgc_ctx();
  c->nx = g->nx; c->ny = g->ny; c->nz = g->nz;
  c->N = g->nx * g->ny * g->nz;
  c->dx = g->dx; c->dy = g->dy; c->dz = g->dz;
  c->stream = (hipStream_t)stream;
  hipGetDevice(&c->device);
  if (hipDeviceGetAttribute(&c->ncu, hipDeviceAttributeMultiprocessorCount,
                            c->device) != hipSuccess)
    c->ncu = 0;
  c->no_ypersist = getenv("LLGC_NO_YPERSIST") != nullptr;
  c->step_begin = getenv("LLGC_NO_STEP_BEGIN") == nullptr;
  c->no_fuse = getenv("LLGC_NO_FUSE") != nullptr;
  c->force_fuse = getenv("LLGC_FUSE") != nullptr;
  c->batch_plan = bplan;
  c->graphs = getenv("LLGC_NO_GRAPHS") == nullptr;
  c->Px = g->nx == 1 ? 1 : pow2_ceil(2 * g->nx);
  c->Py = g->ny == 1 ? 1 : pow2_ceil(2 * g->ny);
  if (bplan) {
    // batch plan: padded lengths of at least 64 (one plan family for the
    // 16..128-cell instances of a sweep)
    c->Px = std::max(c->Px, 64);
    c->Py = std::max(c->Py, 64);
  }
  c->Hx = c->Px / 2 + 1;
  c->Hy = c->Py / 2 + 1;
  c->logPx = ilog2(c->Px);
  c->logPy = ilog2(c->Py);
  c->logTw = ilog2(std::max(c->Px, c->Py));
  // --- plan: rows per x-pass block, kx columns per spectral block
  const int VPTT = VPT * kTX;
  int npf = std::max(1, std::min(8, VPTT / c->Px));
  int npi = std::max(1, std::min(8, VPTT / (3 * c->Px)));
  if (npf * c->Px > VPTT || 3 * npi * c->Px > VPTT) {
    delete c;
    return LLGC_E_UNSUPPORTED;
  }
  // rows per x-pass tile: even (rows are paired into complex transforms)
  auto pick_rows = [&](int npmax) {
    int R = 2 * npmax;
    while (R > 2 && ((c->ny + R - 1) / R) * c->nz < 512) R -= 2;
    return std::min(R, c->ny + (c->ny & 1));
  };
  c->Rf = pick_rows(npf);
  c->Ri = pick_rows(npi);
  // tuning overrides (rounded up to even, capped by the register budget)
  if (const char* s = getenv("LLGC_RF"))
    c->Rf = std::min(2 * npf, std::max(2, (atoi(s) + 1) & ~1));
  if (const char* s = getenv("LLGC_RI"))
    c->Ri = std::min(2 * npi, std::max(2, (atoi(s) + 1) & ~1));
  const int col = 3 * c->nz * c->Py;
  const int ycap = VPTY * kTyMax;       // complex values one workgroup holds
  int W = std::max(1, std::min(ycap / col, (int)(kLdsCap / (9 * col))));
  while (W > 1 && (c->Hx + W - 1) / W < 256) --W;
  if (const char* s = getenv("LLGC_W"))
    W = std::max(1, std::min(atoi(s), ycap / col));
  c->W = W;
  c->Ty = 256;
  while (c->Ty < kTyMax && W * col > VPTY * c->Ty) c->Ty *= 2;
  // One wavefront per transform with the FFT in registers where that was
  // measured faster than the LDS Stockham kernels (gfx950, DP45 steps of
  // 32^2 x 2 ... 1024^2 x 2 grids): y columns of 128..512 points, forward
  // x rows of 64..256, field-pass x rows of 64..128.  Longer transforms
  // need 128+ VGPRs per lane in registers (2 waves per SIMD) and lose.
  const bool lds_y = getenv("LLGC_LDS_YFFT") != nullptr;
  const bool lds_x = getenv("LLGC_LDS_XFFT") != nullptr;
  const bool wave_all = getenv("LLGC_WAVE_FFT") != nullptr;
  c->use_wy = !lds_y && (wave_all ? (c->Py >= 64 && (c->Py < 2048 || c->nz <= 2))
                                  : (c->Py >= 128 && c->Py <= 512));
  c->Ww = std::max(1, 6 / (3 * c->nz));
  c->use_wxf = !lds_x && c->Px >= 64 && (wave_all || c->Px <= 256);
  c->use_wxi = !lds_x && c->Px >= 64 && (wave_all || c->Px <= 128);
  c->Rw = (((c->ny + 3) / 4) * c->nz >= 512) ? 4 : 2;
  if (const char* s = getenv("LLGC_RW")) c->Rw = (atoi(s) >= 4) ? 4 : 2;
  c->Rwf = 2;
  if (const char* s = getenv("LLGC_RWF")) c->Rwf = (atoi(s) >= 4) ? 4 : 2;
  if (!bplan && c->Px >= 64 && getenv("LLGC_X3")) {
    // the three-component x passes (plan kind bit 3)
    c->use_wxf = c->use_wxi = false;
    c->x3 = true;
    c->Rf = c->Ri = x3_rows(c);
  }
  if (bplan) {
    // the fixed plan of every batched instance (no tuning overrides):
    // register FFTs along x, the LDS spectral pass with kBatchTy threads
    // and as many column slots per workgroup as its VPTY * kBatchTy
    // elements hold (measured 1.3-2x faster per element than the register
    // spectral pass at 64..256 points once the GPU is full)
    c->use_wxf = c->use_wxi = c->use_wy = false;
    // x passes: the 3 (R/2) transforms of a tile fill one kTX-thread
    // workgroup (VPT values each); tiles split ny evenly
    const int npmax = std::max(1, VPT * kTX / (3 * c->Px));
    const int pairs = (c->ny + 1) / 2;
    const int nty = (pairs + npmax - 1) / npmax;
    c->Rf = c->Ri = 2 * ((pairs + nty - 1) / nty);
    c->Ty = kBatchTy;
    W = std::max(1, std::min(VPTY * kBatchTy / col, c->Px / 2));
    c->W = W;
  }
  if (int r = plan_derive(c)) {
    delete c;
    return r;
  }
  // --- buffers
  const size_t n3 = (size_t)3 * c->N;
  bool ok = hipMalloc(&c->yn, n3 * 4) == hipSuccess &&
            hipMalloc(&c->yb[0], n3 * 4) == hipSuccess &&
            hipMalloc(&c->yb[1], n3 * 4) == hipSuccess;
  for (int j = 0; j < 7 && ok; ++j)
    ok = hipMalloc(&c->kb[j], n3 * 4) == hipSuccess;
  const size_t nspec = (size_t)c->Hx * c->nz * 3 * (c->ny + (c->ny & 1));
  const size_t nK = (size_t)c->Hx * c->Hy * kentry(c->nz);
  ok = ok && hipMalloc(&c->spec, nspec * sizeof(float2)) == hipSuccess &&
       hipMalloc(&c->K, nK * sizeof(float)) == hipSuccess &&
       hipMalloc(&c->ctl, sizeof(Ctl)) == hipSuccess &&
       hipMalloc(&c->ctl_eval, sizeof(Ctl)) == hipSuccess;
  const int Ltw = 1 << c->logTw;
  ok = ok && hipMalloc(&c->tw, sizeof(float2) * Ltw) == hipSuccess;
  size_t nb = std::max<size_t>({(size_t)xgrid(c, c->Rf).x,
                                 (size_t)xgrid(c, c->Ri).x,
                                 (size_t)xgrid(c, 2).x,
                                 (size_t)n_pointwise_blocks(c)});
  c->npartials = 4 * nb + 16;
  ok = ok && hipMalloc(&c->partials, sizeof(double) * c->npartials) ==
                 hipSuccess;
  if (!ok) {
    llgc_destroy(c);
    return LLGC_E_OOM;
  }
  std::vector<float2> tw(Ltw);
  for (int m = 0; m < Ltw; ++m) {
    double a = -2.0 * M_PI * m / Ltw;
    tw[m] = make_float2((float)std::cos(a), (float)std::sin(a));
  }
  Ctl z{};
  if (hipMemcpy(c->tw, tw.data(), sizeof(float2) * Ltw,
                hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->ctl, &z, sizeof(Ctl), hipMemcpyHostToDevice) !=
          hipSuccess ||
      hipMemcpy(c->ctl_eval, &z, sizeof(Ctl), hipMemcpyHostToDevice) !=
          hipSuccess ||
      hipMemset(c->spec, 0, nspec * sizeof(float2)) != hipSuccess) {
    llgc_destroy(c);
    return LLGC_E_HIP;
  }
  if (ensure_rec(c, 16)) {
    llgc_destroy(c);
    return LLGC_E_OOM;
  }
  *out = c;
  return LLGC_OK;
}

int llgc_destroy(llgc_ctx* c) {
  if (!c) return LLGC_OK;
  if (c->stream) hipStreamSynchronize(c->stream);
  else hipDeviceSynchronize();
  timers_collect(c);
  for (hipEvent_t e : c->event_pool) hipEventDestroy(e);
  graph_release(c, 0);
  graph_release(c, 1);
  if (c->cap_stream) hipStreamDestroy(c->cap_stream);
  hipFree(c->yn);
  hipFree(c->yb[0]);
  hipFree(c->yb[1]);
  for (auto* p : c->kb) hipFree(p);
  hipFree(c->spec);
  hipFree(c->K);
  hipFree(c->tensor);
  hipFree(c->tw);
  hipFree(c->partials);
  hipFree(c->rec);
  hipFree(c->ctl);
  hipFree(c->ctl_eval);
  hipFree(c->ms_map);
  hipFree(c->brms_map);
  hipFree(c->fdrive_map);
  hipFree(c->modes_dev);
  hipFree(c->mode_maps);
  hipFree(c->mpart);
  hipFree(c->ku_map);
  delete c;
  return LLGC_OK;
}

const char* llgc_last_error(const llgc_ctx* c) {
  if (!c) return "null context";
  return c->err.c_str();
}

int llgc_set_params(llgc_ctx* c, const llgc_params* p) {
  if (!c) return LLGC_E_ARG;
  if (!p) return fail(c, LLGC_E_ARG, "params is NULL");
  if (!p->ms_map && !(p->ms > 0))
    return fail(c, LLGC_E_ARG, "ms must be > 0 without a map");
  if (!(p->alpha >= 0) || !(p->aex >= 0))
    return fail(c, LLGC_E_ARG, "alpha and aex must be >= 0");
  if (p->method != LLGC_RK4 && p->method != LLGC_DP45)
    return fail(c, LLGC_E_ARG, "unknown method %d", p->method);
  if (p->fdrive_kind < 0 || p->fdrive_kind > 2 || p->cdrive_kind < 0 ||
      p->cdrive_kind > 2)
    return fail(c, LLGC_E_ARG, "unknown drive kind");
  if (!(p->dt > 0)) return fail(c, LLGC_E_ARG, "dt must be > 0");
  if (p->method == LLGC_DP45 && !(p->tol > 0))
    return fail(c, LLGC_E_ARG, "tol must be > 0");
  if (!(p->kappa >= 0)) return fail(c, LLGC_E_ARG, "kappa must be >= 0");
  if (p->cavity_mode != LLGC_CAVITY_ODE &&
      p->cavity_mode != LLGC_CAVITY_MEMORY)
    return fail(c, LLGC_E_ARG, "unknown cavity mode %d", p->cavity_mode);
  if (p->cavity_mode == LLGC_CAVITY_MEMORY &&
      (p->method != LLGC_RK4 || p->cdrive_kind != 0))
    return fail(c, LLGC_E_UNSUPPORTED,
                "the memory recursion runs with RK4 and no cavity drive");
  if (p->cavity_mode == LLGC_CAVITY_MEMORY && c->nmodes)
    return fail(c, LLGC_E_UNSUPPORTED,
                "the memory recursion is written for one mode");
  if (!(p->temperature >= 0)) return fail(c, LLGC_E_ARG, "temperature < 0");
  if (p->temperature > 0 && p->method != LLGC_RK4)
    return fail(c, LLGC_E_UNSUPPORTED,
                "the thermal field needs fixed steps (RK4)");
  c->prm = *p;
  const size_t nb = sizeof(float) * c->N;
  if (p->ms_map) {
    // geometry: cells with Ms = 0 are outside the magnet; values must be
    // finite and >= 0 with at least one magnetic cell
    std::vector<float> h(c->N);
    HIPCHK(c, hipMemcpy(h.data(), p->ms_map, nb, hipMemcpyDeviceToHost));
    int64_t nm = 0;
    for (float v : h) {
      if (!(v >= 0.f) || !std::isfinite(v))
        return fail(c, LLGC_E_ARG, "ms_map values must be finite and >= 0");
      nm += v > 0.f ? 1 : 0;
    }
    if (nm == 0) return fail(c, LLGC_E_ARG, "ms_map has no magnetic cell");
    if (!c->ms_map) HIPCHK(c, hipMalloc(&c->ms_map, nb));
    HIPCHK(c, hipMemcpyAsync(c->ms_map, p->ms_map, nb,
                             hipMemcpyDeviceToDevice, c->stream));
    c->masked = nm < c->N;
    c->nmag = (double)nm;
  } else {
    if (c->ms_map) {
      HIPCHK(c, hipFree(c->ms_map));
      c->ms_map = nullptr;
    }
    c->masked = false;
    c->nmag = (double)c->N;
  }
  if (p->ku1_map) {
    if (!c->ku_map) HIPCHK(c, hipMalloc(&c->ku_map, nb));
    HIPCHK(c, hipMemcpyAsync(c->ku_map, p->ku1_map, nb,
                             hipMemcpyDeviceToDevice, c->stream));
  } else if (c->ku_map) {
    HIPCHK(c, hipFree(c->ku_map));
    c->ku_map = nullptr;
  }
  if (p->brms_map) {
    if (!c->brms_map) HIPCHK(c, hipMalloc(&c->brms_map, 3 * nb));
    HIPCHK(c, hipMemcpyAsync(c->brms_map, p->brms_map, 3 * nb,
                             hipMemcpyDeviceToDevice, c->stream));
  } else if (c->brms_map) {
    HIPCHK(c, hipFree(c->brms_map));
    c->brms_map = nullptr;
  }
  if (p->fdrive_map) {
    if (!c->fdrive_map) HIPCHK(c, hipMalloc(&c->fdrive_map, 3 * nb));
    HIPCHK(c, hipMemcpyAsync(c->fdrive_map, p->fdrive_map, 3 * nb,
                             hipMemcpyDeviceToDevice, c->stream));
  } else if (c->fdrive_map) {
    HIPCHK(c, hipFree(c->fdrive_map));
    c->fdrive_map = nullptr;
  }
  fill_prm(c);
  if (c->have_state && c->masked) {
    hipLaunchKernelGGL(k_clear_empty<kT>, dim3(n_pointwise_blocks(c)),
                       dim3(kT), 0, c->stream, c->P, c->yn);
    if (int r = check_launch(c, "k_clear_empty")) return r;
  }
  const double mu0 = p->mu0 > 0 ? p->mu0 : 4e-7 * M_PI;
  if (p->enable_demag && (!c->kernel_built || c->kernel_mu0 != mu0)) {
    if (int r = build_demag_kernel(c, mu0)) return r;
  }
  Ctl h{};
  if (int r = ctl_read(c, &h, c->ctl)) return r;
  if (!c->have_state) {
    h.t = 0.0;
    h.a_re = 0.5 * p->x0;
    h.a_im = -0.5 * p->p0;
  }
  h.dt = p->dt;
  h.as_re[1] = h.a_re;
  h.as_im[1] = h.a_im;
  if (int r = ctl_write(c, c->ctl, &h)) return r;
  c->have_params = true;
  c->need_init = true;
  return LLGC_OK;
}

int llgc_set_state(llgc_ctx* c, const float* m, double t, double are,
                   double aim) {
  if (!c) return LLGC_E_ARG;
  if (!m) return fail(c, LLGC_E_ARG, "m is NULL");
  HIPCHK(c, hipMemcpyAsync(c->yn, m, sizeof(float) * 3 * c->N,
                           hipMemcpyDeviceToDevice, c->stream));
  if (c->have_params && c->masked) {   // no magnetisation outside
    hipLaunchKernelGGL(k_clear_empty<kT>, dim3(n_pointwise_blocks(c)),
                       dim3(kT), 0, c->stream, c->P, c->yn);
    if (int r = check_launch(c, "k_clear_empty")) return r;
  }
  Ctl h{};
  if (int r = ctl_read(c, &h, c->ctl)) return r;
  h.t = t;
  h.a_re = are;
  h.a_im = aim;
  h.as_re[1] = are;
  h.as_im[1] = aim;
  for (int k = 0; k < c->nmodes; ++k) {   // mode amplitudes stay as set
    h.mas_re[1][k] = h.ma_re[k];
    h.mas_im[1][k] = h.ma_im[k];
  }
  h.pending_accept = 0;
  h.done = 0;
  h.status = 0;
  h.prev_rej = 0;
  h.mem_n = 0;
  h.noise_n = 0;
  if (c->have_params) h.dt = c->prm.dt;
  if (int r = ctl_write(c, c->ctl, &h)) return r;
  c->have_state = true;
  c->need_init = true;
  return LLGC_OK;
}

int llgc_get_state(llgc_ctx* c, float* m, double* t, double* a) {
  if (!c) return LLGC_E_ARG;
  if (m)
    HIPCHK(c, hipMemcpyAsync(m, c->yn, sizeof(float) * 3 * c->N,
                             hipMemcpyDeviceToDevice, c->stream));
  Ctl h{};
  if (int r = ctl_read(c, &h, c->ctl)) return r;
  if (t) *t = h.t;
  if (a) {
    a[0] = h.a_re;
    a[1] = h.a_im;
  }
  return LLGC_OK;
}

int llgc_reset_cavity(llgc_ctx* c, double x0, double p0) {
  if (!c) return LLGC_E_ARG;
  Ctl h{};
  if (int r = ctl_read(c, &h, c->ctl)) return r;
  h.t = 0.0;
  h.a_re = 0.5 * x0;
  h.a_im = -0.5 * p0;
  h.as_re[1] = h.a_re;
  h.as_im[1] = h.a_im;
  for (int k = 0; k < c->nmodes; ++k) {   // each mode from its own x0, p0
    h.ma_re[k] = h.mas_re[1][k] = 0.5 * c->mode_h[k].x0;
    h.ma_im[k] = h.mas_im[1][k] = -0.5 * c->mode_h[k].p0;
  }
  h.mem_n = 0;
  if (int r = ctl_write(c, c->ctl, &h)) return r;
  c->need_init = true;
  return LLGC_OK;
}

int llgc_cavity_enabled(const llgc_ctx* c) {
  if (!c) return LLGC_E_ARG;
  if (!c->have_params) return 0;
  const double* b = c->prm.brms;
  if (c->nmodes) {
    for (int k = 0; k < c->nmodes; ++k) {
      const double* q = c->mode_h[k].brms;
      if (c->mode_h[k].brms_map || q[0] != 0.0 || q[1] != 0.0 || q[2] != 0.0)
        return 1;
    }
    return 0;
  }
  if (c->brms_map) return 1;
  return (b[0] != 0.0 || b[1] != 0.0 || b[2] != 0.0) ? 1 : 0;
}

int llgc_relax(llgc_ctx* c, double torque_tol, int64_t max_steps,
               double* max_torque, llgc_run_info* info) {
  if (!c) return LLGC_E_ARG;
  if (!c->have_params || !c->have_state)
    return fail(c, LLGC_E_STATE, "set params and state before relax");
  if (max_steps <= 0) max_steps = 100000;
  Ctl h0{};
  if (int r = ctl_read(c, &h0, c->ctl)) return r;
  {
    // the step controller starts afresh; the decoupled cavity is held at
    // zero (its amplitude is restored afterwards), so it adds nothing to
    // the step-size control
    Ctl hs = h0;
    hs.prev_rej = 0;
    hs.a_re = hs.a_im = hs.as_re[1] = hs.as_im[1] = 0.0;
    for (int k = 0; k < kMaxModes; ++k)
      hs.ma_re[k] = hs.ma_im[k] = hs.mas_re[1][k] = hs.mas_im[1][k] = 0.0;
    if (int r = ctl_write(c, c->ctl, &hs)) return r;
  }
  // relaxation problem: precession off, cavity decoupled, drives off,
  // Dormand-Prince; everything restored on the way out
  struct Saved {
    llgc_ctx* c;
    llgc_params prm;
    float *bm, *fm;
    int nm;
    ~Saved() {
      c->prm = prm;
      c->brms_map = bm;
      c->fdrive_map = fm;
      c->nmodes = nm;
      fill_prm(c);
      c->need_init = true;
    }
  } saved{c, c->prm, c->brms_map, c->fdrive_map, c->nmodes};
  c->prm.no_precession = 1;
  c->prm.method = LLGC_DP45;
  c->prm.brms[0] = c->prm.brms[1] = c->prm.brms[2] = 0.0;
  c->prm.cdrive_kind = LLGC_DRIVE_NONE;
  c->prm.fdrive_kind = LLGC_DRIVE_NONE;
  c->prm.cavity_mode = LLGC_CAVITY_ODE;
  c->prm.temperature = 0.0;   // relax runs cold
  if (!(c->prm.tol > 0)) c->prm.tol = 1e-6;
  c->brms_map = nullptr;
  c->fdrive_map = nullptr;
  c->nmodes = 0;
  fill_prm(c);
  c->need_init = true;
  const int nblk = n_pointwise_blocks(c);
  std::vector<double> part(2 * (size_t)nblk);
  int64_t acc = 0, rej = 0, evals = 0, blocks = 0;
  double prev = -1.0, mx2 = 0.0, last_err = 0.0, dt = 0.0;
  int r = LLGC_OK;
  while (acc < max_steps) {
    const int64_t nb = std::min<int64_t>(8, max_steps - acc);
    llgc_run_info bi{};
    if ((r = llgc_run(c, nb, 1e300, 0, nullptr, 0, nullptr, &bi))) break;
    acc += bi.accepted;
    rej += bi.rejected;
    evals += bi.rhs_evals;
    last_err = bi.last_err;
    dt = bi.dt;
    ++blocks;
    // torque of the current state (relaxation dynamics) into a k register
    // that the next attempt recomputes before reading
    if ((r = llgc_eval_rhs(c, c->yn, 0.0, 0.0, bi.t, c->kb[1], nullptr,
                           nullptr)))
      break;
    hipLaunchKernelGGL(k_torque_stats<kT>, dim3(nblk), dim3(kT), 0,
                       c->stream, c->P, c->kb[1], c->partials);
    if ((r = check_launch(c, "k_torque_stats"))) break;
    HIPCHK(c, hipMemcpyAsync(part.data(), c->partials,
                             sizeof(double) * part.size(),
                             hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    double s2 = 0.0;
    mx2 = 0.0;
    for (int b = 0; b < nblk; ++b) {
      s2 += part[2 * b];
      mx2 = std::max(mx2, part[2 * b + 1]);
    }
    const double mean2 = s2 / (c->nmag > 0 ? c->nmag : (double)c->N);
    if (torque_tol > 0) {
      if (std::sqrt(mx2) < torque_tol) break;
    } else if (prev >= 0.0 && mean2 >= prev) {
      break;
    }
    prev = mean2;
  }
  // time, amplitudes and step counts as before the relaxation
  Ctl h{};
  if (int q = ctl_read(c, &h, c->ctl)) return q;
  h.t = h0.t;
  h.dt = h0.dt;
  h.a_re = h.as_re[1] = h0.a_re;
  h.a_im = h.as_im[1] = h0.a_im;
  for (int k = 0; k < kMaxModes; ++k) {
    h.ma_re[k] = h.mas_re[1][k] = h0.ma_re[k];
    h.ma_im[k] = h.mas_im[1][k] = h0.ma_im[k];
  }
  h.accepted = h0.accepted;
  h.rejected = h0.rejected;
  h.mem_n = 0;
  if (int q = ctl_write(c, c->ctl, &h)) return q;
  if (max_torque) *max_torque = std::sqrt(mx2);
  if (info) {
    info->accepted = acc;
    info->rejected = rej;
    info->rhs_evals = evals;
    info->t = h0.t;
    info->dt = dt;
    info->last_err = last_err;
  }
  (void)blocks;
  return r;
}

int llgc_set_modes(llgc_ctx* c, int32_t n, const llgc_mode* modes) {
  if (!c) return LLGC_E_ARG;
  if (!c->have_params)
    return fail(c, LLGC_E_STATE, "set params before the modes");
  if (n < 0 || n > kMaxModes || (n > 0 && !modes))
    return fail(c, LLGC_E_ARG, "0..%d modes", kMaxModes);
  if (n > 0 && c->prm.cavity_mode != LLGC_CAVITY_ODE)
    return fail(c, LLGC_E_UNSUPPORTED,
                "the memory recursion is written for one mode");
  if (n > 0 && c->batch_plan)
    return fail(c, LLGC_E_UNSUPPORTED,
                "batched instances have a single cavity mode");
  bool any_map = false;
  for (int k = 0; k < n; ++k) {
    const llgc_mode& q = modes[k];
    if (!(q.kappa >= 0) || q.cdrive_kind < 0 || q.cdrive_kind > 2)
      return fail(c, LLGC_E_ARG, "mode %d: kappa >= 0, known drive kind", k);
    any_map = any_map || q.brms_map;
  }
  const size_t n3 = (size_t)3 * c->N;
  if (n > 0) {
    if (!c->modes_dev) HIPCHK(c, hipMalloc(&c->modes_dev, sizeof(Modes)));
    if (!c->mpart)
      HIPCHK(c, hipMalloc(&c->mpart, sizeof(double) * kMaxModes *
                                         c->npartials));
  }
  if (c->mode_maps) {
    HIPCHK(c, hipFree(c->mode_maps));
    c->mode_maps = nullptr;
  }
  Modes h{};
  h.n = n;
  if (any_map) {
    // the maps of the modes that have one, one 3 N block each
    int nmap = 0;
    for (int k = 0; k < n; ++k) nmap += modes[k].brms_map ? 1 : 0;
    HIPCHK(c, hipMalloc(&c->mode_maps, sizeof(float) * n3 * nmap));
    for (int k = 0, j = 0; k < n; ++k) {
      if (!modes[k].brms_map) continue;
      float* dst = c->mode_maps + n3 * j++;
      HIPCHK(c, hipMemcpyAsync(dst, modes[k].brms_map, sizeof(float) * n3,
                               hipMemcpyDeviceToDevice, c->stream));
      h.map[k] = dst;
    }
    h.any_map = 1;
  }
  for (int k = 0; k < n; ++k) {
    const llgc_mode& q = modes[k];
    for (int j = 0; j < 3; ++j) h.br[k][j] = q.brms[j];
    h.wc[k] = q.wc;
    h.kappa[k] = q.kappa;
    h.ckind[k] = q.cdrive_kind;
    h.camp[k] = q.cdrive_amp;
    h.cw[k] = q.cdrive_w;
    c->mode_h[k] = q;
    c->mode_h[k].brms_map = nullptr;   // borrowed only for this call
  }
  if (n > 0)
    HIPCHK(c, hipMemcpyAsync(c->modes_dev, &h, sizeof(Modes),
                             hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->nmodes = n;
  fill_prm(c);
  // amplitudes start at (x0 - i p0)/2 of each mode
  Ctl q{};
  if (int r = ctl_read(c, &q, c->ctl)) return r;
  for (int k = 0; k < kMaxModes; ++k) {
    const double ar = k < n ? 0.5 * modes[k].x0 : 0.0;
    const double ai = k < n ? -0.5 * modes[k].p0 : 0.0;
    q.ma_re[k] = q.mas_re[1][k] = ar;
    q.ma_im[k] = q.mas_im[1][k] = ai;
  }
  if (int r = ctl_write(c, c->ctl, &q)) return r;
  c->need_init = true;
  return LLGC_OK;
}

int llgc_set_mode_amplitudes(llgc_ctx* c, const double* a) {
  if (!c) return LLGC_E_ARG;
  if (!c->nmodes) return fail(c, LLGC_E_STATE, "no multimode cavity set");
  if (!a) return fail(c, LLGC_E_ARG, "amplitudes are NULL");
  Ctl q{};
  if (int r = ctl_read(c, &q, c->ctl)) return r;
  for (int k = 0; k < c->nmodes; ++k) {
    q.ma_re[k] = q.mas_re[1][k] = a[2 * k];
    q.ma_im[k] = q.mas_im[1][k] = a[2 * k + 1];
  }
  if (int r = ctl_write(c, c->ctl, &q)) return r;
  c->need_init = true;
  return LLGC_OK;
}

int llgc_get_mode_amplitudes(llgc_ctx* c, double* a) {
  if (!c) return LLGC_E_ARG;
  if (!c->nmodes) return fail(c, LLGC_E_STATE, "no multimode cavity set");
  if (!a) return fail(c, LLGC_E_ARG, "amplitudes are NULL");
  Ctl q{};
  if (int r = ctl_read(c, &q, c->ctl)) return r;
  for (int k = 0; k < c->nmodes; ++k) {
    a[2 * k] = q.ma_re[k];
    a[2 * k + 1] = q.ma_im[k];
  }
  return c->nmodes;
}

}  // extern "C" (reopened below)

namespace {

// Run set-up shared by llgc_run and the batched engine: control block,
// initial record, and for Dormand-Prince the first stage and the first
// attempt's start (k_begin), so that what follows is whole attempts.
struct RunPrep {
  long long acc0 = 0, rej0 = 0;
  int64_t nsteps = 0, cap = 0, evals = 0;
  bool rk4 = false, done = false;
};

int run_prepare(llgc_ctx* c, int64_t nsteps, double t_end, int32_t rec_every,
                double* rec, int64_t rec_cap, RunPrep* rp) {
  if (!c->have_params || !c->have_state)
    return fail(c, LLGC_E_STATE, "set params and state before running");
  if (rec_every > 0 && (!rec || rec_cap < 1))
    return fail(c, LLGC_E_ARG, "records requested without a buffer");
  rp->cap = rec_every > 0 ? rec_cap : 0;
  if (int r = ensure_rec(c, std::max<int64_t>(rp->cap, 1))) return r;
  Ctl h{};
  if (int r = ctl_read(c, &h, c->ctl)) return r;
  rp->acc0 = h.accepted;
  rp->rej0 = h.rejected;
  h.rec_every = rec_every > 0 ? rec_every : 0;
  h.rec_cap = (int)rp->cap;
  h.nrec = 0;
  h.status = 0;
  h.done = 0;
  h.accepted = 0;
  h.rejected = 0;
  h.cnt_xfwd = h.cnt_field = h.cnt_begin = h.cnt_rec = 0;
  h.emax_bits = 0;
  rp->rk4 = c->prm.method == LLGC_RK4;
  rp->evals = 0;
  if (rp->rk4) {
    h.dt = c->prm.dt;
    if (nsteps <= 0) nsteps = (int64_t)std::llround((t_end - h.t) / h.dt);
    rp->nsteps = std::max<int64_t>(nsteps, 0);
    h.t_end = 1e300;
    // the commit of step `nsteps` marks the run done
    h.max_accepted = rp->nsteps;
    h.done = rp->nsteps == 0 ? 1 : 0;
  } else {
    h.t_end = t_end;
    h.max_accepted = nsteps > 0 ? nsteps : ((long long)1 << 62);
    if (c->need_init) h.dt = c->prm.dt;
    h.dt = std::min(h.dt, t_end - h.t);
    h.done = (h.t >= t_end) ? 1 : 0;
    h.pending_accept = 0;
    if (!h.done && !c->need_init) {
      // current dt may differ from the one y2 was formed with
      h.as_re[2] = h.a_re + h.dt * 0.2 * h.ka_re[1];
      h.as_im[2] = h.a_im + h.dt * 0.2 * h.ka_im[1];
      for (int k = 0; k < c->nmodes; ++k) {
        h.mas_re[2][k] = h.ma_re[k] + h.dt * 0.2 * h.mka_re[1][k];
        h.mas_im[2][k] = h.ma_im[k] + h.dt * 0.2 * h.mka_im[1][k];
      }
    }
  }
  rp->done = h.done != 0;
  if (rp->rk4 && !rp->done) {
    // the steps read their base state from the scratch register (epi_rk4)
    HIPCHK(c, hipMemcpyAsync(c->yb[0], c->yn, sizeof(float) * 3 * c->N,
                             hipMemcpyDeviceToDevice, c->stream));
  }
  if (int r = ctl_write(c, c->ctl, &h)) return r;
  if (rp->cap > 0) {
    if (int r = launch_record(c)) return r;
  }
  if (!rp->rk4 && !rp->done) {
    if (c->need_init) {
      if (int r = rhs_stage(c, c->yn, c->ctl, 1, epi_eval(c->kb[0], nullptr),
                            0))
        return r;
      rp->evals = 1;
    }
    if (int r = launch_begin(c)) return r;
  }
  return LLGC_OK;
}

// Reads the outcome of a run back: records, info, totals, status.
int run_conclude(llgc_ctx* c, const RunPrep& rp, double* rec,
                 int64_t* n_rec, llgc_run_info* info) {
  c->need_init = false;
  Ctl e{};
  if (int q = ctl_read(c, &e, c->ctl)) return q;
  const int64_t evals = rp.rk4 ? 4 * e.accepted
                               : 6 * (e.accepted + e.rejected) + rp.evals;
  if (rp.cap > 0 && e.nrec > 0) {
    HIPCHK(c, hipMemcpy(rec, c->rec,
                        sizeof(double) * rec_width(c) * e.nrec,
                        hipMemcpyDeviceToHost));
  }
  if (rp.rk4 && e.status == ST_OK && e.accepted > 0) {
    // the last step's state is committed from the scratch register
    HIPCHK(c, hipMemcpyAsync(c->yn, c->yb[0], sizeof(float) * 3 * c->N,
                             hipMemcpyDeviceToDevice, c->stream));
  }
  if (n_rec) *n_rec = e.nrec;
  if (info) {
    info->accepted = e.accepted;
    info->rejected = e.rejected;
    info->rhs_evals = evals;
    info->t = e.t;
    info->dt = e.dt;
    info->last_err = e.last_err;
  }
  // keep totals across runs
  e.accepted += rp.acc0;
  e.rejected += rp.rej0;
  const int st = e.status;
  e.status = 0;
  if (int q = ctl_write(c, c->ctl, &e)) return q;
  if (st == ST_UNDERFLOW)
    return fail(c, LLGC_E_DT_UNDERFLOW, "time step fell below dt_min");
  if (st == ST_NONFINITE)
    return fail(c, LLGC_E_NONFINITE, "non-finite state or error estimate");
  return LLGC_OK;
}

}  // namespace

extern "C" {

int llgc_run(llgc_ctx* c, int64_t nsteps, double t_end, int32_t rec_every,
             double* rec, int64_t rec_cap, int64_t* n_rec,
             llgc_run_info* info) {
  if (!c) return LLGC_E_ARG;
  if (n_rec) *n_rec = 0;
  RunPrep rp;
  if (int r = run_prepare(c, nsteps, t_end, rec_every, rec, rec_cap, &rp))
    return r;
  int r = LLGC_OK;
  if (rp.rk4) {
    for (int64_t n = 0; n < rp.nsteps && !r; ++n) r = run_chunk(c, 1);
  } else if (!rp.done) {
    const int64_t max_attempts = 50000000;
    int64_t attempts = 0;
    // accepted steps still allowed: when fewer than a chunk remain, only
    // that many attempts are queued (launches past the end of a run would
    // exit at once on the done flag and only cost launch time)
    const int64_t cap = nsteps > 0 ? nsteps : INT64_MAX;
    int64_t accepted = 0;
    while (!r) {
      const int64_t rem = cap - accepted;
      if (rem <= 0) break;
      if (rem < kDpChunk) {
        r = chunk_direct(c, 0, (int)rem);
        attempts += rem;
      } else {
        r = run_chunk(c, 0);
        attempts += kDpChunk;
      }
      if (r) break;
      // accepted count and done flag of the control block
      struct {
        long long accepted;
        int done;
      } chk{};
      HIPCHK(c, hipMemcpyAsync(&chk.accepted, &c->ctl->accepted,
                               sizeof(long long), hipMemcpyDeviceToHost,
                               c->stream));
      HIPCHK(c, hipMemcpyAsync(&chk.done, &c->ctl->done, sizeof(int),
                               hipMemcpyDeviceToHost, c->stream));
      HIPCHK(c, hipStreamSynchronize(c->stream));
      accepted = chk.accepted;
      const int done = chk.done;
      if (done) break;
      if (attempts > max_attempts) {
        r = fail(c, LLGC_E_DT_UNDERFLOW, "attempt limit reached");
        break;
      }
    }
  }
  if (r) return r;
  return run_conclude(c, rp, rec, n_rec, info);
}

int llgc_step(llgc_ctx* c, llgc_run_info* info) {
  if (!c) return LLGC_E_ARG;
  return llgc_run(c, 1, 1e300, 0, nullptr, 0, nullptr, info);
}

}  // extern "C"

namespace {

// Control block of a right-hand-side evaluation: time and amplitude given;
// with a multimode cavity the amplitudes are the context's current ones.
int eval_ctl(llgc_ctx* c, double t, double are, double aim, Ctl* h) {
  if (c->nmodes) {
    Ctl cur{};
    if (int r = ctl_read(c, &cur, c->ctl)) return r;
    for (int k = 0; k < c->nmodes; ++k) {
      h->mas_re[1][k] = h->ma_re[k] = cur.ma_re[k];
      h->mas_im[1][k] = h->ma_im[k] = cur.ma_im[k];
    }
  }
  h->t = t;
  h->dt = c->prm.dt;   // enters only the thermal field's variance
  h->a_re = are;
  h->a_im = aim;
  h->as_re[1] = are;
  h->as_im[1] = aim;
  h->t_end = 1e300;
  return LLGC_OK;
}

// d alpha/dt of the evaluation: 2 doubles, or 2 per mode.
void eval_rates(const llgc_ctx* c, const Ctl& e, double* dadt) {
  if (!dadt) return;
  if (c->nmodes) {
    for (int k = 0; k < c->nmodes; ++k) {
      dadt[2 * k] = e.mka_re[1][k];
      dadt[2 * k + 1] = e.mka_im[1][k];
    }
    return;
  }
  dadt[0] = e.rhs_dadt_re;
  dadt[1] = e.rhs_dadt_im;
}

}  // namespace

extern "C" {

int llgc_eval_rhs(llgc_ctx* c, const float* m, double are, double aim,
                  double t, float* dmdt, float* beff, double* dadt) {
  if (!c) return LLGC_E_ARG;
  if (!c->have_params)
    return fail(c, LLGC_E_STATE, "set params before evaluating");
  if (!m || !dmdt) return fail(c, LLGC_E_ARG, "m and dmdt are required");
  Ctl h{};
  if (int r = eval_ctl(c, t, are, aim, &h)) return r;
  if (int r = ctl_write(c, c->ctl_eval, &h)) return r;
  if (int r = rhs_stage(c, m, c->ctl_eval, 1, epi_eval(dmdt, beff), 1))
    return r;
  Ctl e{};
  if (int r = ctl_read(c, &e, c->ctl_eval)) return r;
  eval_rates(c, e, dadt);
  return LLGC_OK;
}

}  // extern "C"

// ------------------------------------------- evaluation without allocation
// Device memory of llgc_eval_rhs_noalloc: its control block, partial sums
// and half spectrum live in this file-scope array instead of the context's
// buffers.  Each device holds one copy for the life of the process; host
// code reaches it only through the address hipGetSymbolAddress gives for the
// current device (the array's name is not a device address on the host).
namespace {
constexpr size_t kScratchBytes = (size_t)16 << 20;
}
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_scratch_mu;
std::map<int, unsigned char*> g_scratch_addr;   // device -> its copy

// Address of the current device's copy, looked up once per device.
int scratch_addr(llgc_ctx* c, int dev, unsigned char** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  auto it = g_scratch_addr.find(dev);
  if (it == g_scratch_addr.end()) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(c, LLGC_E_HIP, "hipGetSymbolAddress(scratch): %s",
                  hipGetErrorString(e));
    it = g_scratch_addr.emplace(dev, (unsigned char*)p).first;
  }
  *out = it->second;
  return LLGC_OK;
}

__global__ void k_zero4(float4* __restrict__ p, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Bytes of scratch an evaluation on this context needs: control block,
// partial sums, half spectrum (demag only).
size_t noalloc_bytes(const llgc_ctx* c, size_t* off_part, size_t* off_spec,
                     size_t* nspec) {
  *nspec = c->P.demag ? (size_t)c->Hx * c->nz * 3 * (c->ny + (c->ny & 1))
                      : 0;
  *off_part = align256(sizeof(Ctl));
  *off_spec = *off_part + align256(sizeof(double) * c->npartials);
  return *off_spec + sizeof(float2) * *nspec;
}

}  // namespace

extern "C" {

int llgc_eval_rhs_noalloc(llgc_ctx* c, const float* m, double are,
                          double aim, double t, float* dmdt, float* beff,
                          double* dadt) {
  if (!c) return LLGC_E_ARG;
  if (!c->have_params)
    return fail(c, LLGC_E_STATE, "set params before evaluating");
  if (!m || !dmdt) return fail(c, LLGC_E_ARG, "m and dmdt are required");
  int dev = -1;
  HIPCHK(c, hipGetDevice(&dev));
  if (dev != c->device)
    return fail(c, LLGC_E_ARG, "current device %d is not the context's (%d)",
                dev, c->device);
  size_t off_part, off_spec, nspec;
  const size_t need = noalloc_bytes(c, &off_part, &off_spec, &nspec);
  if (need > kScratchBytes)
    return fail(c, LLGC_E_UNSUPPORTED,
                "evaluation needs %zu bytes of static scratch; the limit is "
                "%zu (padded grid too large: use llgc_eval_rhs)",
                need, kScratchBytes);
  unsigned char* base = nullptr;
  if (int r = scratch_addr(c, dev, &base)) return r;
  Ctl* ctl = (Ctl*)base;
  double* part = (double*)(base + off_part);
  float2* spec = (float2*)(base + off_spec);
  Ctl h{};
  if (int r = eval_ctl(c, t, are, aim, &h)) return r;
  if (int r = ctl_write(c, ctl, &h)) return r;
  if (nspec > 0) {
    // the previous call's spectrum is cleared (the context's own spectrum
    // starts zeroed at creation)
    const size_t n4 = nspec / 2;   // nspec is even: rows padded to even
    hipLaunchKernelGGL(k_zero4, dim3((unsigned)std::min<size_t>(
                                    2048, (n4 + 255) / 256)),
                       dim3(256), 0, c->stream, (float4*)spec, n4);
    if (int r = check_launch(c, "k_zero4")) return r;
  }
  // the launches below take the scratch spectrum and partials in place of
  // the context's; no events (timing off for this call)
  struct Swap {
    llgc_ctx* c;
    float2* spec;
    double* part;
    bool timing;
    ~Swap() {
      c->spec = spec;
      c->partials = part;
      c->timing = timing;
    }
  } restore{c, c->spec, c->partials, c->timing};
  c->spec = spec;
  c->partials = part;
  c->timing = false;
  if (int r = rhs_stage(c, m, ctl, 1, epi_eval(dmdt, beff), 1)) return r;
  Ctl e{};
  if (int r = ctl_read(c, &e, ctl)) return r;
  eval_rates(c, e, dadt);
  return LLGC_OK;
}

int llgc_autotune(llgc_ctx* c, int32_t reps, int32_t* choice) {
  if (!c) return LLGC_E_ARG;
  if (c->batch_plan)
    return fail(c, LLGC_E_ARG, "batch-plan contexts keep their fixed plan");
  if (!c->have_params)
    return fail(c, LLGC_E_STATE, "set params before tuning");
  const auto key = std::make_tuple(c->nx, c->ny, c->nz, c->P.demag ? 1 : 0);
  const PlanShape s0 = plan_get(c);
  PlanShape best = s0;
  const bool timing = c->timing;
  c->timing = false;                     // keep tuning out of the timers
  struct Restore {
    llgc_ctx* c;
    bool t;
    ~Restore() { c->timing = t; }
  } restore{c, timing};
  auto undo = [&](int r) {
    plan_put(c, s0);
    plan_derive(c);
    return r;
  };
  if (reps <= 0) {
    std::lock_guard<std::mutex> lock(g_tuned_mu);
    auto it = g_tuned.find(key);
    if (it != g_tuned.end()) best = it->second;
  } else {
    // 1) FFT kind of each pass: two rounds over the candidate kinds with
    // the default shapes (the first round also brings the clocks up); each
    // kind keeps its faster round
    double tbest[16];
    for (double& v : tbest) v = 1e300;
    for (int round = 0; round < 2; ++round) {
      for (int k = 0; k < 16; ++k) {
        if (!plan_kind_ok(c, k)) continue;
        PlanShape sk = s0;
        sk.kind = k;
        if ((k & 8) && !(s0.kind & 8)) {
          plan_set_kind(c, k);
          sk.Rf = sk.Ri = x3_rows(c);
        }
        plan_put(c, sk);
        if (plan_derive(c)) continue;             // does not fit this grid
        double ms = 0.0;
        if (int r = time_rhs(c, reps, &ms)) return undo(r);
        tbest[k] = std::min(tbest[k], ms);
      }
    }
    int kb = s0.kind;
    for (int k = 0; k < 16; ++k)
      if (tbest[k] < tbest[kb]) kb = k;
    best.kind = kb;
    if ((kb & 8) && !(s0.kind & 8)) {
      plan_set_kind(c, kb);
      best.Rf = best.Ri = x3_rows(c);
    }
    // 2) tile shapes of the chosen kind, one parameter at a time: halve or
    // double the rows of the passes in LDS (2, 4 for the register ones) and
    // the spectral column slots; a change is kept when 2% faster
    int rf_max, ri_max, w_max;
    plan_put(c, best);
    plan_limits(c, &rf_max, &ri_max, &w_max);
    const int rcap = c->ny + (c->ny & 1);
    double tcur = tbest[kb];
    auto attempt = [&](PlanShape t) -> int {
      plan_put(c, t);
      if (plan_derive(c)) return LLGC_OK;
      double ms = 0.0;
      if (int r = time_rhs(c, reps, &ms)) return r;
      if (ms < 0.98 * tcur) {
        best = t;
        tcur = ms;
      }
      return LLGC_OK;
    };
    auto rows = [&](int r, int rmax, int* out) {
      int n = 0;
      for (int v : {r / 2, 2 * r}) {
        v &= ~1;
        if (v >= 2 && v <= std::min(rmax, std::max(2, rcap)) && v != r)
          out[n++] = v;
      }
      return n;
    };
    int cand[2];
    const PlanShape base = best;
    if (!(base.kind & 2)) {
      for (int i = 0, n = rows(base.Rf, rf_max, cand); i < n; ++i) {
        PlanShape t = best;
        t.Rf = cand[i];
        if (int r = attempt(t)) return undo(r);
      }
    } else if (sizeof(float2) * 3 * 2 * (size_t)c->Px <= 65536) {
      // the register forward pass keeps 3 (R/2) rows in LDS: R = 4 only
      // where that stays within the default 64 KB
      PlanShape t = best;
      t.Rwf = base.Rwf == 2 ? 4 : 2;
      if (int r = attempt(t)) return undo(r);
    }
    if (!(base.kind & 4)) {
      for (int i = 0, n = rows(base.Ri, ri_max, cand); i < n; ++i) {
        PlanShape t = best;
        t.Ri = cand[i];
        if (int r = attempt(t)) return undo(r);
      }
    } else {
      PlanShape t = best;
      t.Rw = base.Rw == 2 ? 4 : 2;
      if (int r = attempt(t)) return undo(r);
    }
    if (!(base.kind & 1)) {
      for (int v : {base.W / 2, 2 * base.W}) {
        if (v < 1 || v > w_max || v == base.W) continue;
        PlanShape t = best;
        t.W = v;
        if (int r = attempt(t)) return undo(r);
      }
    }
    std::lock_guard<std::mutex> lock(g_tuned_mu);
    g_tuned[key] = best;
  }
  plan_put(c, best);
  if (int r = plan_derive(c)) return undo(r);
  if (choice) *choice = best.kind;
  c->err.clear();
  return LLGC_OK;
}

int llgc_demag_kernel(llgc_ctx* c, float* out, int64_t cap, int32_t* dims) {
  if (!c) return LLGC_E_ARG;
  if (dims) {
    dims[0] = c->Px;
    dims[1] = c->Py;
    dims[2] = c->Hx;
    dims[3] = c->Hy;
  }
  if (!out) return LLGC_OK;
  const int nz = c->nz, ke = kentry(nz);
  const int64_t ne = (int64_t)c->Hx * c->Hy;
  const int64_t n = ne * 6 * nz;
  if (cap < n) return fail(c, LLGC_E_ARG, "need %lld floats", (long long)n);
  if (!c->kernel_built) return fail(c, LLGC_E_STATE, "no demag kernel");
  // the stored entries omit xz and yz at dz = 0 (zero): expand
  std::vector<float> packed((size_t)(ne * ke));
  HIPCHK(c, hipMemcpy(packed.data(), c->K, sizeof(float) * packed.size(),
                      hipMemcpyDeviceToHost));
  for (int64_t e = 0; e < ne; ++e)
    for (int comp = 0; comp < 6; ++comp)
      for (int dz = 0; dz < nz; ++dz)
        out[(e * 6 + comp) * nz + dz] =
            (comp >= 4 && dz == 0) ? 0.f
                                   : packed[(size_t)(e * ke +
                                                     kslot(comp, dz, nz))];
  return LLGC_OK;
}

int llgc_demag_tensor(llgc_ctx* c, double* out, int64_t cap) {
  if (!c) return LLGC_E_ARG;
  const int64_t n = (int64_t)6 * c->N;
  if (!out || cap < n) return fail(c, LLGC_E_ARG, "need %lld doubles",
                                   (long long)n);
  if (!c->tensor) return fail(c, LLGC_E_STATE, "no demag tensor");
  HIPCHK(c, hipStreamSynchronize(c->stream));
  HIPCHK(c, hipMemcpy(out, c->tensor, sizeof(double) * n,
                      hipMemcpyDeviceToHost));
  return LLGC_OK;
}

int llgc_set_timing(llgc_ctx* c, int32_t enable) {
  if (!c) return LLGC_E_ARG;
  c->timing = enable != 0;
  return LLGC_OK;
}

int llgc_set_timing_only(llgc_ctx* c, const char* kernel) {
  if (!c) return LLGC_E_ARG;
  c->timing_only = kernel ? kernel : "";
  return LLGC_OK;
}

int llgc_kernel_times(llgc_ctx* c, double* ms, int64_t* launches,
                      int32_t cap, char* names, int32_t names_cap,
                      int32_t reset) {
  if (!c) return LLGC_E_ARG;
  if (int r = timers_collect(c)) return r;
  std::string joined;
  int i = 0;
  for (auto& kv : c->timers) {
    if (i < cap) {
      if (ms) ms[i] = kv.second.ms;
      if (launches) launches[i] = kv.second.launches;
    }
    if (!joined.empty()) joined += ";";
    joined += kv.first;
    ++i;
  }
  if (names && names_cap > 0) {
    std::strncpy(names, joined.c_str(), names_cap - 1);
    names[names_cap - 1] = 0;
  }
  if (reset) c->timers.clear();
  return i;
}

int llgc_plan_info(const llgc_ctx* c, int32_t* info) {
  if (!c || !info) return LLGC_E_ARG;
  info[0] = c->Px;
  info[1] = c->Py;
  info[2] = c->Rf;
  info[3] = c->W;
  info[4] = kTX;
  info[5] = c->yhalf ? c->Tyh : c->Ty;
  info[6] = (int32_t)c->lds_f;
  info[7] = (int32_t)(c->yhalf ? c->lds_yh : c->lds_y);
  return LLGC_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- adjoint
namespace {

struct AdjBuf {
  std::vector<void*> owned;
  template <class T>
  int alloc(llgc_ctx* c, T** p, size_t n) {
    if (hipMalloc(p, sizeof(T) * std::max<size_t>(n, 1)) != hipSuccess)
      return fail(c, LLGC_E_OOM, "adjoint buffer of %zu bytes", sizeof(T) * n);
    owned.push_back(*p);
    return LLGC_OK;
  }
  ~AdjBuf() {
    for (void* p : owned) hipFree(p);
  }
};

__global__ void k_d2f(const double* __restrict__ a, float* __restrict__ b,
                      int n) {
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256)
    b[i] = (float)a[i];
}

// One RK4 step of the forward map whose stage inputs, stage fields and
// pre-normalisation norms are stored for the reverse sweep.
int rk4_step_stored(llgc_ctx* c, float* Yk /*4 x 3N*/, float* Bk /*4 x 3N*/,
                    float* nk /*N*/) {
  const size_t n3 = (size_t)3 * c->N;
  int r = 0;
  HIPCHK(c, hipMemcpyAsync(Yk, c->yn, n3 * 4, hipMemcpyDeviceToDevice,
                           c->stream));
  const bool fz = fusable(c);
  c->fused_run = fz;
  for (int s = 1; s <= 4 && !r; ++s) {
    Epi E = epi_rk4(c, s, true);
    E.bout = Bk + (size_t)(s - 1) * n3;
    if (s < 4) E.ynext = Yk + (size_t)s * n3;
    else E.nout = nk;
    r = rhs_stage(c, Yk + (size_t)(s - 1) * n3, c->ctl, s, E, 0,
                  !fz || s == 1, fz && s < 4);
  }
  c->fused_run = false;
  return r;
}

}  // namespace

extern "C" int llgc_adjoint(llgc_ctx* c, int64_t n_steps, double dt,
                            int64_t stride, int64_t n0, int64_t n1,
                            double* loss, float* grad_ms, float* grad_ku,
                            double* grad_brms, double* grad_eps) {
  if (!c) return LLGC_E_ARG;
  if (!c->have_params || !c->have_state)
    return fail(c, LLGC_E_STATE, "set params and state before llgc_adjoint");
  if (n_steps < 1 || n0 < 1 || n1 < n0 || n1 > n_steps || !(dt > 0))
    return fail(c, LLGC_E_ARG, "bad step count, window or dt");
  if (c->Px < 64)
    return fail(c, LLGC_E_UNSUPPORTED, "adjoint needs padded nx >= 64");
  if (c->prm.cavity_mode != LLGC_CAVITY_ODE)
    return fail(c, LLGC_E_UNSUPPORTED, "adjoint of the cavity ODE form only");
  if (c->brms_map)
    return fail(c, LLGC_E_UNSUPPORTED, "adjoint with a uniform B_rms only");
  if (c->fdrive_map)
    return fail(c, LLGC_E_UNSUPPORTED,
                "adjoint with a uniform field-drive direction only");
  if (c->nmodes)
    return fail(c, LLGC_E_UNSUPPORTED, "adjoint with a single cavity mode");
  if (c->prm.dmi_int != 0.0 || c->prm.dmi_bulk != 0.0)
    return fail(c, LLGC_E_UNSUPPORTED, "adjoint without DMI");
  if (c->prm.temperature > 0)
    return fail(c, LLGC_E_UNSUPPORTED, "adjoint without the thermal field");
  if (c->masked)
    return fail(c, LLGC_E_UNSUPPORTED, "adjoint without empty cells only");
  if (c->prm.ku2 != 0.0 || c->prm.no_precession)
    return fail(c, LLGC_E_UNSUPPORTED,
                "adjoint without Ku2 and with precession only");
  if (stride <= 0) stride = (int64_t)std::ceil(std::sqrt((double)n_steps));
  const int64_t S = stride;
  const int64_t nseg = (n_steps + S - 1) / S;
  const size_t N = c->N, n3 = 3 * N;
  // the adjoint runs the RK4 path with the given dt
  const llgc_params saved = c->prm;
  const Prm savedP = c->P;
  c->prm.method = LLGC_RK4;
  c->prm.dt = dt;
  fill_prm(c);
  struct Restore {
    llgc_ctx* c; llgc_params p; Prm P;
    ~Restore() { c->prm = p; c->P = P; }
  } restore{c, saved, savedP};
  AdjBuf B;
  float *ck = nullptr, *SY = nullptr, *SB = nullptr, *SN = nullptr;
  float *lam = nullptr, *hat = nullptr, *acc = nullptr, *lamK = nullptr,
        *lamB = nullptr, *lamM = nullptr;
  double *gms = nullptr, *gku = nullptr, *hist = nullptr, *part = nullptr;
  AdjCtl* A = nullptr;
  const int nlb = std::max(1, std::min(1024, (int)((N + 255) / 256)));
  int r;
  if ((r = B.alloc(c, &ck, n3 * nseg)) || (r = B.alloc(c, &SY, n3 * 4 * S + n3)) ||
      (r = B.alloc(c, &SB, n3 * 4 * S)) || (r = B.alloc(c, &SN, N * S)) ||
      (r = B.alloc(c, &lam, n3)) || (r = B.alloc(c, &hat, n3)) ||
      (r = B.alloc(c, &acc, n3)) || (r = B.alloc(c, &lamK, n3)) ||
      (r = B.alloc(c, &lamB, n3)) || (r = B.alloc(c, &lamM, n3)) ||
      (r = B.alloc(c, &gms, N)) || (r = B.alloc(c, &gku, N)) ||
      (r = B.alloc(c, &hist, (size_t)10 * S)) ||
      (r = B.alloc(c, &part, (size_t)7 * nlb)) || (r = B.alloc(c, &A, 1)))
    return r;
  // ---- forward with checkpoints and the windowed loss
  std::vector<double> cks(3 * nseg);
  Ctl h{};
  if ((r = ctl_read(c, &h, c->ctl))) return r;
  h.dt = dt;
  h.accepted = 0;
  h.max_accepted = 0;
  h.loss_n0 = n0;
  h.loss_n1 = n1;
  h.loss_acc = 0.0;
  h.ahist = nullptr;
  h.done = 0;
  h.status = 0;
  h.rec_every = 0;
  h.as_re[1] = h.a_re;
  h.as_im[1] = h.a_im;
  h.t_end = 1e300;
  if ((r = ctl_write(c, c->ctl, &h))) return r;
  for (int64_t j = 0; j < nseg; ++j) {
    Ctl q{};
    if ((r = ctl_read(c, &q, c->ctl))) return r;
    cks[3 * j] = q.t;
    cks[3 * j + 1] = q.a_re;
    cks[3 * j + 2] = q.a_im;
    HIPCHK(c, hipMemcpyAsync(ck + n3 * j, c->yn, n3 * 4,
                             hipMemcpyDeviceToDevice, c->stream));
    const int64_t Sj = std::min(S, n_steps - j * S);
    const bool fz = fusable(c);
    c->fused_run = fz;
    for (int64_t k = 0; k < Sj && !r; ++k)
      for (int s = 1; s <= 4 && !r; ++s)
        r = rhs_stage(c, rk4_input(c, s, true), c->ctl, s,
                      epi_rk4(c, s, true), 0, !fz || s == 1, fz && s < 4);
    c->fused_run = false;
    if (r) return r;
  }
  Ctl fin{};
  if ((r = ctl_read(c, &fin, c->ctl))) return r;
  if (fin.status) return fail(c, LLGC_E_NONFINITE, "non-finite forward state");
  const double Lval = fin.loss_acc / (double)(n1 - n0 + 1);
  // final state saved to restore after the sweep
  float* mfin = nullptr;
  if ((r = B.alloc(c, &mfin, n3))) return r;
  HIPCHK(c, hipMemcpyAsync(mfin, c->yn, n3 * 4, hipMemcpyDeviceToDevice,
                           c->stream));
  // ---- reverse sweep
  HIPCHK(c, hipMemsetAsync(lam, 0, n3 * 4, c->stream));
  HIPCHK(c, hipMemsetAsync(gms, 0, N * 8, c->stream));
  HIPCHK(c, hipMemsetAsync(gku, 0, N * 8, c->stream));
  AdjCtl a0{};
  a0.loss_scale = 1.0 / (double)(n1 - n0 + 1);
  HIPCHK(c, hipMemcpyAsync(A, &a0, sizeof(AdjCtl), hipMemcpyHostToDevice,
                           c->stream));
  // unit-weight parameters for the demag pipeline applied to lamB
  Prm Pu = c->P;
  Pu.ms = 1.f;
  Pu.ms_map = nullptr;
  Pu.brms_map = nullptr;
  Pu.brx = Pu.bry = Pu.brz = 0.f;
  Pu.brxd = Pu.bryd = Pu.brzd = 0.0;
  Ctl he{};
  he.t_end = 1e300;
  if ((r = ctl_write(c, c->ctl_eval, &he))) return r;
  const int R = c->Rw;
  const dim3 fg = xgrid(c, R), fb(64 * 3 * (R / 2));
  const size_t flds = c->P.demag ? sizeof(float) * 3 * R * c->nx : 0;
  const double cs[5] = {0.0, 0.0, 0.5, 0.5, 1.0};
  for (int64_t j = nseg - 1; j >= 0 && !r; --j) {
    const int64_t Sj = std::min(S, n_steps - j * S);
    // restore the checkpoint and recompute the segment with storage
    HIPCHK(c, hipMemcpyAsync(c->yn, ck + n3 * j, n3 * 4,
                             hipMemcpyDeviceToDevice, c->stream));
    Ctl q{};
    if ((r = ctl_read(c, &q, c->ctl))) return r;
    q.t = cks[3 * j];
    q.a_re = cks[3 * j + 1];
    q.a_im = cks[3 * j + 2];
    q.as_re[1] = q.a_re;
    q.as_im[1] = q.a_im;
    q.accepted = 0;
    q.loss_n0 = q.loss_n1 = 0;
    q.ahist = hist;
    q.dt = dt;
    if ((r = ctl_write(c, c->ctl, &q))) return r;
    for (int64_t k = 0; k < Sj && !r; ++k)
      r = rk4_step_stored(c, SY + n3 * 4 * k, SB + n3 * 4 * k, SN + N * k);
    if (r) return r;
    HIPCHK(c, hipMemcpyAsync(SY + n3 * 4 * Sj, c->yn, n3 * 4,
                             hipMemcpyDeviceToDevice, c->stream));
    for (int64_t k = Sj - 1; k >= 0 && !r; --k) {
      const int64_t n = j * S + k + 1;
      const double tn = cks[3 * j] + (double)k * dt;
      const float* m_end = SY + n3 * 4 * (k + 1);
      hipLaunchKernelGGL(k_adj_begin, dim3(nlb), dim3(256), 0, c->stream,
                         (int)N, m_end, SN + N * k, lam, hat, acc, lamK,
                         (float)(dt / 6.0));
      hipLaunchKernelGGL(k_adj_begin_scalar, dim3(1), dim3(64), 0, c->stream,
                         A, hist + 10 * k + 8, (n >= n0 && n <= n1) ? 1 : 0,
                         dt / 6.0);
      for (int s = 4; s >= 1 && !r; --s) {
        const float* Y = SY + n3 * (4 * k + (s - 1));
        const float* Bs = SB + n3 * (4 * k + (s - 1));
        const double cK = (s == 4 || s == 3) ? dt / 3.0 : (s == 2 ? dt / 6.0 : 0.0);
        const double cY = s == 4 ? dt : (s > 1 ? 0.5 * dt : 0.0);
        hipLaunchKernelGGL(k_vjp_local, dim3(nlb), dim3(256), 0, c->stream,
                           c->P, Y, Bs, lamK, A, lamB, lamM, gms, gku, part);
        if (c->P.demag) {
          Prm keep = c->P;
          c->P = Pu;
          r = launch_xfwd(c, lamB, c->ctl_eval, 1, 1);
          if (!r) r = launch_yspec(c, c->ctl_eval, 1, 1);
          c->P = keep;
          if (r) break;
        }
#define LLGC_VF_ARGS c->P, Y, c->spec, lamB, lamM, gms, acc, hat, lamK, \
                     (float)cK, (float)cY, R, c->tw, c->logTw
        switch (c->Px) {
          case 64: hipLaunchKernelGGL((k_vjp_field_w<1>), fg, fb, flds, c->stream, LLGC_VF_ARGS); break;
          case 128: hipLaunchKernelGGL((k_vjp_field_w<2>), fg, fb, flds, c->stream, LLGC_VF_ARGS); break;
          case 256: hipLaunchKernelGGL((k_vjp_field_w<4>), fg, fb, flds, c->stream, LLGC_VF_ARGS); break;
          case 512: hipLaunchKernelGGL((k_vjp_field_w<8>), fg, fb, flds, c->stream, LLGC_VF_ARGS); break;
          case 1024: hipLaunchKernelGGL((k_vjp_field_w<16>), fg, fb, flds, c->stream, LLGC_VF_ARGS); break;
          default: hipLaunchKernelGGL((k_vjp_field_w<32>), fg, fb, flds, c->stream, LLGC_VF_ARGS); break;
        }
#undef LLGC_VF_ARGS
        hipLaunchKernelGGL(k_vjp_scalar, dim3(1), dim3(256), 0, c->stream,
                           c->P, A, part, nlb, hist + 10 * k + 2 * (s - 1),
                           tn + cs[s] * dt, cK, cY);
        r = check_launch(c, "adjoint stage");
      }
      std::swap(lam, acc);
      hipLaunchKernelGGL(k_adj_end_scalar, dim3(1), dim3(64), 0, c->stream, A);
    }
  }
  if (r) return r;
  // outputs; the state is left at the end of the forward run
  HIPCHK(c, hipMemcpyAsync(c->yn, mfin, n3 * 4, hipMemcpyDeviceToDevice,
                           c->stream));
  fin.ahist = nullptr;
  fin.loss_n0 = fin.loss_n1 = 0;
  fin.accepted = 0;
  if ((r = ctl_write(c, c->ctl, &fin))) return r;
  if (grad_ms)
    hipLaunchKernelGGL(k_d2f, dim3(nlb), dim3(256), 0, c->stream, gms,
                       grad_ms, (int)N);
  if (grad_ku)
    hipLaunchKernelGGL(k_d2f, dim3(nlb), dim3(256), 0, c->stream, gku,
                       grad_ku, (int)N);
  AdjCtl af{};
  HIPCHK(c, hipMemcpyAsync(&af, A, sizeof(AdjCtl), hipMemcpyDeviceToHost,
                           c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (loss) *loss = Lval;
  if (grad_brms)
    for (int k = 0; k < 3; ++k) grad_brms[k] = af.g_brms[k];
  if (grad_eps) *grad_eps = af.g_eps0;
  c->need_init = true;
  return check_launch(c, "llgc_adjoint");
}

#include "llgc_batch_api.hip"
