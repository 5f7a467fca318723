// Host side of the batched engine (part of the llgc_api translation unit).
// Instances are ordinary contexts created with the batch plan; a run
// prepares each one exactly as llgc_run does, then drives all of them with
// one launch per kernel type and stage over a work-item table, and rebuilds
// the tables without the instances that have finished.

struct llgc_batch {
  int n = 0;
  std::vector<llgc_ctx*> inst;
  hipStream_t stream = nullptr;
  BInst* dI = nullptr;
  int2 *it_x = nullptr, *it_y = nullptr, *it_b = nullptr;
  int* act = nullptr;
  int* flags = nullptr;        // [0]: finished count, [1 + k]: done flag k
  int n_x = 0, n_y = 0, n_b = 0, n_act = 0;
  bool any_map = false;   // some instance has a per-cell B_rms map
  size_t cap_x = 0, cap_y = 0, cap_b = 0;   // work-table capacities
  size_t lds_x = 0, lds_f = 0, lds_y = 0;
  std::string err;
  // HIP graph of one round of attempts over the current work tables
  bool graphs = true;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
};

namespace {

int bfail(llgc_batch* b, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  b->err = buf;
  return code;
}

#define BHIPCHK(b, call)                                                    \
  do {                                                                      \
    hipError_t e_ = (call);                                                 \
    if (e_ != hipSuccess)                                                   \
      return bfail(b, LLGC_E_HIP, "%s failed: %s", #call,                   \
                   hipGetErrorString(e_));                                  \
  } while (0)

int b_tiles(const llgc_ctx* c) { return (int)xgrid(c, c->Rf).x; }
// spectral workgroups: column slots (kx = 0 and Px/2 share slot 0) per W
int b_yblocks(const llgc_ctx* c) {
  return c->P.demag ? (c->Px / 2 + c->W - 1) / c->W : 1;
}

void bgraph_release(llgc_batch* b) {
  if (b->gexec) hipGraphExecDestroy(b->gexec);
  if (b->graph) hipGraphDestroy(b->graph);
  b->gexec = nullptr;
  b->graph = nullptr;
}

BInst make_binst(llgc_ctx* c, bool rk4) {
  BInst B{};
  B.P = c->P;
  B.ctl = c->ctl;
  B.tw = c->tw;
  B.logTw = c->logTw;
  B.R = c->Rf;
  B.W = c->W;
  B.nf = b_tiles(c);
  B.nbeg = n_pointwise_blocks(c);
  // the operands launch_begin passes
  B.yn = c->yn;
  B.k1 = c->kb[0];
  B.y7 = c->yb[1];
  B.k7 = c->kb[6];
  B.y2 = c->yb[0];
  B.spec = c->spec;
  B.K = c->K;
  B.partials = c->partials;
  B.rec = c->rec;
  for (int s = 1; s < kMaxStages; ++s) {
    if (rk4 && s <= 4) {
      B.ys[s] = rk4_input(c, s);
      B.E[s] = epi_rk4(c, s);
    } else if (!rk4 && s >= 2) {
      B.ys[s] = c->yb[s % 2];
      B.E[s] = epi_dp(c, s);
    }
  }
  return B;
}

// Work tables of the instances marked active.
int batch_tables(llgc_batch* b, const std::vector<char>& active) {
  std::vector<int2> ix, iy, ib;
  std::vector<int> act;
  for (int k = 0; k < b->n; ++k) {
    if (!active[k]) continue;
    const llgc_ctx* c = b->inst[k];
    for (int t = 0, m = b_tiles(c); t < m; ++t) ix.push_back(make_int2(k, t));
    for (int t = 0, m = b_yblocks(c); t < m; ++t) iy.push_back(make_int2(k, t));
    for (int t = 0, m = n_pointwise_blocks(c); t < m; ++t)
      ib.push_back(make_int2(k, t));
    act.push_back(k);
  }
  b->n_x = (int)ix.size();
  b->n_y = (int)iy.size();
  b->n_b = (int)ib.size();
  b->n_act = (int)act.size();
  bgraph_release(b);                 // launch sizes change with the tables
  if (b->n_act == 0) return LLGC_OK;
  if (ix.size() > b->cap_x || iy.size() > b->cap_y || ib.size() > b->cap_b)
    return bfail(b, LLGC_E_STATE, "work tables exceed their allocation");
  BHIPCHK(b, hipMemcpy(b->it_x, ix.data(), ix.size() * sizeof(int2),
                       hipMemcpyHostToDevice));
  BHIPCHK(b, hipMemcpy(b->it_y, iy.data(), iy.size() * sizeof(int2),
                       hipMemcpyHostToDevice));
  BHIPCHK(b, hipMemcpy(b->it_b, ib.data(), ib.size() * sizeof(int2),
                       hipMemcpyHostToDevice));
  BHIPCHK(b, hipMemcpy(b->act, act.data(), act.size() * sizeof(int),
                       hipMemcpyHostToDevice));
  return LLGC_OK;
}

// One stage of every active instance.
int batch_stage(llgc_batch* b, int stage) {
  hipLaunchKernelGGL(kb_xfwd, dim3(b->n_x), dim3(kBXT), b->lds_x, b->stream,
                     b->dI, b->it_x, stage);
  if (b->any_map)
    hipLaunchKernelGGL(kb_coupling, dim3(b->n_x), dim3(256), 0, b->stream,
                       b->dI, b->it_x, stage);
  hipLaunchKernelGGL(kb_yspec, dim3(b->n_y), dim3(kBYT), b->lds_y, b->stream,
                     b->dI, b->it_y, stage, 0);
  hipLaunchKernelGGL(kb_xfield, dim3(b->n_x), dim3(kBXT), b->lds_f,
                     b->stream, b->dI, b->it_x, stage);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess)
    return bfail(b, LLGC_E_HIP, "batched stage launch failed: %s",
                 hipGetErrorString(e));
  return LLGC_OK;
}

constexpr int kBatchRound = 8;   // attempts per host check

// One round of attempts for every active instance, issued on b->stream.
int batch_round_direct(llgc_batch* b, bool rk4) {
  int r = LLGC_OK;
  for (int q = 0; q < kBatchRound && !r; ++q) {
    if (rk4) {
      for (int s = 1; s <= 4 && !r; ++s) r = batch_stage(b, s);
      if (!r)
        hipLaunchKernelGGL(kb_finish_step, dim3(b->n_act), dim3(256), 0,
                           b->stream, b->dI, b->act, 2, b->flags);
    } else {
      for (int s = 2; s <= 7 && !r; ++s) r = batch_stage(b, s);
      if (!r) {
        hipLaunchKernelGGL(kb_finish_step, dim3(b->n_act), dim3(256), 0,
                           b->stream, b->dI, b->act, 3, b->flags);
        hipLaunchKernelGGL(kb_begin, dim3(b->n_b), dim3(kBPT), 0,
                           b->stream, b->dI, b->it_b);
      }
    }
  }
  if (!r) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess)
      r = bfail(b, LLGC_E_HIP, "batched launch failed: %s",
                hipGetErrorString(e));
  }
  return r;
}

// The round replayed from a HIP graph (kernel nodes only), captured once per
// set of work tables on a private stream and launched on b->stream.
int batch_round(llgc_batch* b, bool rk4) {
  if (!b->graphs) return batch_round_direct(b, rk4);
  if (!b->gexec) {
    if (!b->cap_stream)
      BHIPCHK(b, hipStreamCreateWithFlags(&b->cap_stream,
                                          hipStreamNonBlocking));
    hipStream_t user = b->stream;
    b->stream = b->cap_stream;
    if (hipStreamBeginCapture(b->cap_stream,
                              hipStreamCaptureModeThreadLocal) != hipSuccess) {
      // capture unavailable: this batch launches directly from now on
      b->stream = user;
      (void)hipGetLastError();
      b->graphs = false;
      return batch_round_direct(b, rk4);
    }
    int r = batch_round_direct(b, rk4);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(b->cap_stream, &g);
    b->stream = user;
    if (!r && e != hipSuccess)
      r = bfail(b, LLGC_E_HIP, "hipStreamEndCapture: %s",
                hipGetErrorString(e));
    if (!r && hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0) !=
                  hipSuccess) {
      b->gexec = nullptr;
      r = bfail(b, LLGC_E_HIP, "hipGraphInstantiate failed");
    }
    if (r) {
      if (g) hipGraphDestroy(g);
      (void)hipGetLastError();
      return r;
    }
    b->graph = g;
  }
  BHIPCHK(b, hipGraphLaunch(b->gexec, b->stream));
  return LLGC_OK;
}

}  // namespace

extern "C" {

int llgc_batch_create(const llgc_grid* grids, int32_t n, void* stream,
                      llgc_batch** out) {
  if (!grids || !out || n < 1) return LLGC_E_ARG;
  *out = nullptr;
  llgc_batch* b = new llgc_batch();
  b->n = n;
  b->stream = (hipStream_t)stream;
  b->graphs = getenv("LLGC_NO_GRAPHS") == nullptr;
  b->inst.assign(n, nullptr);
  size_t cx = 0, cy = 0, cb = 0;
  for (int k = 0; k < n; ++k) {
    int r = llgc_create_ex(&grids[k], stream, LLGC_PLAN_BATCH, &b->inst[k]);
    if (r) {
      llgc_batch_destroy(b);
      return r;
    }
    const llgc_ctx* c = b->inst[k];
    cx += b_tiles(c);
    cy += (c->Px / 2 + c->W - 1) / c->W;   // demag may be set later
    cb += n_pointwise_blocks(c);
    b->lds_x = std::max(b->lds_x, c->lds_f);
    b->lds_f = std::max(b->lds_f, c->lds_i);
    b->lds_y = std::max(b->lds_y, c->lds_y);
  }
  raise_lds_limit((const void*)kb_yspec, b->lds_y);
  raise_lds_limit((const void*)kb_xfwd, b->lds_x);
  raise_lds_limit((const void*)kb_xfield, b->lds_f);
  b->cap_x = cx;
  b->cap_y = cy;
  b->cap_b = cb;
  bool ok = hipMalloc(&b->dI, sizeof(BInst) * n) == hipSuccess &&
            hipMalloc(&b->it_x, sizeof(int2) * cx) == hipSuccess &&
            hipMalloc(&b->it_y, sizeof(int2) * cy) == hipSuccess &&
            hipMalloc(&b->it_b, sizeof(int2) * cb) == hipSuccess &&
            hipMalloc(&b->act, sizeof(int) * n) == hipSuccess &&
            hipMalloc(&b->flags, sizeof(int) * (n + 1)) == hipSuccess;
  if (!ok) {
    llgc_batch_destroy(b);
    return LLGC_E_OOM;
  }
  *out = b;
  return LLGC_OK;
}

int llgc_batch_destroy(llgc_batch* b) {
  if (!b) return LLGC_OK;
  bgraph_release(b);
  if (b->cap_stream) hipStreamDestroy(b->cap_stream);
  for (auto* c : b->inst) llgc_destroy(c);
  hipFree(b->dI);
  hipFree(b->it_x);
  hipFree(b->it_y);
  hipFree(b->it_b);
  hipFree(b->act);
  hipFree(b->flags);
  delete b;
  return LLGC_OK;
}

const char* llgc_batch_last_error(const llgc_batch* b) {
  return b ? b->err.c_str() : "null batch";
}

llgc_ctx* llgc_batch_instance(llgc_batch* b, int32_t k) {
  if (!b || k < 0 || k >= b->n) return nullptr;
  return b->inst[k];
}

int llgc_batch_run(llgc_batch* b, int64_t nsteps, double t_end,
                   int32_t rec_every, double* rec, int64_t rec_cap,
                   int64_t* n_rec, llgc_run_info* info, int32_t* status) {
  if (!b) return LLGC_E_ARG;
  const int n = b->n;
  if (rec_every > 0 && (!rec || rec_cap < 1))
    return bfail(b, LLGC_E_ARG, "records requested without a buffer");
  for (int k = 0; k < n; ++k) {
    const llgc_ctx* c = b->inst[k];
    if (!c->have_params || !c->have_state)
      return bfail(b, LLGC_E_STATE, "instance %d: set params and state "
                   "before running", k);
    if (c->prm.method != b->inst[0]->prm.method)
      return bfail(b, LLGC_E_ARG, "instances use different methods");
    if (c->nmodes)
      return bfail(b, LLGC_E_UNSUPPORTED,
                   "instance %d: batched instances have one cavity mode", k);
  }
  if (n_rec)
    for (int k = 0; k < n; ++k) n_rec[k] = 0;
  const bool rk4 = b->inst[0]->prm.method == LLGC_RK4;
  // per-instance set-up, as llgc_run
  std::vector<RunPrep> rp(n);
  std::vector<char> active(n, 0);
  int ndone0 = 0;
  for (int k = 0; k < n; ++k) {
    llgc_ctx* c = b->inst[k];
    double* rk = rec_every > 0 ? rec + (size_t)6 * rec_cap * k : nullptr;
    if (int r = run_prepare(c, nsteps, t_end, rec_every, rk, rec_cap, &rp[k]))
      return bfail(b, r, "instance %d: %s", k, c->err.c_str());
    active[k] = rp[k].done ? 0 : 1;
    ndone0 += rp[k].done ? 1 : 0;
  }
  std::vector<BInst> hI(n);
  b->any_map = false;
  for (int k = 0; k < n; ++k) {
    hI[k] = make_binst(b->inst[k], rk4);
    if (b->inst[k]->brms_map) b->any_map = true;
  }
  BHIPCHK(b, hipMemcpyAsync(b->dI, hI.data(), sizeof(BInst) * n,
                            hipMemcpyHostToDevice, b->stream));
  BHIPCHK(b, hipMemcpyAsync(b->flags, &ndone0, sizeof(int),
                            hipMemcpyHostToDevice, b->stream));
  BHIPCHK(b, hipStreamSynchronize(b->stream));
  if (int r = batch_tables(b, active)) return r;
  int r = LLGC_OK;
  int ndone = ndone0, ndone_tables = ndone0;
  const int64_t max_rounds = 50000000 / kBatchRound;
  // a graph from an earlier run may hold the other method's launches
  bgraph_release(b);
  for (int64_t round = 0; ndone < n && !r; ++round) {
    r = batch_round(b, rk4);
    if (r) break;
    BHIPCHK(b, hipMemcpyAsync(&ndone, b->flags, sizeof(int),
                              hipMemcpyDeviceToHost, b->stream));
    BHIPCHK(b, hipStreamSynchronize(b->stream));
    if (ndone >= n) break;
    if (round >= max_rounds) {
      r = bfail(b, LLGC_E_DT_UNDERFLOW, "attempt limit reached");
      break;
    }
    // retire finished instances once enough of them have dropped out
    if (ndone - ndone_tables >= std::max(1, b->n_act / 8)) {
      hipLaunchKernelGGL(kb_done_flags, dim3((n + 255) / 256), dim3(256), 0,
                         b->stream, b->dI, n, b->flags + 1);
      std::vector<int> fl(n);
      BHIPCHK(b, hipMemcpyAsync(fl.data(), b->flags + 1, sizeof(int) * n,
                                hipMemcpyDeviceToHost, b->stream));
      BHIPCHK(b, hipStreamSynchronize(b->stream));
      for (int k = 0; k < n; ++k) active[k] = fl[k] ? 0 : 1;
      if ((r = batch_tables(b, active))) break;
      ndone_tables = ndone;
    }
  }
  if (r) return r;
  // per-instance outcome, as llgc_run
  int first = LLGC_OK;
  for (int k = 0; k < n; ++k) {
    llgc_ctx* c = b->inst[k];
    double* rk = rec_every > 0 ? rec + (size_t)6 * rec_cap * k : nullptr;
    const int q = run_conclude(c, rp[k], rk, n_rec ? n_rec + k : nullptr,
                               info ? info + k : nullptr);
    if (status) status[k] = q;
    if (q && first == LLGC_OK) {
      first = q;
      bfail(b, q, "instance %d: %s", k, c->err.c_str());
    }
  }
  return first;
}

}  // extern "C"
