/*
 * llgc -- cavity-coupled Landau-Lifshitz-Gilbert integrator for MI355X.
 *
 * Plain C ABI over the HIP library.  Every call returns a status code
 * (LLGC_OK or a negative LLGC_E_* value) and never throws; the message of
 * the last failure on a context is returned by llgc_last_error().
 *
 * The problem follows the paper's statement of it (arXiv 2410.00966):
 *   - finite-difference cells with a unit vector m_i at each cell centre and
 *     the LLG equation in Landau-Lifshitz form with Gilbert damping,
 *     Eq. (llg);
 *   - effective field = Zeeman + exchange + uniaxial anisotropy +
 *     demagnetisation (the field contributions listed after Eq. (llg)) +
 *     the cavity field B_rms (alpha + alpha^*) of the mean-field equations
 *     (eqmotionspinclasical)/(eqmotionaclasical), used in both the
 *     precession and the damping term;
 *   - one damped cavity mode, Eq. (eqmotionaclasical) with
 *     omega_c -> omega_c - i kappa:
 *       d alpha/dt = -(i wc + kappa) alpha
 *                    + i (V_c/hbar) sum_i Ms_i m_i . B_rms  - i eps(t).
 *     The cavity parameters mirror the paper's script additions B_rms, Wc,
 *     Kappa, X0 = 2 Re alpha_0, P0 = -2 Im alpha_0 and HBAR (section
 *     "Workflow in Mumax3-cQED").
 *
 * Units are SI.  Magnetisation arrays are float32 structure-of-arrays
 * m[c][z][y][x] (x fastest, c = component), N = nx*ny*nz cells per
 * component plane, in device memory.  Scalars and the cavity amplitude are
 * float64.  All device work of a context runs on the HIP stream given at
 * creation; calls that return host values synchronise that stream only.
 * One host thread per context.
 */
#ifndef LLGC_H
#define LLGC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct llgc_ctx llgc_ctx;

enum {
  LLGC_OK = 0,
  LLGC_E_ARG = -1,          /* invalid argument (null pointer, bad size)   */
  LLGC_E_OOM = -2,          /* device allocation failed                    */
  LLGC_E_HIP = -3,          /* a HIP runtime call failed                   */
  LLGC_E_NONFINITE = -4,    /* non-finite state or error estimate          */
  LLGC_E_DT_UNDERFLOW = -5, /* adaptive step fell below dt_min             */
  LLGC_E_STATE = -6,        /* call out of order (no params / no state)    */
  LLGC_E_UNSUPPORTED = -7   /* grid or option outside what is implemented  */
};

enum { LLGC_RK4 = 0, LLGC_DP45 = 1 };
/* Cavity treatment.  ODE: alpha is part of the integrated state, advanced
 * by the same Runge-Kutta scheme as m (default).  MEMORY: the paper's own
 * scheme with the cavity integrated out (section "Adapting the memory
 * term"): the cavity field B_rms Gamma_n is held over step n and Gamma_n
 * follows the rectangle-rule recursion Eqs. (Sdiscrete), (Cdiscrete),
 * (gammadiscretefinal) on the coupling sum of the step-start state, first
 * order in dt.  Evaluated in the equivalent amplitude form
 * alpha_n = e^{-(i wc + kappa) dt} alpha_{n-1} + i (V_c/hbar) F_n dt
 * (alpha_0 from the state; Gamma_n = 2 Re alpha_n), which needs no
 * e^{kappa t} factors.  RK4 only, no cavity drive; the amplitude reported
 * after step n is e^{-(i wc + kappa) dt} alpha_n. */
enum { LLGC_CAVITY_ODE = 0, LLGC_CAVITY_MEMORY = 1 };
enum { LLGC_DRIVE_NONE = 0, LLGC_DRIVE_SINC = 1, LLGC_DRIVE_CW = 2 };

/* Grid of orthorhombic cells (section "The LLG equation in Mumax3").
 * 1 <= nx, ny; 1 <= nz <= 4; cell sizes in metres. */
typedef struct {
  int32_t nx, ny, nz;
  double dx, dy, dz;
} llgc_grid;

/* Material, field, cavity and integrator parameters.
 * Field drive: B_ext(t) = bext + fdrive_amp * f(t) * fdrive_dir, or with
 * fdrive_map the per-cell vector in place of fdrive_dir.
 * Maps (ms_map, ku1_map) are device pointers to N float32 values in
 * [z][y][x] order, or NULL for the uniform scalar; they are copied by
 * llgc_set_params, so the caller keeps ownership.
 * Field drive: B_ext(t) = bext + fdrive_amp * f(t) * fdrive_dir.
 * Cavity drive: d alpha/dt gains -i * cdrive_amp * f(t).
 * f(t) = sinc(w t) (with sinc(0) = 1) or cos(w t), chosen by *_kind.
 * gamma, hbar, mu0 <= 0 select the defaults 1.7595e11 rad/(s T),
 * 1.05457182e-34 J s and 4 pi 1e-7 T m/A. */
typedef struct {
  double ms;               /* A/m, used when ms_map == NULL              */
  const float *ms_map;     /* A/m per cell (device, N float32, copied), or
                              NULL.  Cells with 0 are outside the geometry:
                              m = 0 there, exchange omits them as it omits
                              cells beyond the grid, records average m over
                              the magnetic cells.  Values must be finite and
                              >= 0 with one magnetic cell at least. */
  double aex;              /* J/m, exchange stiffness                   */
  double alpha;            /* Gilbert damping                           */
  double ku1;              /* J/m^3, used when ku1_map == NULL          */
  const float *ku1_map;
  double anis_u[3];        /* uniaxial axis (normalised internally)     */
  double bext[3];          /* T                                         */
  int32_t fdrive_kind;
  double fdrive_amp, fdrive_w; /* T, rad/s                              */
  double fdrive_dir[3];
  int32_t enable_demag;    /* 0: no demagnetising field                 */
  double brms[3];          /* T, uniform vacuum field of the mode       */
  double wc, kappa;        /* rad/s                                     */
  double x0, p0;           /* initial 2 Re alpha, -2 Im alpha           */
  int32_t cdrive_kind;
  double cdrive_amp, cdrive_w; /* rad/s, rad/s                          */
  double gamma, hbar, mu0;
  int32_t method;          /* LLGC_RK4 (fixed dt) or LLGC_DP45 (adaptive) */
  double dt;               /* s: fixed step, or first trial step         */
  double tol;              /* DP45 error tolerance on |m5-m4|           */
  double dt_min, dt_max;   /* s, DP45 bounds (<= 0: 1e-20 and 1e-10)    */
  int32_t cavity_mode;     /* LLGC_CAVITY_ODE or LLGC_CAVITY_MEMORY      */
  const float *brms_map;   /* T, vacuum field of the mode per cell, 3 N
                              float32 as [c][z][y][x] (device; copied), or
                              NULL for the uniform brms.  Section "Workflow
                              in Mumax3-cQED": B_rms may vary in space.
                              Not with llgc_adjoint. */
  double ku2;              /* J/m^3, second-order uniaxial anisotropy on
                              anis_u: energy density -Ku2 (u.m)^4, field
                              (4 Ku2/Ms)(u.m)^3 u.  Not with llgc_adjoint. */
  int32_t no_precession;   /* 1: torque -gamma alpha/(1+alpha^2) m x (m x B)
                              only (relaxation dynamics, as Mumax3's
                              relax); 0: full LL torque.  Not with
                              llgc_adjoint. */
  const float *fdrive_map; /* T per unit drive, 3 N float32 as [c][z][y][x]
                              (device; copied), or NULL for the uniform
                              fdrive_dir.  Replaces fdrive_dir cell by cell:
                              B_ext,i(t) = bext + fdrive_amp f(t) map_i, the
                              excitation of the paper's example script
                              (B_ext += amp B_rms(r) sinc(w t), appendix
                              "Micromagnetic simulations with Mumax3-cQED").
                              Not with llgc_adjoint. */
  double dmi_int, dmi_bulk; /* J/m^2, Dzyaloshinskii-Moriya constants (one
                              of the effective-field terms listed after
                              Eq. (llg)): interfacial, energy density
                              D [m_z div m - (m.grad) m_z] (film normal z),
                              and bulk, D m.curl m; discretised on the bonds
                              between magnetic neighbours, E = sum_bonds
                              c_ij.(m_i x m_j), c_ij = D_int V_c (z x e_ij)
                              /d - D_bulk V_c e_ij/d, a missing neighbour's
                              bond omitted.  Not with llgc_adjoint. */
  double temperature;      /* K; > 0 adds Brown's thermal field (the last
                              effective-field term listed after Eq. (llg)):
                              per cell and component a Gaussian of variance
                              2 alpha kB T / (gamma Ms_i V_c dt), drawn
                              afresh each RK4 step (counted from
                              llgc_set_state) and held over its stages.
                              RK4 only (LLGC_E_UNSUPPORTED with DP45); not
                              with llgc_adjoint; off during llgc_relax. */
  uint64_t seed;           /* key of the thermal field's Philox4x32-10
                              generator (counter: cell, step) */
} llgc_params;

typedef struct {
  int64_t accepted, rejected, rhs_evals;
  double t, dt, last_err;
} llgc_run_info;

/* Creates a context for one grid of finite-difference cells, the
 * discretisation the paper inherits from Mumax3 (section "The LLG equation
 * in Mumax3"; the script's SetGridSize / SetCellSize of appendix
 * "Micromagnetic simulations with Mumax3-cQED").  `hip_stream` is a
 * hipStream_t (NULL = the default stream).  Allocates every device buffer the grid needs and
 * plans the padded FFT sizes; no parameters or state are set yet.
 * Errors: LLGC_E_ARG (bad sizes, out == NULL), LLGC_E_UNSUPPORTED (nz > 4
 * or padded sizes beyond the on-chip FFT limits), LLGC_E_OOM, LLGC_E_HIP. */
int llgc_create(const llgc_grid *grid, void *hip_stream, llgc_ctx **out);

/* Energy minimisation by damped dynamics: the relax() the paper's example
 * script calls before its run (appendix "Micromagnetic simulations with
 * Mumax3-cQED"; the relax of Mumax3).  With the precession term off, the
 * cavity decoupled (no cavity field; amplitudes kept) and the drives off,
 * Dormand-Prince steps (params.tol, or 1e-6) run in blocks of 8 accepted
 * steps; after each block the torque |dm/dt| of the current state is
 * evaluated: with `torque_tol` > 0 (rad/s) the relaxation stops once its
 * maximum is below it; with `torque_tol` <= 0, once the mean of |dm/dt|^2
 * over the magnetic cells has not decreased since the previous block; in
 * any case after `max_steps` accepted steps (<= 0: 100000).  m keeps the relaxed state;
 * t, the cavity amplitudes, the step counters and every parameter are as
 * before the call.  `max_torque` (host, may be NULL) receives the last
 * block's largest |dm/dt|; `info` (may be NULL) the relaxation's steps.
 * Errors: LLGC_E_STATE (no params/state), and as llgc_run. */
int llgc_relax(llgc_ctx *ctx, double torque_tol, int64_t max_steps,
               double *max_torque, llgc_run_info *info);

/* ---------------------------------------------------------------------
 * Multimode cavity.  The paper simulates one mode at a time and notes that
 * a cavity of several modes follows by summing them (section
 * "Ferromagnetic materials in a cavity", subsection "Effects of the parity
 * of the magnetic mode").  Here each mode k has its own vacuum field
 * B_rms,k (uniform, or per cell), frequency, loss, initial amplitude and
 * drive; the cavity field is sum_k B_rms,k (alpha_k + alpha_k^*) in both
 * torque terms, and every amplitude obeys the single-mode equation
 *   d alpha_k/dt = -(i wc_k + kappa_k) alpha_k
 *                  + i (V_c/hbar) sum_i Ms_i m_i . B_rms,k,i - i eps_k(t)
 * with its own coupling sum.  The DP45 amplitude error is the 2-norm over
 * the modes relative to max(1, |alpha|_2). */
#define LLGC_MAX_MODES 8
typedef struct {
  double brms[3];          /* T, uniform vacuum field of the mode           */
  const float *brms_map;   /* T per cell, 3 N float32 [c][z][y][x] (device;
                              copied), or NULL for brms                     */
  double wc, kappa;        /* rad/s                                          */
  double x0, p0;           /* initial 2 Re alpha_k, -2 Im alpha_k            */
  int32_t cdrive_kind;     /* LLGC_DRIVE_*: d alpha_k/dt -= i amp f(t)      */
  double cdrive_amp, cdrive_w;
} llgc_mode;

/* Replaces the single mode of the parameters (the llgc_params fields brms,
 * brms_map, wc, kappa, x0, p0, cdrive_*) by `n_modes` modes (host array; maps copied); n_modes = 0
 * returns to the single mode of the parameters.  Sets every amplitude to
 * (x0_k - i p0_k)/2.  With modes set: records (llgc_run) have 4 + 2 n_modes
 * columns (t, <m>, then Re, Im of each mode); llgc_set_state keeps the
 * amplitudes and ignores its a_re, a_im; llgc_get_state returns mode 0's;
 * llgc_reset_cavity sets each mode to its own x0, p0 (its arguments are
 * ignored); llgc_eval_rhs uses the current amplitudes and writes 2 doubles
 * per mode to dadt.  Call after llgc_set_params (which keeps the modes).
 * Errors: LLGC_E_STATE (no params), LLGC_E_ARG (n_modes outside
 * 0..LLGC_MAX_MODES, negative kappa, unknown drive), LLGC_E_UNSUPPORTED
 * (the memory recursion, batch-plan instances; llgc_adjoint refuses a
 * context with modes), LLGC_E_OOM, LLGC_E_HIP. */
int llgc_set_modes(llgc_ctx *ctx, int32_t n_modes, const llgc_mode *modes);

/* Amplitudes of the modes: host arrays of 2 n_modes doubles (Re, Im per
 * mode).  The getter returns n_modes (or an error); both synchronise the
 * stream.  Errors: LLGC_E_STATE (no modes set), LLGC_E_ARG (NULL). */
int llgc_set_mode_amplitudes(llgc_ctx *ctx, const double *a_re_im);
int llgc_get_mode_amplitudes(llgc_ctx *ctx, double *a_re_im);

/* Plan flags of llgc_create_ex. */
enum { LLGC_PLAN_BATCH = 1 };

/* As llgc_create, with plan flags.  LLGC_PLAN_BATCH selects the fixed plan
 * that every instance of a batch (llgc_batch_create) uses: padded lengths
 * of at least 64 points, LDS Stockham FFTs in every pass, x passes that
 * transform the three components of a tile of rows at once (rows per tile
 * chosen so one 512-thread workgroup is full) and a spectral pass with a
 * fixed workgroup size.  A context created with it performs bit for bit
 * the same arithmetic as the same problem run inside a batch (the sweeps
 * of section "Benchmark").  It needs 2 <= nx, ny <= 128.
 * Errors: as llgc_create; LLGC_E_ARG for unknown flags;
 * LLGC_E_UNSUPPORTED outside the batched size range. */
int llgc_create_ex(const llgc_grid *grid, void *hip_stream, int32_t flags,
                   llgc_ctx **out);

/* Frees every buffer of the context.  NULL is accepted. */
int llgc_destroy(llgc_ctx *ctx);

/* Message of the last failed call on `ctx` (owned by ctx, valid until the
 * next call).  Never NULL. */
const char *llgc_last_error(const llgc_ctx *ctx);

/* Sets the material, field, cavity and integrator parameters: the
 * quantities of Eq. (llg) and its effective field (section "The LLG
 * equation in Mumax3") and the cavity additions B_rms, Wc, Kappa, X0, P0,
 * HBAR of section "Workflow in Mumax3-cQED".  Copies parameters and maps;
 * (re)builds the demag kernel when the cell geometry requires it (first
 * call); resets the cavity amplitude to
 * alpha_0 = (x0 - i p0)/2 and t to 0 only if no state was set before.
 * Errors: LLGC_E_ARG (non-positive ms without map, negative alpha, unknown
 * method or drive kind, dt <= 0), LLGC_E_HIP. */
int llgc_set_params(llgc_ctx *ctx, const llgc_params *p);

/* Sets the joint state of Eqs. (eqmotionspinclasical)/(eqmotionaclasical):
 * m (device pointer, 3*N float32 SoA, copied; the reduced magnetisation of
 * Eq. (llg), one unit vector per cell), the time t and the cavity amplitude
 * alpha = a_re + i a_im.  The vectors are used as given
 * (callers normalise).  Errors: LLGC_E_ARG (m == NULL). */
int llgc_set_state(llgc_ctx *ctx, const float *m_dev, double t, double a_re,
                   double a_im);

/* Reads the joint state back: the outputs the paper's runs record, the
 * magnetisation (section "Workflow in Mumax3-cQED") and the cavity
 * amplitude whose modulus squared is the photon number (section
 * "Introducing the effect of the cavity").  Copies m into `m_dev` (device,
 * 3*N float32; may be NULL) and returns t and alpha (host pointers, may be
 * NULL).  Synchronises the stream. */
int llgc_get_state(llgc_ctx *ctx, float *m_dev, double *t, double *a_re_im);

/* ResetMemoryTerm analogue (paper, script additions): declares the current
 * state to be t = 0 with cavity amplitude alpha_0 = (x0 - i p0)/2. */
int llgc_reset_cavity(llgc_ctx *ctx, double x0, double p0);

/* CavityFeatureStatus analogue: 1 if |B_rms| > 0, else 0 (or an error). */
int llgc_cavity_enabled(const llgc_ctx *ctx);

/* Integrates the joint (m, alpha) system of Eq. (llg) with the cavity
 * field and Eq. (eqmotionaclasical) with loss, the script's Run(t) of
 * appendix "Micromagnetic simulations with Mumax3-cQED", with one of the
 * ODE integrators the paper keeps unchanged from Mumax3 (section "Adapting
 * the memory term for efficient computation"): classic RK4 or
 * Dormand-Prince 5(4).
 * RK4: `nsteps` fixed steps of params.dt (t_end ignored if nsteps > 0;
 *      otherwise nsteps = round((t_end - t)/dt)).
 * DP45: adaptive steps until t == t_end (the last step is truncated to land
 *      on t_end); nsteps > 0 caps the number of accepted steps.
 * Records (host buffer `rec`, rows of 6 float64: t, <mx>, <my>, <mz>,
 * Re alpha, Im alpha) are written for the initial state and after every
 * `record_every`-th accepted step (record_every <= 0: none), up to
 * `rec_cap` rows; `n_rec` receives the count.  `info` may be NULL.
 * Errors: LLGC_E_STATE (no params/state), LLGC_E_DT_UNDERFLOW,
 * LLGC_E_NONFINITE (adaptive error non-finite until underflow), LLGC_E_HIP.
 * On any failure (LLGC_E_NONFINITE, LLGC_E_DT_UNDERFLOW) m, t and alpha
 * are those of the last accepted step: RK4 writes each new state into a
 * scratch register and commits it once the step is known to be finite;
 * DP45 commits only accepted attempts.
 * Launches: the kernels of a chunk (8 DP45 attempts, or one RK4 step) are
 * captured once into a HIP graph on a private stream and replayed on the
 * context's stream; the graph is captured again after anything passed by
 * value changes (params, plan, record buffer).  Timed contexts
 * (llgc_set_timing) and contexts created with the environment variable
 * LLGC_NO_GRAPHS set launch directly; results are identical either way. */
int llgc_run(llgc_ctx *ctx, int64_t nsteps, double t_end,
             int32_t record_every, double *rec, int64_t rec_cap,
             int64_t *n_rec, llgc_run_info *info);

/* One accepted step of llgc_run's integration (Eq. (llg) with the cavity,
 * Eq. (eqmotionaclasical)): RK4 with params.dt, or DP45 adaptive with
 * retries inside.  Errors and state on failure as llgc_run. */
int llgc_step(llgc_ctx *ctx, llgc_run_info *info);

/* Evaluates the right-hand side once, for parity checks: given m (device,
 * 3*N float32), alpha and t, writes dm/dt to `dmdt_dev` (device, 3*N
 * float32), the total effective field to `beff_dev` (device, 3*N float32,
 * may be NULL) and d alpha/dt to `dadt` (host, 2 float64, may be NULL).
 * Does not change the integrator state. */
int llgc_eval_rhs(llgc_ctx *ctx, const float *m_dev, double a_re,
                  double a_im, double t, float *dmdt_dev, float *beff_dev,
                  double *dadt);

/* As llgc_eval_rhs, for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the evaluation's control block, partial sums and half
 * spectrum live in a static device array of the library (16 MiB per
 * device, held until the process ends) instead of the context's buffers,
 * and the call allocates nothing.  The context still supplies the
 * parameters and the demag kernel; the caller passes m, dmdt and beff as
 * for llgc_eval_rhs.  Calls share the array of their device: calls that
 * overlap on one GPU (other threads, other streams) race; each call clears
 * what it reads before use.  The current HIP device must be the one the
 * context was created on.
 * Errors: as llgc_eval_rhs; LLGC_E_ARG (another device current);
 * LLGC_E_UNSUPPORTED when the grid needs more than 16 MiB of scratch
 * (roughly (nx+1) * ny * nz * 24 bytes with demag; 512 x 512 x 2 fits);
 * LLGC_E_HIP. */
int llgc_eval_rhs_noalloc(llgc_ctx *ctx, const float *m_dev, double a_re,
                          double a_im, double t, float *dmdt_dev,
                          float *beff_dev, double *dadt);

/* Plan autotuner for the demag convolution of Eq. (llg)'s effective field
 * (section "The LLG equation in Mumax3").  Each of the three FFT passes (y
 * spectral pass, forward x pass, field x pass) can hold its transforms in
 * registers (one wavefront per transform) or in LDS (Stockham passes); which
 * is faster depends on the padded lengths, the layer count and how full the
 * GPU is.  With `reps` > 0, times every feasible combination on this
 * context's grid (two rounds of `reps` right-hand-side evaluations of the
 * current state, result discarded), keeps the fastest, then tries halving
 * and doubling the rows per x-pass tile and the kx columns per spectral
 * workgroup of that plan one at a time (kept when 2% faster, within the
 * kernels' register and LDS limits), and records the plan for the grid
 * shape (nx, ny, nz, demag on/off) in a process-wide table; with
 * `reps` <= 0, applies the recorded plan for this shape if there is one
 * and otherwise keeps the current plan.  The integrator state is not
 * changed; results of later calls differ from the untuned plan's only by
 * float32 rounding.  `choice` (host, may be NULL) receives the plan kind:
 * bit 0 register y pass, bit 1 register forward x pass, bit 2 register
 * field x pass, bit 3 LDS x passes over the three components of a tile at
 * once (padded x length >= 64).  Not thread-safe against other calls on the same context.
 * Errors: LLGC_E_ARG (NULL context, or a batch-plan instance, whose plan
 * is fixed), LLGC_E_STATE (no params), LLGC_E_HIP. */
int llgc_autotune(llgc_ctx *ctx, int32_t reps, int32_t *choice);

/* Gradient of a cavity observable by the discrete adjoint of the RK4 path.
 * Runs `n_steps` RK4 steps of size `dt` from the current state (the state
 * advances), with the loss
 *     L = (1/(n1-n0+1)) sum_{n=n0..n1} |alpha_n|^2
 * over step endpoints n (1-based, 1 <= n0 <= n1 <= n_steps), then sweeps
 * the discrete adjoint backwards with checkpoints every `ckpt_stride` steps
 * (0: ceil(sqrt(n_steps))), recomputing each segment once.  Outputs:
 * `loss` (host), dL/dMs and dL/dKu per cell (device, N float32 each, may be
 * NULL), dL/dB_rms (host, 3 float64, may be NULL) and dL/d(cavity drive
 * amplitude) (host, may be NULL).  This is the gradient the paper's
 * observables (photon number |alpha|^2, section "Introducing the effect of
 * the cavity") admit with respect to the material maps and the coupling.
 * Errors: LLGC_E_STATE (no params/state), LLGC_E_ARG (window),
 * LLGC_E_UNSUPPORTED (padded x length < 64), LLGC_E_OOM, LLGC_E_HIP. */
int llgc_adjoint(llgc_ctx *ctx, int64_t n_steps, double dt,
                 int64_t ckpt_stride, int64_t n0, int64_t n1, double *loss,
                 float *grad_ms, float *grad_ku, double *grad_brms,
                 double *grad_cdrive_amp);

/* Copies the demagnetising kernel the context built, for inspection: the
 * real coefficients K[kx][ky][comp][dz] (comp = xx, yy, zz, xy, xz, yz;
 * xz and yz are the coefficients of -i) already scaled by
 * -mu0/(Px*Py), kx in [0, Px/2], ky in [0, Py/2], dz in [0, nz).
 * `dims` (host, 4 int32) receives Px, Py, Px/2+1, Py/2+1.  `out` is a host
 * buffer of at least 6*nz*(Px/2+1)*(Py/2+1) floats, or NULL. */
int llgc_demag_kernel(llgc_ctx *ctx, float *out, int64_t cap, int32_t *dims);

/* Real-space demag tensor N(Delta) for non-negative offsets (octant),
 * float64 [comp][dz][dy][dx] with comp = xx, yy, zz, xy, xz, yz, as
 * computed on the device (host buffer of 6*N doubles). */
int llgc_demag_tensor(llgc_ctx *ctx, double *out, int64_t cap);

/* Per-kernel timing with HIP events recorded around every launch on the
 * context's stream (off by default; enabling adds events, not syncs).
 * llgc_kernel_times fills, for up to `cap` kernels, total milliseconds and
 * launch counts, and writes the kernel names joined by ';' into `names`
 * (size names_cap).  Synchronises the stream.  `reset` != 0 clears. */
int llgc_set_timing(llgc_ctx *ctx, int32_t enable);
/* Restricts timing to the launches of one kernel (name as reported by
 * llgc_kernel_times; NULL or "" = all kernels), so that the events perturb
 * a timed run as little as possible.  Events are pooled per context. */
int llgc_set_timing_only(llgc_ctx *ctx, const char *kernel);
int llgc_kernel_times(llgc_ctx *ctx, double *ms, int64_t *launches,
                      int32_t cap, char *names, int32_t names_cap,
                      int32_t reset);

/* ---------------------------------------------------------------------
 * Batched engine: many independent problems of different grid sizes
 * advanced together, one launch per kernel and stage for all of them.
 * This is the shape of the paper's parameter studies (the Dicke-model
 * validation repeated over the whole range of omega_c, omega_z and lambda,
 * section "Benchmark"; material and size scans of section "Ferromagnetic
 * materials in a cavity"), where each run alone is too small to fill the
 * GPU.  Each instance is an ordinary context with the LLGC_PLAN_BATCH plan
 * owned by the batch; it is configured with llgc_set_params /
 * llgc_set_state and read with llgc_get_state as usual.  Every instance
 * keeps its own time, step size, step controller and cavity; instances
 * that finish drop out of the launches. */
typedef struct llgc_batch llgc_batch;

/* Creates `n_inst` instances, instance k on grids[k] (host array).  All
 * instances share `hip_stream`.  Grid limits as LLGC_PLAN_BATCH.
 * Errors: LLGC_E_ARG (n_inst < 1, NULL pointers), LLGC_E_UNSUPPORTED,
 * LLGC_E_OOM, LLGC_E_HIP. */
int llgc_batch_create(const llgc_grid *grids, int32_t n_inst,
                      void *hip_stream, llgc_batch **out);

/* Frees the batch and all its instances.  NULL is accepted. */
int llgc_batch_destroy(llgc_batch *b);

/* Message of the last failed batch call (owned by b).  Never NULL. */
const char *llgc_batch_last_error(const llgc_batch *b);

/* Instance k (0 <= k < n_inst), owned by the batch (do not destroy), or
 * NULL for an invalid index. */
llgc_ctx *llgc_batch_instance(llgc_batch *b, int32_t k);

/* Runs every instance as llgc_run would run it alone, with the same
 * `nsteps`, `t_end` and `record_every` for all instances (t_end is an
 * absolute time on each instance's own clock).  All instances must use
 * the same method.  Records: host buffer of n_inst * rec_cap rows of 6
 * float64, instance k's rows starting at row k * rec_cap; `n_rec`
 * (n_inst int64), `info` (n_inst entries) and `status` (n_inst int32,
 * each instance's llgc_run status) may be NULL.  Returns LLGC_OK when every
 * instance succeeded, else the first failing instance's status (its
 * message in llgc_batch_last_error).
 * Each round of 8 attempts over the active instances is one HIP graph
 * (captured again when finished instances are retired from the work
 * tables), unless LLGC_NO_GRAPHS was set when the batch was created.
 * Errors: LLGC_E_STATE (an instance without params/state), LLGC_E_ARG
 * (mixed methods, records without a buffer), LLGC_E_HIP. */
int llgc_batch_run(llgc_batch *b, int64_t nsteps, double t_end,
                   int32_t record_every, double *rec, int64_t rec_cap,
                   int64_t *n_rec, llgc_run_info *info, int32_t *status);

/* Plan facts (host ints, 8 entries): Px, Py, rows per x-pass block,
 * kx columns per spectral block, x-pass threads, spectral threads,
 * x-pass LDS bytes, spectral LDS bytes. */
int llgc_plan_info(const llgc_ctx *ctx, int32_t *info8);

#ifdef __cplusplus
}
#endif
#endif /* LLGC_H */
