// Shared device/host definitions of the llgc library (gfx950 only).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace llgc {

constexpr int kMaxStages = 8;
constexpr int kMaxModes = 8;   // modes of a multimode cavity

// Constants of a multimode cavity (device memory owned by the context):
// each mode k has its own vacuum field (uniform vector, or a per-cell map),
// frequency, loss and drive.
struct Modes {
  int n;                          // 1..kMaxModes
  double br[kMaxModes][3];        // uniform B_rms of each mode (T)
  double wc[kMaxModes], kappa[kMaxModes];
  int ckind[kMaxModes];
  double camp[kMaxModes], cw[kMaxModes];
  const float* map[kMaxModes];    // per-cell field [c][cell] of mode k, or
                                  // nullptr for its uniform br[k]
  int any_map;                    // some mode has a map
};

// Device-resident integrator control block.  Everything that decides the
// next step (time, step size, cavity amplitude and stage values, accept /
// reject) lives here so that a run needs no host round trip per step.
struct Ctl {
  double t, dt, t_end;
  double a_re, a_im;                         // cavity amplitude at t
  double as_re[kMaxStages], as_im[kMaxStages];  // stage inputs a_s (s>=1)
  double ka_re[kMaxStages], ka_im[kMaxStages];  // stage rates k_a,s
  double anext_re, anext_im;                 // RK4 end-of-step amplitude
  double err_a, last_err, F_last;
  double rhs_dadt_re, rhs_dadt_im;
  long long accepted, rejected, rhs_evals, max_accepted;
  int pending_accept, done, status, prev_rej;
  int nrec, rec_every, rec_cap;
  unsigned int emax_bits;   // Dormand-Prince error: atomic maximum (float bits)
  unsigned int cnt_xfwd, cnt_field, cnt_begin, cnt_rec;
  // optional: per-step cavity history (stage amplitudes a_1..a_4 and the
  // end-of-step amplitude, 5 complex per step) and the windowed loss
  // sum_{n0 <= n <= n1} |alpha_n|^2 over accepted RK4 steps n (1-based)
  double* ahist;
  long long mem_n;   // memory recursion: steps since the state was set
  long long loss_n0, loss_n1;
  double loss_acc;
  // multimode cavity (Prm::modes set): these replace the single-mode
  // amplitude fields above, one entry per mode
  double ma_re[kMaxModes], ma_im[kMaxModes];            // at t
  double mas_re[kMaxStages][kMaxModes], mas_im[kMaxStages][kMaxModes];
  double mka_re[kMaxStages][kMaxModes], mka_im[kMaxStages][kMaxModes];
  double manext_re[kMaxModes], manext_im[kMaxModes];    // RK4 end of step
  long long noise_n;   // thermal field: index of the current RK4 step
};

enum { ST_OK = 0, ST_UNDERFLOW = 1, ST_NONFINITE = 2 };

// Scalar problem parameters passed by value to every kernel.
struct Prm {
  int nx, ny, nz, ncell;
  int nyp;                      // spectrum row length (ny rounded up to even)
  int Px, Py, Hx, Hy, logPx, logPy;
  float idx2, idy2, idz2;       // 1/d^2 per axis
  float ms;                     // uniform Ms (A/m) when ms_map == nullptr
  float ims;                    // 1 / ms (0 if ms = 0)
  const float* ms_map;
  int masked;                   // ms_map has cells with Ms = 0 (geometry)
  double nmag;                  // magnetic cells (averages)
  float aex2;                   // 2 A
  float ku2;                    // 2 Ku (J/m^3) when ku_map == nullptr
  const float* ku_map;
  float ux, uy, uz;             // anisotropy axis
  float bx, by, bz;             // static external field
  int fkind;
  double famp, fw;
  float fdx, fdy, fdz;          // field drive direction (0 with a map)
  const float* fdrive_map;      // per-cell drive vector [c][cell] or nullptr
  int demag;
  float brx, bry, brz;          // B_rms
  const float* brms_map;        // per-cell B_rms [c][cell] or nullptr
  double brxd, bryd, brzd;
  double wc, kappa, vc_hbar;    // V_c / hbar
  int ckind;
  double camp, cw;
  float gpref;                  // -gamma / (1 + alpha^2)
  float ku4;                    // 4 Ku2 (J/m^3)
  float prec;                   // 1: precession term on, 0: off
  float dmi_i, dmi_b;           // DMI constants (J/m^2): interfacial, bulk
  float idx1, idy1, idz1;       // 1/d per axis
  double therm;                 // 2 alpha kB T / (gamma V_c); 0: no thermal
  unsigned int seed_lo, seed_hi;  // key of the thermal generator
  int plain;                    // none of: B_rms map, geometry, Ku2, no precession
  float alpha;
  int method;                   // 0 RK4, 1 DP45
  int cmode;                    // 0 cavity ODE, 1 memory recursion
  double tol, dt_min, dt_max;
  const Modes* modes;           // multimode cavity, or nullptr (one mode)
  double* mpart;                // multimode coupling partials [tile][mode]
  int recw;                     // record row width: 6, or 4 + 2 modes
};

// Runge-Kutta epilogue description of one stage of the field kernel.
struct Epi {
  int kind;            // 0: evaluate only, 1: stage, 2: RK4 final, 3: DP45 error
  int np;              // number of previous k's used
  const float* yn;     // base state y_n
  const float* kp[6];  // previous k_j
  float ca[6];         // their coefficients (times dt)
  float cself;         // coefficient of this stage's k
  float* ynext;        // y_{s+1}, or y_n itself for the RK4 final stage
  float* kout;         // k_s output (may be null)
  float* bout;         // B_eff output (may be null)
  float* nout;         // RK4 final: |m_hat| before renormalisation (or null)
  float* commit;       // RK4 stage 1 of a run: the stage input (the state
                       // the previous step left in a scratch register) is
                       // copied here, committing it as y_n (or null)
  unsigned int* emax;  // DP45 error: also kept as the atomic maximum of the
                       // workgroups' errors' float bits here (or null)
};

// Demag-kernel table entry: the real coefficients of one (kx, |ky|) for all
// z offsets dz, comp = xx yy zz xy at dz = 0 .. nz-1, then xz yz at
// dz = 1 .. nz-1 (odd in dz, they vanish at dz = 0 and are not stored):
// 6 nz - 2 floats.
__host__ __device__ constexpr int kentry(int nz) { return 6 * nz - 2; }
__host__ __device__ constexpr int kslot(int comp, int dz, int nz) {
  return comp < 4 ? comp * nz + dz : 4 * nz + (comp - 4) * (nz - 1) + dz - 1;
}

__host__ __device__ inline int ilog2(int v) {
  int r = 0;
  while ((1 << r) < v) ++r;
  return r;
}

}  // namespace llgc
