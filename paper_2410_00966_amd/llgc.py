"""Python binding of the llgc C ABI (include/llgc.h).

Argument marshalling only: every step of the integration runs in the HIP
kernels of libllgc.so.  PyTorch supplies device memory and the stream.
Importing works without a GPU; creating a `Sim` requires the built library
and a visible GPU and raises otherwise (there is no CPU fallback).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libllgc.so")

LLGC_OK = 0
ERRORS = {-1: "LLGC_E_ARG", -2: "LLGC_E_OOM", -3: "LLGC_E_HIP",
          -4: "LLGC_E_NONFINITE", -5: "LLGC_E_DT_UNDERFLOW",
          -6: "LLGC_E_STATE", -7: "LLGC_E_UNSUPPORTED"}
RK4, DP45 = 0, 1

EXPORTED = ("llgc_create", "llgc_destroy", "llgc_last_error",
            "llgc_set_params", "llgc_set_state", "llgc_get_state",
            "llgc_reset_cavity", "llgc_cavity_enabled", "llgc_run",
            "llgc_step", "llgc_eval_rhs", "llgc_adjoint", "llgc_demag_kernel",
            "llgc_demag_tensor", "llgc_set_timing", "llgc_kernel_times",
            "llgc_plan_info", "llgc_create_ex", "llgc_batch_create",
            "llgc_batch_destroy", "llgc_batch_last_error",
            "llgc_batch_instance", "llgc_batch_run", "llgc_set_timing_only",
            "llgc_autotune", "llgc_eval_rhs_noalloc", "llgc_set_modes",
            "llgc_set_mode_amplitudes", "llgc_get_mode_amplitudes",
            "llgc_relax")
PLAN_BATCH = 1


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("nz", ctypes.c_int32), ("dx", ctypes.c_double),
                ("dy", ctypes.c_double), ("dz", ctypes.c_double)]


_D3 = ctypes.c_double * 3
_FP = ctypes.c_void_p


class Params(ctypes.Structure):
    _fields_ = [
        ("ms", ctypes.c_double), ("ms_map", _FP),
        ("aex", ctypes.c_double), ("alpha", ctypes.c_double),
        ("ku1", ctypes.c_double), ("ku1_map", _FP), ("anis_u", _D3),
        ("bext", _D3),
        ("fdrive_kind", ctypes.c_int32), ("fdrive_amp", ctypes.c_double),
        ("fdrive_w", ctypes.c_double), ("fdrive_dir", _D3),
        ("enable_demag", ctypes.c_int32),
        ("brms", _D3),
        ("wc", ctypes.c_double), ("kappa", ctypes.c_double),
        ("x0", ctypes.c_double), ("p0", ctypes.c_double),
        ("cdrive_kind", ctypes.c_int32), ("cdrive_amp", ctypes.c_double),
        ("cdrive_w", ctypes.c_double),
        ("gamma", ctypes.c_double), ("hbar", ctypes.c_double),
        ("mu0", ctypes.c_double),
        ("method", ctypes.c_int32), ("dt", ctypes.c_double),
        ("tol", ctypes.c_double), ("dt_min", ctypes.c_double),
        ("dt_max", ctypes.c_double), ("cavity_mode", ctypes.c_int32),
        ("brms_map", _FP), ("ku2", ctypes.c_double),
        ("no_precession", ctypes.c_int32), ("fdrive_map", _FP),
        ("dmi_int", ctypes.c_double), ("dmi_bulk", ctypes.c_double),
        ("temperature", ctypes.c_double), ("seed", ctypes.c_uint64),
    ]


class Mode(ctypes.Structure):
    _fields_ = [("brms", _D3), ("brms_map", _FP),
                ("wc", ctypes.c_double), ("kappa", ctypes.c_double),
                ("x0", ctypes.c_double), ("p0", ctypes.c_double),
                ("cdrive_kind", ctypes.c_int32),
                ("cdrive_amp", ctypes.c_double),
                ("cdrive_w", ctypes.c_double)]


class RunInfo(ctypes.Structure):
    _fields_ = [("accepted", ctypes.c_int64), ("rejected", ctypes.c_int64),
                ("rhs_evals", ctypes.c_int64), ("t", ctypes.c_double),
                ("dt", ctypes.c_double), ("last_err", ctypes.c_double)]


class LLGCError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


_lib = None


def load():
    """Loads libllgc.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "__graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                         ctypes.c_double)
    P = ctypes.POINTER
    sig = {
        "llgc_create": ([P(Grid), vp, P(vp)], ctypes.c_int),
        "llgc_destroy": ([vp], ctypes.c_int),
        "llgc_last_error": ([vp], ctypes.c_char_p),
        "llgc_set_params": ([vp, P(Params)], ctypes.c_int),
        "llgc_set_state": ([vp, vp, dbl, dbl, dbl], ctypes.c_int),
        "llgc_get_state": ([vp, vp, P(dbl), P(dbl)], ctypes.c_int),
        "llgc_reset_cavity": ([vp, dbl, dbl], ctypes.c_int),
        "llgc_cavity_enabled": ([vp], ctypes.c_int),
        "llgc_run": ([vp, i64, dbl, i32, P(dbl), i64, P(i64), P(RunInfo)],
                     ctypes.c_int),
        "llgc_step": ([vp, P(RunInfo)], ctypes.c_int),
        "llgc_eval_rhs": ([vp, vp, dbl, dbl, dbl, vp, vp, P(dbl)],
                          ctypes.c_int),
        "llgc_adjoint": ([vp, i64, dbl, i64, i64, i64, P(dbl), vp, vp,
                          P(dbl), P(dbl)], ctypes.c_int),
        "llgc_demag_kernel": ([vp, P(ctypes.c_float), i64, P(i32)],
                              ctypes.c_int),
        "llgc_demag_tensor": ([vp, P(dbl), i64], ctypes.c_int),
        "llgc_set_timing": ([vp, i32], ctypes.c_int),
        "llgc_kernel_times": ([vp, P(dbl), P(i64), i32, ctypes.c_char_p, i32,
                               i32], ctypes.c_int),
        "llgc_plan_info": ([vp, P(i32)], ctypes.c_int),
        "llgc_create_ex": ([P(Grid), vp, i32, P(vp)], ctypes.c_int),
        "llgc_batch_create": ([P(Grid), i32, vp, P(vp)], ctypes.c_int),
        "llgc_batch_destroy": ([vp], ctypes.c_int),
        "llgc_batch_last_error": ([vp], ctypes.c_char_p),
        "llgc_batch_instance": ([vp, i32], vp),
        "llgc_batch_run": ([vp, i64, dbl, i32, P(dbl), i64, P(i64),
                            P(RunInfo), P(i32)], ctypes.c_int),
        "llgc_set_timing_only": ([vp, ctypes.c_char_p], ctypes.c_int),
        "llgc_autotune": ([vp, i32, P(i32)], ctypes.c_int),
        "llgc_eval_rhs_noalloc": ([vp, vp, dbl, dbl, dbl, vp, vp, P(dbl)],
                                  ctypes.c_int),
        "llgc_set_modes": ([vp, i32, P(Mode)], ctypes.c_int),
        "llgc_set_mode_amplitudes": ([vp, P(dbl)], ctypes.c_int),
        "llgc_get_mode_amplitudes": ([vp, P(dbl)], ctypes.c_int),
        "llgc_relax": ([vp, dbl, i64, P(dbl), P(RunInfo)], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def grid_of(prob) -> Grid:
    return Grid(prob.nx, prob.ny, prob.nz, prob.dx, prob.dy, prob.dz)


def make_params(prob, ms_map=None, ku_map=None, brms_map=None,
                fdrive_map=None) -> Params:
    """Marshals an inputs.Problem into the C struct (maps: device tensors)."""
    p = Params()
    p.ms = prob.ms
    p.ms_map = ms_map.data_ptr() if ms_map is not None else None
    p.aex = prob.aex
    p.alpha = prob.alpha
    p.ku1 = prob.ku1
    p.ku1_map = ku_map.data_ptr() if ku_map is not None else None
    p.anis_u = _D3(*prob.anis_u)
    p.bext = _D3(*prob.bext)
    p.fdrive_kind = prob.fdrive_kind
    p.fdrive_amp = prob.fdrive_amp
    p.fdrive_w = prob.fdrive_w
    p.fdrive_dir = _D3(*prob.fdrive_dir)
    p.enable_demag = 1 if prob.enable_demag else 0
    p.brms = _D3(*prob.brms)
    p.wc, p.kappa, p.x0, p.p0 = prob.wc, prob.kappa, prob.x0, prob.p0
    p.cdrive_kind = prob.cdrive_kind
    p.cdrive_amp = prob.cdrive_amp
    p.cdrive_w = prob.cdrive_w
    p.gamma, p.hbar, p.mu0 = prob.gamma, prob.hbar, prob.mu0
    p.method = prob.method
    p.cavity_mode = getattr(prob, "cavity_mode", 0)
    p.brms_map = brms_map.data_ptr() if brms_map is not None else None
    p.ku2 = getattr(prob, "ku2", 0.0)
    p.no_precession = 0 if getattr(prob, "precession", 1) else 1
    p.fdrive_map = fdrive_map.data_ptr() if fdrive_map is not None else None
    p.dmi_int = getattr(prob, "dmi_int", 0.0)
    p.dmi_bulk = getattr(prob, "dmi_bulk", 0.0)
    p.temperature = getattr(prob, "temperature", 0.0)
    p.seed = int(getattr(prob, "seed", 0)) & ((1 << 64) - 1)
    p.dt, p.tol = prob.dt, prob.tol
    p.dt_min, p.dt_max = prob.dt_min, prob.dt_max
    return p


class Sim:
    """One llgc context on the current torch CUDA/HIP device and stream."""

    def __init__(self, prob, stream=None, batch_plan=False, _handle=None,
                 _owner=None):
        """`batch_plan`: use the fixed plan of batched instances (the same
        arithmetic as this problem inside a `Batch`)."""
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("llgc needs a GPU: no HIP device is visible")
        self.torch = torch
        self.L = load()
        self.prob = prob
        self.shape = (3, prob.nz, prob.ny, prob.nx)
        self.stream = stream or torch.cuda.current_stream()
        self._owner = _owner
        if _handle is None:
            g = grid_of(prob)
            h = ctypes.c_void_p()
            rc = self.L.llgc_create_ex(
                ctypes.byref(g), ctypes.c_void_p(self.stream.cuda_stream),
                PLAN_BATCH if batch_plan else 0, ctypes.byref(h))
            if rc != LLGC_OK:
                raise LLGCError(rc, "llgc_create_ex")
            self.h = h
        else:
            self.h = ctypes.c_void_p(_handle)
        self.set_params(prob)

    # ------------------------------------------------------------ helpers
    def _check(self, rc, what):
        if rc < 0:
            msg = self.L.llgc_last_error(self.h).decode()
            raise LLGCError(rc, f"{what}: {msg}")
        return rc

    def _dev(self, a, dtype=None):
        t = self.torch
        dtype = dtype or t.float32
        if isinstance(a, t.Tensor):
            return a.to(device="cuda", dtype=dtype).contiguous()
        return t.as_tensor(np.ascontiguousarray(a), dtype=dtype,
                           device="cuda")

    # ---------------------------------------------------------------- API
    def set_params(self, prob):
        self.prob = prob
        msm = self._dev(prob.ms_map) if prob.ms_map is not None else None
        kum = self._dev(prob.ku1_map) if prob.ku1_map is not None else None
        bm = getattr(prob, "brms_map", None)
        brm = self._dev(bm).reshape(-1) if bm is not None else None
        fm = getattr(prob, "fdrive_map", None)
        fdm = self._dev(fm).reshape(-1) if fm is not None else None
        p = make_params(prob, msm, kum, brm, fdm)
        self._check(self.L.llgc_set_params(self.h, ctypes.byref(p)),
                    "llgc_set_params")
        modes = getattr(prob, "modes", None)
        if modes is not None or getattr(self, "nmodes", 0):
            self.set_modes(modes or [])
        self.stream.synchronize()

    def set_modes(self, modes):
        """Multimode cavity (llgc_set_modes): `modes` is a list of
        inputs.Mode (maps: (3, nz, ny, nx) arrays); [] = the single mode of
        the parameters.  Amplitudes start at (x0 - i p0)/2 of each mode."""
        n = len(modes)
        arr = (Mode * max(n, 1))()
        keep = []
        for k, md in enumerate(modes):
            arr[k].brms = _D3(*md.brms)
            if md.brms_map is not None:
                bm = self._dev(md.brms_map).reshape(-1)
                keep.append(bm)
                arr[k].brms_map = bm.data_ptr()
            else:
                arr[k].brms_map = None
            arr[k].wc, arr[k].kappa = md.wc, md.kappa
            arr[k].x0, arr[k].p0 = md.x0, md.p0
            arr[k].cdrive_kind = md.cdrive_kind
            arr[k].cdrive_amp = md.cdrive_amp
            arr[k].cdrive_w = md.cdrive_w
        self._check(self.L.llgc_set_modes(self.h, n, arr), "llgc_set_modes")
        self.nmodes = n
        self.stream.synchronize()

    def mode_amplitudes(self):
        a = (ctypes.c_double * (2 * self.nmodes))()
        self._check(self.L.llgc_get_mode_amplitudes(self.h, a),
                    "llgc_get_mode_amplitudes")
        return np.array(a[0::2]) + 1j * np.array(a[1::2])

    def set_mode_amplitudes(self, a):
        a = np.asarray(a, dtype=complex).reshape(-1)
        if a.size == 1 and self.nmodes > 1:
            a = np.full(self.nmodes, a[0])
        buf = (ctypes.c_double * (2 * self.nmodes))()
        for k in range(self.nmodes):
            buf[2 * k], buf[2 * k + 1] = a[k].real, a[k].imag
        self._check(self.L.llgc_set_mode_amplitudes(self.h, buf),
                    "llgc_set_mode_amplitudes")

    def set_state(self, m, t=0.0, a=0j):
        """m, t and the amplitude (with several modes: one per mode, or one
        value for all)."""
        md = self._dev(m).reshape(self.shape)
        if getattr(self, "nmodes", 0):
            self.set_mode_amplitudes(a)
            a = 0j
        a = complex(a)
        self._check(self.L.llgc_set_state(self.h, md.data_ptr(), t, a.real,
                                          a.imag), "llgc_set_state")
        self.stream.synchronize()

    def get_state(self):
        m = self.torch.empty(self.shape, dtype=self.torch.float32,
                             device="cuda")
        t = ctypes.c_double()
        a = (ctypes.c_double * 2)()
        self._check(self.L.llgc_get_state(self.h, m.data_ptr(),
                                          ctypes.byref(t), a),
                    "llgc_get_state")
        self.stream.synchronize()
        if getattr(self, "nmodes", 0):
            return m, t.value, self.mode_amplitudes()
        return m, t.value, complex(a[0], a[1])

    def reset_cavity(self, x0=0.0, p0=0.0):
        self._check(self.L.llgc_reset_cavity(self.h, x0, p0),
                    "llgc_reset_cavity")

    def cavity_enabled(self):
        return self._check(self.L.llgc_cavity_enabled(self.h),
                           "llgc_cavity_enabled")

    def run(self, nsteps=0, t_end=0.0, record_every=0, rec_cap=0):
        """Returns (records (n, 6) float64, info dict)."""
        if record_every > 0 and rec_cap <= 0:
            rec_cap = (nsteps // record_every + 2) if nsteps else 100000
        width = 4 + 2 * getattr(self, "nmodes", 0) if getattr(
            self, "nmodes", 0) else 6
        rec = np.zeros((max(rec_cap, 1), width))
        nrec = ctypes.c_int64()
        info = RunInfo()
        rc = self.L.llgc_run(
            self.h, int(nsteps), float(t_end), int(record_every),
            rec.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
            int(rec_cap), ctypes.byref(nrec), ctypes.byref(info))
        self._check(rc, "llgc_run")
        return rec[: nrec.value].copy(), dict(
            accepted=info.accepted, rejected=info.rejected,
            rhs_evals=info.rhs_evals, t=info.t, dt=info.dt,
            last_err=info.last_err)

    def relax(self, torque_tol=0.0, max_steps=0):
        """llgc_relax: damped-dynamics energy minimisation of m (t, the
        cavity and the parameters unchanged).  Returns dict(accepted,
        rejected, rhs_evals, max_torque)."""
        info = RunInfo()
        mt = ctypes.c_double()
        self._check(self.L.llgc_relax(self.h, float(torque_tol),
                                      int(max_steps), ctypes.byref(mt),
                                      ctypes.byref(info)), "llgc_relax")
        return dict(accepted=info.accepted, rejected=info.rejected,
                    rhs_evals=info.rhs_evals, max_torque=mt.value)

    def step(self):
        info = RunInfo()
        self._check(self.L.llgc_step(self.h, ctypes.byref(info)),
                    "llgc_step")
        return dict(accepted=info.accepted, rejected=info.rejected,
                    t=info.t, dt=info.dt, last_err=info.last_err)

    def eval_rhs(self, m, a=0j, t=0.0, want_field=True):
        """One right-hand side: (dm/dt, B_eff, d alpha/dt).  With several
        modes `a` (one per mode) is set as the current amplitudes first and
        d alpha/dt is an array over the modes."""
        md = self._dev(m).reshape(self.shape)
        dm = self.torch.empty_like(md)
        B = self.torch.empty_like(md) if want_field else None
        nm = getattr(self, "nmodes", 0)
        if nm:
            # the evaluation reads the current amplitudes: set, then restore
            keep = self.mode_amplitudes()
            self.set_mode_amplitudes(a)
            a = 0j
        da = (ctypes.c_double * max(2, 2 * nm))()
        a = complex(a)
        self._check(self.L.llgc_eval_rhs(
            self.h, md.data_ptr(), a.real, a.imag, float(t), dm.data_ptr(),
            B.data_ptr() if B is not None else None, da), "llgc_eval_rhs")
        self.stream.synchronize()
        if nm:
            self.set_mode_amplitudes(keep)
            return dm, B, np.array(da[0::2]) + 1j * np.array(da[1::2])
        return dm, B, complex(da[0], da[1])

    def eval_rhs_noalloc(self, m, dm, B=None, a=0j, t=0.0):
        """llgc_eval_rhs_noalloc: as eval_rhs into caller-provided `dm` (and
        `B`), with the library's static scratch instead of allocations.
        Returns d alpha/dt."""
        md = self._dev(m).reshape(self.shape)
        da = (ctypes.c_double * 2)()
        a = complex(a)
        self._check(self.L.llgc_eval_rhs_noalloc(
            self.h, md.data_ptr(), a.real, a.imag, float(t), dm.data_ptr(),
            B.data_ptr() if B is not None else None, da),
            "llgc_eval_rhs_noalloc")
        self.stream.synchronize()
        return complex(da[0], da[1])

    def adjoint(self, n_steps, dt, n0, n1, stride=0):
        """Discrete-adjoint gradient of L = mean_{n0<=n<=n1} |alpha_n|^2
        after n_steps RK4 steps from the current state.  Returns dict(loss,
        g_ms, g_ku (device tensors shaped like one component plane),
        g_brms (3,), g_eps0)."""
        shape = self.shape[1:]
        gms = self.torch.empty(shape, dtype=self.torch.float32,
                               device="cuda")
        gku = self.torch.empty_like(gms)
        loss = ctypes.c_double()
        gb = (ctypes.c_double * 3)()
        ge = ctypes.c_double()
        self._check(self.L.llgc_adjoint(
            self.h, int(n_steps), float(dt), int(stride), int(n0), int(n1),
            ctypes.byref(loss), gms.data_ptr(), gku.data_ptr(), gb,
            ctypes.byref(ge)), "llgc_adjoint")
        self.stream.synchronize()
        return dict(loss=loss.value, g_ms=gms, g_ku=gku,
                    g_brms=np.array(list(gb)), g_eps0=ge.value)

    def demag_kernel(self):
        dims = (ctypes.c_int32 * 4)()
        self._check(self.L.llgc_demag_kernel(self.h, None, 0, dims),
                    "llgc_demag_kernel")
        Px, Py, Hx, Hy = list(dims)
        n = Hx * Hy * 6 * self.prob.nz
        out = np.zeros(n, dtype=np.float32)
        self._check(self.L.llgc_demag_kernel(
            self.h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), n,
            dims), "llgc_demag_kernel")
        return out.reshape(Hx, Hy, 6, self.prob.nz), (Px, Py)

    def demag_tensor(self):
        n = 6 * self.prob.nx * self.prob.ny * self.prob.nz
        out = np.zeros(n)
        self._check(self.L.llgc_demag_tensor(
            self.h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), n),
            "llgc_demag_tensor")
        return out.reshape(6, self.prob.nz, self.prob.ny, self.prob.nx)

    def autotune(self, reps=20):
        """Times the register/LDS FFT plan kinds on this grid and keeps the
        fastest (reps <= 0: reuse the kind recorded for this grid shape).
        Returns the kind: bit 0 register y pass, bit 1 register forward x
        pass, bit 2 register field x pass, bit 3 three-component LDS x
        passes."""
        k = ctypes.c_int32(-1)
        self._check(self.L.llgc_autotune(self.h, int(reps), ctypes.byref(k)),
                    "llgc_autotune")
        return k.value

    def set_timing(self, on=True, only=None):
        """Per-kernel HIP-event timing; `only` restricts it to one kernel."""
        self._check(self.L.llgc_set_timing(self.h, 1 if on else 0),
                    "llgc_set_timing")
        self._check(self.L.llgc_set_timing_only(
            self.h, only.encode() if only else None), "llgc_set_timing_only")

    def kernel_times(self, reset=False):
        cap = 32
        ms = (ctypes.c_double * cap)()
        ln = (ctypes.c_int64 * cap)()
        names = ctypes.create_string_buffer(1024)
        n = self._check(self.L.llgc_kernel_times(self.h, ms, ln, cap, names,
                                                 1024, 1 if reset else 0),
                        "llgc_kernel_times")
        keys = names.value.decode().split(";") if n else []
        return {k: (ms[i], ln[i]) for i, k in enumerate(keys)}

    def plan_info(self):
        info = (ctypes.c_int32 * 8)()
        self._check(self.L.llgc_plan_info(self.h, info), "llgc_plan_info")
        keys = ("Px", "Py", "rows_xfwd", "kx_per_block", "threads_x",
                "threads_y", "lds_xfwd", "lds_yspec")
        return dict(zip(keys, list(info)))

    def close(self):
        if getattr(self, "h", None):
            if self._owner is None:        # batch instances belong to it
                self.L.llgc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_cavity_loss_cls = None


def _cavity_loss_function():
    """torch.autograd.Function over llgc_adjoint (built on first use so that
    importing this module does not import torch)."""
    global _cavity_loss_cls
    if _cavity_loss_cls is not None:
        return _cavity_loss_cls
    import torch

    class CavityLoss(torch.autograd.Function):
        """L = mean over steps n0..n1 of |alpha_n|^2 after RK4 steps from
        m0 (the photon number of section "Introducing the effect of the
        cavity") as a function of the Ms map, the Ku map, the coupling field
        B_rms (3,) and the cavity drive amplitude.  forward runs the
        discrete adjoint once (llgc_adjoint: forward sweep with checkpoints,
        reverse sweep) and keeps its gradients; backward scales them by the
        incoming gradient."""

        @staticmethod
        def forward(ctx, ms_map, ku_map, brms, cdrive_amp, sim, m0, a0,
                    n_steps, n0, n1, stride):
            from . import inputs as I
            q = I.Problem(**{**sim.prob.__dict__})
            q.ms_map = ms_map.detach()
            q.ku1_map = ku_map.detach()
            q.brms = tuple(float(v) for v in brms.detach().cpu())
            q.cdrive_amp = float(cdrive_amp.detach())
            sim.set_params(q)
            sim.set_state(m0, 0.0, a0)
            g = sim.adjoint(n_steps, q.dt, n0, n1, stride)
            ctx.save_for_backward(
                g["g_ms"].reshape(ms_map.shape).to(ms_map.device,
                                                   ms_map.dtype),
                g["g_ku"].reshape(ku_map.shape).to(ku_map.device,
                                                   ku_map.dtype),
                torch.as_tensor(g["g_brms"], dtype=brms.dtype,
                                device=brms.device),
                torch.as_tensor(g["g_eps0"], dtype=cdrive_amp.dtype,
                                device=cdrive_amp.device))
            return torch.tensor(g["loss"], dtype=torch.float64,
                                device=ms_map.device)

        @staticmethod
        def backward(ctx, gl):
            gms, gku, gb, ge = ctx.saved_tensors
            return (gms * gl.to(gms.dtype), gku * gl.to(gku.dtype),
                    gb * gl.to(gb.dtype), ge * gl.to(ge.dtype),
                    None, None, None, None, None, None, None)

    _cavity_loss_cls = CavityLoss
    return CavityLoss


def cavity_loss(sim, m0, ms_map, ku_map, brms, cdrive_amp, n_steps, n0, n1,
                a0=0j, stride=0):
    """Differentiable windowed photon number (see CavityLoss).  `sim` is an
    RK4 context whose problem supplies everything else (its params and
    state are overwritten); `ms_map`, `ku_map` are tensors shaped
    (nz, ny, nx), `brms` a (3,) tensor in T, `cdrive_amp` a 0-d tensor;
    any of them may require grad.  Returns a 0-d float64 tensor."""
    return _cavity_loss_function().apply(
        ms_map, ku_map, brms, cdrive_amp, sim, m0, complex(a0), int(n_steps),
        int(n0), int(n1), int(stride))


class Batch:
    """Many problems of different sizes advanced together (llgc_batch_*).
    `sims[k]` is instance k, a `Sim` owned by the batch (set_state,
    get_state, set_params work on it as on a standalone context)."""

    def __init__(self, probs, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("llgc needs a GPU: no HIP device is visible")
        self.L = load()
        self.n = len(probs)
        self.stream = stream or torch.cuda.current_stream()
        grids = (Grid * self.n)(*[grid_of(p) for p in probs])
        h = ctypes.c_void_p()
        rc = self.L.llgc_batch_create(
            grids, self.n, ctypes.c_void_p(self.stream.cuda_stream),
            ctypes.byref(h))
        if rc != LLGC_OK:
            raise LLGCError(rc, "llgc_batch_create")
        self.h = h
        self.sims = []
        for k, p in enumerate(probs):
            hk = self.L.llgc_batch_instance(self.h, k)
            self.sims.append(Sim(p, self.stream, _handle=hk, _owner=self))

    def run(self, nsteps=0, t_end=0.0, record_every=0, rec_cap=0,
            check=True):
        """Runs every instance as `Sim.run` would.  Returns (records: list
        of (n_k, 6) arrays, infos: list of dicts, status: int32 array)."""
        if record_every > 0 and rec_cap <= 0:
            rec_cap = (nsteps // record_every + 2) if nsteps else 100000
        rec = np.zeros((self.n, max(rec_cap, 1), 6))
        nrec = (ctypes.c_int64 * self.n)()
        info = (RunInfo * self.n)()
        st = (ctypes.c_int32 * self.n)()
        rc = self.L.llgc_batch_run(
            self.h, int(nsteps), float(t_end), int(record_every),
            rec.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
            int(rec_cap), nrec, info, st)
        if check and rc < 0:
            msg = self.L.llgc_batch_last_error(self.h).decode()
            raise LLGCError(rc, f"llgc_batch_run: {msg}")
        recs = [rec[k, : nrec[k]].copy() for k in range(self.n)]
        infos = [dict(accepted=i.accepted, rejected=i.rejected,
                      rhs_evals=i.rhs_evals, t=i.t, dt=i.dt,
                      last_err=i.last_err) for i in info]
        return recs, infos, np.array(list(st), dtype=np.int32)

    def last_error(self):
        return self.L.llgc_batch_last_error(self.h).decode()

    def close(self):
        if getattr(self, "h", None):
            for s in self.sims:
                s.h = None
            self.L.llgc_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
