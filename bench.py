"""Benchmark: cavity-LLG cell-steps/s on one MI355X.

Workload: textured film, 1024 x 1024 x 2 cells of 4 nm (Ms 8e5 A/m,
A 1.3e-11 J/m), 64 seeded vortex/domain-wall centres relaxed for 0.5 ns at
alpha = 0.5 (untimed), then alpha = 0.02, B_ext 20 mT along x, one cavity mode
at 4.01 GHz coupled with g/omega_c = 0.005, Dormand-Prince 5(4) at tol 1e-6,
float32 state.  A step is one accepted adaptive step of the whole path:
demag (zero-padded FFT convolution), exchange, anisotropy, Zeeman and cavity
fields, LL torque, stage combination, error-norm reduction, step control and
renormalisation.  Inputs are resident in HBM when timing starts.

Prints one JSON line.  `value` = cells * accepted steps / wall seconds.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

METRIC = ("cavity-LLG cell-steps/s (fwd; fwd+adjoint; batched vs plain), "
          "% HBM peak")


def kernel_bytes(plan, prob, method, kernel, fused=False):
    """Algorithmic HBM bytes of one launch of `kernel`, averaged over its
    launches in one step (every array read or written once).  `fused`: the
    run fused the forward x pass of stage s+1 into the field pass of stage s
    (k_xfield_fwd), leaving k_xfield for the last stage only."""
    N = prob.ncells
    nx, ny, nz = prob.nx, prob.ny, prob.nz
    Px, Py = plan["Px"], plan["Py"]
    Hx, Hy = Px // 2 + 1, Py // 2 + 1
    spec = Hx * nz * 3 * ny * 8
    # kernel coefficients: six tensor components per z offset, less the xz
    # and yz ones at offset 0, which vanish (odd in the z offset)
    kern = Hx * Hy * (6 * nz - 2) * 4
    state = 12 * N

    def field(s):
        """Field pass of stage s: spectrum in, y_s, k_s out, the earlier
        k's, and (except the last stage) y_n in and y_{s+1} out."""
        if method == "dp45":
            prev = {2: 1, 3: 2, 4: 3, 5: 4, 6: 4, 7: 5}[s]
            return (spec + 2 * state + (0 if s == 7 else 2 * state)
                    + prev * state)
        return spec + 2 * state + (2 * state if s < 4 else 4 * state)

    stages = list(range(2, 8)) if method == "dp45" else list(range(1, 5))
    if kernel in ("k_xfwd", "k_xfwd_fx"):
        return state + spec
    if kernel == "k_yspec":
        return 2 * spec + kern
    if kernel == "k_xfield_fwd":
        # the field pass of every stage but the last, plus the next stage's
        # half spectrum (its input y_{s+1} is this kernel's own output)
        per = [field(s) + spec for s in stages[:-1]]
        return sum(per) / len(per)
    if kernel == "k_xfield":
        per = [field(stages[-1])] if fused else [field(s) for s in stages]
        return sum(per) / len(per)
    if kernel in ("k_begin", "k_step_begin"):
        return 5 * state
    if kernel == "k_record":
        return state
    return 0


def _counter_line(tag, kernel):
    """Value of `tag kernel V sources H` in the committed counter summary
    when H is the hash of the library sources as they are now, else None."""
    import glob
    import hashlib
    path = os.path.join(ROOT, "profiles", "film_1024x1024x2_hbm_counters.md")
    if not os.path.exists(path):
        return None
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2410_00966_amd",
                                           "csrc", "*"))):
        with open(f, "rb") as fh:
            h.update(fh.read())
    for line in open(path):
        w = line.split()
        if (len(w) == 5 and w[0] == tag and w[1] == kernel
                and w[3] == "sources"):
            return float(w[2]) if w[4] == h.hexdigest()[:16] else None
    return None


def counted_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, if it was taken on the library sources as they are now;
    otherwise None (the kernel changed since the counters were taken)."""
    return _counter_line("traffic_bytes_per_launch", kernel)


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(prob, m0, dt, nsteps=3):
    """The oracle on the same workload and state: `nsteps` Dormand-Prince
    steps (six right-hand-side evaluations each, FSAL, at the step size the
    GPU run settled on) timed on the host; tensor and FFT-kernel set-up and
    the first stage of the first step are outside the timing.  numpy's FFT
    and elementwise kernels run on one thread."""
    from oracle.llg import CavityLLG, normalise
    o = CavityLLG(prob, demag="fft")
    m = m0.astype(np.float64)
    a = 0j
    km, ka = o.rhs(m, a, 0.0)
    t = 0.0
    t0 = time.perf_counter()
    for _ in range(nsteps):
        m5, a5, _, km, ka = o.dp45_attempt(m, a, t, dt, km, ka)
        m, a, t = normalise(m5), a5, t + dt
    el = time.perf_counter() - t0
    return dict(value=prob.ncells * nsteps / el, unit="cell-steps/s",
                cores=1, kind="oracle",
                nproc=os.cpu_count(), cpu_model=_cpu_model(),
                sample=(f"{nsteps} Dormand-Prince steps ({6 * nsteps} "
                        "right-hand-side evaluations, numpy float64, one "
                        f"thread) of the relaxed {prob.nx}x{prob.ny}x"
                        f"{prob.nz} film at dt = {dt:.3g} s: {el:.1f} s"))


def bench_batched(torch, t_end, n_plain):
    """The 512-instance size/coupling sweep (grids U{16..128}^2 x U{1..4} of
    5 nm cells, Dormand-Prince tol 1e-6) as one batch, against a sample of
    the same instances solved one after another with standalone contexts.
    Set-up (contexts, demag kernels) is outside both timed regions."""
    from paper_2410_00966_amd import inputs as I
    from paper_2410_00966_amd.llgc import Batch, Sim
    inst = I.c4_instances()
    probs = [p for p, _, _ in inst]
    m0s = [m0 for _, m0, _ in inst]
    t_set = time.perf_counter()
    b = Batch(probs)
    for s, m0 in zip(b.sims, m0s):
        s.set_state(torch.from_numpy(m0))
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t_set
    t0 = time.perf_counter()
    _, infos, st = b.run(t_end=t_end)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    assert (st == 0).all(), st
    cs = sum(p.ncells * i["accepted"] for p, i in zip(probs, infos))
    b.close()
    idx = np.linspace(0, len(probs) - 1, n_plain).round().astype(int)
    wall_p, cs_p = 0.0, 0
    kinds = []
    for k in idx:
        s = Sim(probs[k])
        s.set_state(torch.from_numpy(m0s[k]))
        kinds.append(s.autotune(reps=5))       # untimed: best plain plan
        s.run(nsteps=1, t_end=t_end)           # untimed: graph capture
        s.set_state(torch.from_numpy(m0s[k]))
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, info = s.run(t_end=t_end)
        torch.cuda.synchronize()
        wall_p += time.perf_counter() - t1
        cs_p += probs[k].ncells * info["accepted"]
        s.close()
    rate_b, rate_p = cs / wall, cs_p / wall_p
    return {
        "workload": ("512 ragged instances, grids U{16..128}^2 x U{1..4} of "
                     "5 nm, g/wc log-uniform 1e-3..1e-1, Bz U(0,0.3) T, "
                     f"wc/2pi 5..15 GHz, Dormand-Prince tol 1e-6 to "
                     f"{t_end * 1e12:g} ps"),
        "value": rate_b, "unit": "cell-steps/s",
        "cells": int(sum(p.ncells for p in probs)),
        "accepted_total": int(sum(i["accepted"] for i in infos)),
        "wall_s": wall, "setup_s": round(setup_s, 2),
        "plain": {"value": rate_p, "unit": "cell-steps/s",
                  "sample": (f"{len(idx)} evenly spaced instances solved one "
                             "after another, standalone contexts with "
                             "autotuned plans (tuning and graph capture "
                             "untimed)"),
                  "plan_kinds": kinds,
                  "wall_s": wall_p},
        "speedup_vs_plain": rate_b / rate_p,
    }


def bench_wire(torch, nsteps):
    """Nanowire 512x32x4 of 4 nm (Ku along x, cavity at its uniform mode,
    sinc cavity drive), Dormand-Prince tol 1e-6: forward cell-steps/s."""
    from paper_2410_00966_amd import inputs as I
    from paper_2410_00966_amd.llgc import Sim
    p, m0, _ = I.c2_nanowire()
    s = Sim(p)
    s.set_state(torch.from_numpy(m0))
    kind = s.autotune(reps=10)                         # untimed
    s.run(nsteps=20, t_end=1.0)                        # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, info = s.run(nsteps=nsteps, t_end=1.0)
    torch.cuda.synchronize()
    w = time.perf_counter() - t0
    s.close()
    return {"workload": ("nanowire 512x32x4 cells of 4 nm, Ku 5e3 J/m^3 x, "
                         "cavity at the uniform mode, g/wc=0.02, sinc cavity "
                         "drive, Dormand-Prince tol 1e-6"),
            "value": p.ncells * info["accepted"] / w, "unit": "cell-steps/s",
            "accepted": info["accepted"], "rejected": info["rejected"],
            "ms_per_step": 1e3 * w / info["accepted"], "plan_kind": kind}


def bench_adjoint(torch, nsteps):
    """256x256x2 film with Ms and Ku maps, RK4 dt 1e-13 s: forward alone and
    forward with checkpoints + discrete adjoint of the loss
    mean |alpha_n|^2 over the last fifth of the steps."""
    from paper_2410_00966_amd import inputs as I
    from paper_2410_00966_amd.llgc import Sim
    p, m0, _ = I.c5_adjoint()
    s = Sim(p)
    s.set_state(torch.from_numpy(m0))
    s.run(nsteps=20)                                   # warm-up
    s.set_state(torch.from_numpy(m0))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.run(nsteps=nsteps)
    torch.cuda.synchronize()
    w_f = time.perf_counter() - t0
    s.set_state(torch.from_numpy(m0))
    n0 = nsteps - nsteps // 5 + 1
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g = s.adjoint(nsteps, p.dt, n0, nsteps)
    torch.cuda.synchronize()
    w_a = time.perf_counter() - t0
    s.close()
    assert np.isfinite(g["loss"]) and np.isfinite(g["g_brms"]).all()
    return {
        "workload": ("256x256x2 cells of 4 nm, seeded Ms/Ku maps, cavity "
                     f"9.31 GHz, RK4 dt 1e-13 s, {nsteps} steps, loss over "
                     f"steps {n0}..{nsteps}"),
        "fwd_value": p.ncells * nsteps / w_f,
        "fwd_adjoint_value": p.ncells * nsteps / w_a,
        "unit": "cell-steps/s", "steps": nsteps,
        "fwd_s": w_f, "fwd_adjoint_s": w_a,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--relax-ns", type=float, default=0.5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=3)
    ap.add_argument("--no-timing", action="store_true",
                    help="skip per-kernel events (for profiler runs)")
    ap.add_argument("--time-all", action="store_true",
                    help="event every kernel in the timed region (default: "
                         "only the dominant one)")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batch-t-end", type=float, default=2e-9)
    ap.add_argument("--batch-plain", type=int, default=32)
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the default plan (profiling runs: no tuning "
                         "launches in the counters)")
    ap.add_argument("--no-wire", action="store_true")
    ap.add_argument("--wire-steps", type=int, default=400)
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--adjoint-steps", type=int, default=50000)
    ap.add_argument("--only", choices=("film", "adjoint", "batched"),
                    help="run one leg alone (for profiler runs)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy 256 MiB device to device 5 times (the "
                         "reference kernel for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not "
              "supported (the path is single-GPU by design).",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2410_00966_amd import inputs as I
    from paper_2410_00966_amd.llgc import Sim

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_probe:
        # 512 MiB copies; before each, 1 GiB of unrelated writes evicts the
        # source from the 256 MB last-level (Infinity) cache so the copy's
        # reads come from HBM
        x = torch.ones(128 * 2 ** 20, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        flush = torch.empty(256 * 2 ** 20, dtype=torch.float32, device="cuda")
        for _ in range(3):
            flush.fill_(2.0)
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": x.numel() * 4,
                          "copy_probe_bytes_written": y.numel() * 4,
                          "launches": 3}))
        return
    if args.only == "adjoint":
        print(json.dumps({"adjoint": bench_adjoint(torch,
                                                   args.adjoint_steps)}))
        return
    if args.only == "batched":
        print(json.dumps({"batched": bench_batched(
            torch, args.batch_t_end, args.batch_plain)}))
        return
    if args.only == "film":
        args.no_adjoint = args.no_batched = args.no_cpu_baseline = True
        args.no_wire = True
    prob, m0, cfg = I.c3_film()
    brms = prob.brms
    # --- relaxation (untimed): alpha 0.5, no cavity coupling
    relax = I.Problem(**{**prob.__dict__})
    relax.alpha = cfg["relax_alpha"]
    relax.brms = (0.0, 0.0, 0.0)
    t_setup = time.perf_counter()
    sim = Sim(relax)
    sim.set_state(torch.from_numpy(m0))
    if args.relax_ns > 0:
        _, rinfo = sim.run(t_end=args.relax_ns * 1e-9)
    else:
        rinfo = dict(accepted=0, rejected=0)
    m_relaxed, _, _ = sim.get_state()
    # --- coupled run parameters; t <- 0, alpha <- 0
    prob.brms = brms
    sim.set_params(prob)
    sim.set_state(m_relaxed, 0.0, 0j)
    kind = sim.autotune(reps=0 if args.no_tune else 10)   # plan kinds timed
    plan = sim.plan_info()
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t_setup
    # --- warmup (untimed); with per-kernel events, to find the dominant
    # kernel, whose launches alone are then timed inside the timed region
    dom = None
    if not args.no_timing:
        sim.set_timing(True)
        sim.kernel_times(reset=True)
    winfo = None
    if args.warmup > 0:
        _, winfo = sim.run(nsteps=args.warmup, t_end=1.0)
    if not args.no_timing:
        kw = sim.kernel_times(reset=True)
        kw = kw or {"k_yspec": (1.0, 1)}
        fused = "k_xfield_fwd" in kw
        dom = max(kw, key=lambda k: kw[k][0])
        sim.set_timing(True, only=None if args.time_all else dom)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, info = sim.run(nsteps=args.steps, t_end=1.0)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    assert info["accepted"] == args.steps, info
    value = prob.ncells * args.steps / wall
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": ("textured film 1024x1024x2 cells of 4 nm, 64 "
                         "vortex/domain-wall centres relaxed 0.5 ns at "
                         "alpha=0.5, then alpha=0.02, Bext 20 mT x, cavity "
                         "4.01 GHz g/wc=0.005, Dormand-Prince tol 1e-6"),
            "cells": prob.ncells, "padded_fft": [plan["Px"], plan["Py"]],
            "method": "dp45", "tol": prob.tol,
            "accepted": info["accepted"], "rejected": info["rejected"],
            "rhs_evals": info["rhs_evals"],
            "relax_steps": rinfo["accepted"], "setup_s": round(setup_s, 2),
            "plan_kind": kind,
        },
    }
    if not args.no_timing:
        kt = sim.kernel_times()
        ms, n = kt[dom]
        # a run capped at K accepted steps queues only the attempts it can
        # still use, so every stage-kernel launch of the timed region does
        # work when no attempt is rejected: launches == right-hand sides
        per_launch_s = ms * 1e-3 / n
        byts = kernel_bytes(plan, prob, "dp45", dom, fused)
        achieved = byts / per_launch_s / 1e9
        out["roofline"] = {
            "bound": "hbm", "kernel": dom,
            "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": counted_traffic(dom),
            # fraction of the launch the SIMDs spend issuing its VALU
            # instructions (counted; the kernel's actual limiter)
            "valu_issue_frac": _counter_line("valu_issue_frac_per_launch",
                                             dom),
            "bytes_per_launch": byts, "avg_launch_us": per_launch_s * 1e6,
            "launches": n, "rhs_evals": info["rhs_evals"],
        }
        # per-kernel table from the warm-up (all kernels timed there).
        # Model bytes per step count the launches that did work: one per
        # right-hand-side evaluation for the stage kernels, one per attempt
        # for the step kernels (launches queued past the end of a run exit
        # at once on the device flag and move no data).
        wi = winfo or info
        acc = max(1, wi["accepted"])
        # launches per accepted step as counted in the warm-up (every
        # launch of a step-capped run does work)
        sb = sum(kernel_bytes(plan, prob, "dp45", k, fused) * v[1] / acc
                 for k, v in kw.items())
        out["kernels"] = {k: {"ms": round(v[0], 3), "launches": v[1],
                              "us_per_launch": round(1e3 * v[0] / v[1], 2)}
                          for k, v in kw.items()}
        out["kernels_note"] = ("per-kernel table from the warm-up steps (all "
                               "kernels evented); the timed region events "
                               f"only {dom}")
        out["model_bytes_per_step"] = sb
        out["effective_GBs"] = sb * args.steps / wall / 1e9
    sim.close()
    if not args.no_wire:
        out["wire"] = bench_wire(torch, args.wire_steps)
    if not args.no_adjoint:
        out["adjoint"] = bench_adjoint(torch, args.adjoint_steps)
    if not args.no_batched:
        out["batched"] = bench_batched(torch, args.batch_t_end,
                                       args.batch_plain)
    if not args.no_cpu_baseline:
        m_host = m_relaxed.cpu().numpy()
        out["cpu_baseline"] = cpu_baseline(prob, m_host, info["dt"],
                                           args.cpu_steps)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
