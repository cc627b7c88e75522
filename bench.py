"""Benchmark of the SS-CN hot path on one MI355X.

Workload: the 1024^2 FP64 real-time quench (dx = dy = 0.05, dt = 1e-4,
c0 = 2, c2 = +0.1, gamma = 0.8 with gamma p_x Sigma_x, Omega = 0.2) started
from the 256^2 imaginary-time ground state interpolated onto the grid, with
norm, magnetisation, energy and rms sizes taken every 100 steps.  A "step" is
one full SS-CN time step (CALCNU, HERM, SO, LUX, LUY) of the whole grid.

Prints one JSON line:
  value      grid-point-steps per second over the timed steps (state resident
             in HBM when the timed region starts; the observables are recorded
             into a device-side log inside the timed region and read after it;
             the warm-up runs the timed schedule untimed for at least 0.3 s, so
             every graph the timed steps replay is captured beforehand and the
             GPU runs at its working clocks);
  roofline   the dominant kernel's algorithmic bytes per launch over its mean
             duration (HIP start/stop events attached to its launches on the
             library's stream, every 7th step of a window of at least 50
             profiled steps after the timed one) against the 8 TB/s HBM peak;
  copy_ceiling  a device copy of the state (read + write) timed alike;
  cpu_baseline  the CPU oracle on the host cores, on a bounded sample of the
             same workload (first steps from the same initial state), with all
             threads and with one, and the CPU model.
Beside them: the forward+adjoint cost ratio, the batched-vs-serial
comparison, the imaginary-time workloads, the same 1024^2 workload under the
opt-in unitary-SO scheme (unitary_so) and Strang scheme (strang_step), with the
Rashba coupling (rashba_step)
and in complex64 (complex64_step, with its difference from complex128).

Usage: python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_PT_PASS = {"f64": 96, "f32": 48}   # one pass reads and writes 3 complex values
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_xpass_ypass_1024.json")
KERNEL_SOURCES = ["paper_2009_13507_amd/csrc/step_kernels.hpp", "paper_2009_13507_amd/csrc/cplx.hpp"]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, npts: int):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when it is missing or the kernel source has changed since."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("src_sha") != kernel_source_hash() or t.get("npts") != npts:
        return None
    return t.get("bytes_per_launch", {}).get(kernel)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_rate(oracle, cfg, psi0, seconds: float, max_steps: int):
    psi = psi0
    steps = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds and steps < max_steps:
        psi = oracle.step(cfg, psi, 1)
        steps += 1
    return steps, time.perf_counter() - t0


def cpu_baseline(w, psi0, seconds: float):
    """The oracle (plain FP64 C, OpenMP over grid lines) on the host cores:
    the first steps of the same workload from the same initial state, with all
    the threads the process may use and with one thread."""
    import oracle
    cfg = oracle.Cfg(dim=2, nx=w.nx, ny=w.ny, dx=w.dx, dy=w.dy, c0=w.c0, c2=w.c2, gamma=w.gamma,
                     omega=w.omega, dt=w.dt, imag=False, so=w.so)
    nthreads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    oracle.set_num_threads(nthreads)
    used = oracle.num_threads()
    steps, el = _oracle_rate(oracle, cfg, psi0, seconds, 400)
    oracle.set_num_threads(1)
    steps1, el1 = _oracle_rate(oracle, cfg, psi0, seconds / 2, 50)
    oracle.set_num_threads(used)
    npts = w.nx * w.ny
    return {"value": npts * steps / el, "unit": "grid-point-steps/s", "cores": used,
            "kind": "oracle",
            "sample": f"first {steps} steps of the 1024^2 real-time workload from its initial state "
                      f"({el:.1f} s, FP64, OpenMP over grid lines, {used} threads)",
            "single_thread": {"value": npts * steps1 / el1, "steps": steps1, "seconds": el1},
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}


def copy_ceiling(t, reps: int = 50):
    """A plain device copy of a state-sized buffer (read + write), timed with
    HIP events over reps copies: the practical floor of one pass."""
    import torch
    a = t.clone()
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / reps
    nbytes = 2 * a.numel() * a.element_size()
    return {"bytes_per_copy": nbytes, "us": us, "GBs": nbytes / (us * 1e-6) / 1e9,
            "frac_of_peak": nbytes / (us * 1e-6) / (HBM_PEAK_GBS * 1e9)}


def adjoint_ratio(reps: int = 2):
    """Forward and backward (recompute + adjoint) times of the differentiable
    512^2 real-time workload: 2000 steps, 100 Omega segments, checkpoints
    every ceil(sqrt(2000)) = 45 steps, loss = dA sum |psi_{+1}(T)|^2."""
    import time as _t

    import torch

    from paper_2009_13507_amd import autograd
    from paper_2009_13507_amd import workloads as W

    w = W.W2D_ADJ
    psi0 = W.interpolate(W.ground_256(), W.W2D_IMAG.nx, W.W2D_IMAG.dx, w.nx, w.dx)
    omega = W.omega_schedule(100, seed=2)
    prob = autograd.RealTimeProblem(dx=w.dx, dy=w.dy, dt=w.dt, steps=w.steps, steps_per_seg=w.steps // 100,
                                    c0=w.c0, c2=w.c2, gamma=w.gamma, so=w.so)
    dev = torch.device("cuda:0")
    best = None
    for _ in range(reps):
        p0 = torch.from_numpy(psi0).to(dev).requires_grad_(True)
        om = torch.tensor(omega, dtype=torch.float64, device=dev, requires_grad=True)
        torch.cuda.synchronize()
        t0 = _t.perf_counter()
        out = autograd.propagate(p0, om, prob)
        torch.cuda.synchronize()
        t1 = _t.perf_counter()
        loss = w.dx * w.dy * (out[0].abs() ** 2).sum()
        loss.backward()
        torch.cuda.synchronize()
        t2 = _t.perf_counter()
        cur = (t1 - t0, t2 - t1)
        if best is None or sum(cur) < sum(best):
            best = cur
    tf, tb = best
    return {"workload": w.name, "steps": w.steps, "omega_segments": 100, "checkpoint_every": prob.interval(),
            "t_forward_s": tf, "t_backward_s": tb, "R_b": tb / tf, "R_t": (tf + tb) / tf,
            "grad_norm_psi0": float(p0.grad.abs().pow(2).sum().sqrt()),
            "grad_omega_first": float(om.grad[0])}


def imag_workloads():
    """The two imaginary-time workloads: the 1D run (512 points, 20000 steps,
    the whole state in one workgroup's LDS) in full, and the 2D 256^2 SO +
    Rabi run over its first 2000 steps; steps/s, grid-point-steps/s and the
    energy reached."""
    import torch

    from paper_2009_13507_amd import api
    from paper_2009_13507_amd import workloads as W

    out = {}
    for w, psi0, steps in ((W.W1D, W.initial_1d(), W.W1D.steps), (W.W2D_IMAG, W.initial_2d_imag(), 2000)):
        state = torch.from_numpy(psi0).to("cuda:0")
        g = api.Grid(state, w.dx, w.dy if w.dim == 2 else None)
        g.set_params(c0=w.c0, c2=w.c2, gamma=w.gamma, omega=w.omega, dt=w.dt, so=w.so)
        g.step_imag(20)  # warm-up (tables, code objects)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.step_imag(steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        o = g.observables()
        g.close()
        out[w.name] = {"steps": steps, "steps_per_s": steps / el, "pt_steps_per_s": w.npts * steps / el,
                       "ms_per_step": 1e3 * el / steps, "E": o["E"], "N": o["N"]}
    return out


def unitary_so(steps: int = 1000, warmup: int = 50, every: int = 7):
    """The opt-in unitary-SO scheme on the 1024^2 real-time workload: step
    rate, x-pass and y-pass kernel times (HIP events on every `every`-th
    step), the x-pass rate on its algorithmic bytes, and the norm change over
    the run (exact to rounding under this scheme)."""
    import torch

    from paper_2009_13507_amd import api
    from paper_2009_13507_amd import workloads as W

    w = W.W2D_REAL
    psi0 = W.initial_2d_real(w)
    state = torch.from_numpy(psi0).to("cuda:0")
    g = api.Grid(state, w.dx, w.dy)
    g.set_params(c0=w.c0, c2=w.c2, gamma=w.gamma, omega=w.omega, dt=w.dt, so=w.so)
    g.set_scheme(api.SCHEME_UNITARY_SO)
    g.step_real(warmup)
    n0 = g.observables()["N"]
    g.profile(every, capacity=steps // every + 2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.step_real(steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    prof = g.profile_read()
    g.profile(0)
    n1 = g.observables()["N"]
    g.close()
    npts = w.nx * w.ny
    per_launch = BYTES_PER_PT_PASS["f64"] * npts
    return {"workload": w.name + " (unitary-SO scheme)", "steps": steps, "ms_per_step": 1e3 * el / steps,
            "pt_steps_per_s": npts * steps / el,
            "kernels_ms": {"xpass": prof["x_ms"], "ypass": prof["y_ms"], "profiled_steps": prof["steps"]},
            "xpass_achieved_GBs": per_launch / (prof["x_ms"] * 1e-3) / 1e9,
            "norm_change": n1 - n0}


def strang_step(steps: int = 1000, warmup: int = 50, every: int = 7):
    """The 1024^2 real-time workload under the opt-in Strang scheme (second
    order; the second-order pointwise stages merged into the x-pass, the
    joined x solve, the y-pass, and one closing pointwise pass per call):
    step rate, kernel times (HIP events on every `every`-th step) and the
    x-pass rate on its algorithmic bytes."""
    import torch

    from paper_2009_13507_amd import api
    from paper_2009_13507_amd import workloads as W

    w = W.W2D_REAL
    state = torch.from_numpy(W.initial_2d_real(w)).to("cuda:0")
    g = api.Grid(state, w.dx, w.dy)
    g.set_params(c0=w.c0, c2=w.c2, gamma=w.gamma, omega=w.omega, dt=w.dt, so=w.so)
    g.set_scheme(api.SCHEME_STRANG)
    g.step_real(warmup)
    n0 = g.observables()["N"]
    g.profile(every, capacity=steps // every + 2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.step_real(steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    prof = g.profile_read()
    g.profile(0)
    n1 = g.observables()["N"]
    g.close()
    npts = w.nx * w.ny
    per_launch = BYTES_PER_PT_PASS["f64"] * npts
    return {"workload": w.name + " (Strang scheme)", "steps": steps, "ms_per_step": 1e3 * el / steps,
            "pt_steps_per_s": npts * steps / el,
            "kernels_ms": {"xpass": prof["x_ms"], "ypass": prof["y_ms"], "profiled_steps": prof["steps"]},
            "xpass_achieved_GBs": per_launch / (prof["x_ms"] * 1e-3) / 1e9,
            "norm_change": n1 - n0}


def rashba_step(steps: int = 1000, warmup: int = 50, every: int = 7):
    """The 1024^2 real-time workload with the Rashba coupling (y derivatives
    in the SO term: the pointwise sub-steps and the SO update over 2D tiles
    into a scratch buffer, the x-pass with CN_x alone, the y-pass): step rate
    and the x-pass and y-pass kernel times (HIP events on every `every`-th
    step)."""
    import torch

    from paper_2009_13507_amd import api
    from paper_2009_13507_amd import workloads as W

    w = W.W2D_REAL
    state = torch.from_numpy(W.initial_2d_real(w)).to("cuda:0")
    g = api.Grid(state, w.dx, w.dy)
    g.set_params(c0=w.c0, c2=w.c2, gamma=w.gamma, omega=w.omega, dt=w.dt, so=api.SO_RASHBA)
    g.step_real(warmup)
    g.profile(every, capacity=steps // every + 2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.step_real(steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    prof = g.profile_read()
    g.profile(0)
    g.close()
    npts = w.nx * w.ny
    return {"workload": w.name + " (Rashba coupling)", "steps": steps, "ms_per_step": 1e3 * el / steps,
            "pt_steps_per_s": npts * steps / el,
            "kernels_ms": {"xpass": prof["x_ms"], "ypass": prof["y_ms"], "profiled_steps": prof["steps"]}}


def complex64_step(steps: int = 1000, warmup: int = 50):
    """The 1024^2 real-time workload in complex64 (FP32 storage and
    arithmetic): step rate, and the relative L2 difference from the same
    steps in complex128."""
    import torch

    from paper_2009_13507_amd import api
    from paper_2009_13507_amd import workloads as W

    w = W.W2D_REAL
    psi0 = W.initial_2d_real(w)
    out = {}
    for name, dt in (("c64", torch.complex64), ("c128", torch.complex128)):
        warm = torch.from_numpy(psi0).to("cuda:0").to(dt)
        g = api.Grid(warm, w.dx, w.dy)
        g.set_params(c0=w.c0, c2=w.c2, gamma=w.gamma, omega=w.omega, dt=w.dt, so=w.so)
        g.step_real(warmup)
        g.close()
        state = torch.from_numpy(psi0).to("cuda:0").to(dt)
        g = api.Grid(state, w.dx, w.dy)
        g.set_params(c0=w.c0, c2=w.c2, gamma=w.gamma, omega=w.omega, dt=w.dt, so=w.so)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.step_real(steps)
        torch.cuda.synchronize()
        out[name] = (time.perf_counter() - t0, state.to(torch.complex128))
        g.close()
    el, s64 = out["c64"]
    ref = out["c128"][1]
    npts = w.nx * w.ny
    return {"workload": w.name + " (complex64)", "steps": steps, "ms_per_step": 1e3 * el / steps,
            "pt_steps_per_s": npts * steps / el,
            "hbm_frac_step_algorithmic": 2 * BYTES_PER_PT_PASS["f32"] * npts * steps / el / (HBM_PEAK_GBS * 1e9),
            "rel_l2_vs_complex128": float(torch.linalg.vector_norm(s64 - ref) / torch.linalg.vector_norm(ref))}


def batch_compare(steps: int = 200, warmup: int = 20):
    """The 64-instance imaginary-time batch (sizes 128..512, seed-1 draw):
    batched (autotuned launch shape, graph replay) against one grid at a
    time, in complex128 and complex64, over a fixed window after warm-up;
    plus the complex64 error against complex128 after the same steps."""
    import numpy as np
    import torch

    from paper_2009_13507_amd import api
    from paper_2009_13507_amd import workloads as W

    draw = W.batch_draw(64, seed=1)
    states = [W.batch_initial(w, ph) for w, ph in draw]
    prm = [api.params(c0=w.c0, c2=w.c2, gamma=w.gamma, omega=w.omega, dt=w.dt, so=w.so) for w, _ in draw]
    dxs = [w.dx for w, _ in draw]
    npts = sum(w.nx * w.ny for w, _ in draw)
    out = {"workload": "64 instances, N in {128,192,256,384,512}, seed 1, imaginary time, "
                       "gamma p_x Sigma_x", "points": npts, "steps": steps}
    finals = {}
    for name, tdt in (("c128", torch.complex128), ("c64", torch.complex64)):
        b = api.Batch.from_states(states, dxs, prm, dtype=tdt)
        b.step_imag(warmup)  # the first call runs the launch-shape tuner
        b.sync()
        t0 = time.perf_counter()
        b.step_imag(steps)
        b.sync()
        t_b = time.perf_counter() - t0
        b.step_imag_serial(warmup)
        b.sync()
        t0 = time.perf_counter()
        b.step_imag_serial(steps)
        b.sync()
        t_s = time.perf_counter() - t0
        info = b.info()
        bpp = BYTES_PER_PT_PASS["f64" if name == "c128" else "f32"]
        v_b, v_s = npts * steps / t_b, npts * steps / t_s
        out[name] = {"batched_pt_steps_per_s": v_b, "serial_pt_steps_per_s": v_s, "speedup": v_b / v_s,
                     "ms_per_step_batched": 1e3 * t_b / steps, "ms_per_step_serial": 1e3 * t_s / steps,
                     "launch_shape": info["shape"], "persistent_workgroups": info["grid"],
                     "tuned_us_per_step": info["us_per_step"],
                     "hbm_frac_algorithmic": 2 * bpp * v_b / (HBM_PEAK_GBS * 1e9)}
        finals[name] = ([v.cpu().to(torch.complex128).numpy() for v in b.views()],
                        [o["E"] for o in b.observables()])
        b.close()
    errs = [float(np.linalg.norm(a - c) / np.linalg.norm(c)) for a, c in zip(finals["c64"][0], finals["c128"][0])]
    dE = [abs(a - c) for a, c in zip(finals["c64"][1], finals["c128"][1])]
    out["c64_vs_c128"] = {"max_rel_l2": max(errs), "max_abs_dE": max(dE),
                          "after_steps": 2 * (steps + warmup)}
    return out


def progress(msg: str) -> None:
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--warmup-seconds", type=float, default=0.3,
                    help="after the W warm-up steps, repeat the timed schedule untimed for at least this long")
    ap.add_argument("--obs-every", type=int, default=100)
    ap.add_argument("--dtype", choices=["f64", "f32"], default="f64")
    ap.add_argument("--profile-every", type=int, default=0,
                    help="in the kernel-timing window after the timed one, time the kernels of every n-th "
                         "step (default 7)")
    ap.add_argument("--profile-steps", type=int, default=50, help="profiled steps (at least 50)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the forward+adjoint cost ratio")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-vs-serial comparison")
    ap.add_argument("--no-uso", action="store_true", help="skip the unitary-SO scheme and Rashba-coupling figures")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run torch copies of the state size (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the stepper has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2009_13507_amd import api
    from paper_2009_13507_amd import workloads as W

    w = W.W2D_REAL
    psi0 = W.initial_2d_real(w)
    dev = torch.device("cuda:0")
    tdtype = torch.complex128 if args.dtype == "f64" else torch.complex64
    init = torch.from_numpy(psi0).to(dev).to(tdtype)
    state = init.clone()
    g = api.Grid(state, w.dx, w.dy)
    g.set_params(c0=w.c0, c2=w.c2, gamma=w.gamma, omega=w.omega, dt=w.dt, so=w.so)

    K = args.steps
    nobs = K // args.obs_every + 1
    g.obs_log_reserve(nobs)

    def run(k):
        """k steps with the observables of the state after steps 0, obs_every,
        2 obs_every, ... recorded on the device (no host synchronisation)."""
        g.obs_record()
        done = 0
        while done < k:
            n = min(args.obs_every - done % args.obs_every, k - done)
            g.step_real(n)
            done += n
            if done % args.obs_every == 0:
                g.obs_record()

    # warm-up: W steps, then the timed schedule, repeated for at least
    # --warmup-seconds of wall time (every graph length it replays is
    # captured beforehand, and the GPU leaves its idle clocks); then back to
    # the initial state
    g.step_real(args.warmup)
    torch.cuda.synchronize()
    tw = time.perf_counter()
    while True:
        g.obs_log_reserve(nobs)
        run(K)
        torch.cuda.synchronize()
        if time.perf_counter() - tw >= args.warmup_seconds:
            break
    g.obs_log_reserve(nobs)
    state.copy_(init)
    g.step_index = 0
    torch.cuda.synchronize()

    t0 = time.perf_counter()
    run(K)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    obs_log = g.obs_log_read()
    progress(f"timed {K} steps: {1e3 * el / K:.4f} ms/step")

    # kernel times: a separate window after the timed one, HIP start/stop
    # events attached to the x-pass and y-pass launches of every 7th step
    # (the others replayed as graphs), at least 50 profiled steps
    every = args.profile_every if args.profile_every > 0 else 7
    nprof = max(50, args.profile_steps)
    g.profile(every, capacity=nprof + 2)
    g.step_real(every * nprof)
    prof = g.profile_read()
    g.profile(0)

    npts = w.nx * w.ny
    value = npts * K / el
    bpp = BYTES_PER_PT_PASS[args.dtype]
    per_launch = bpp * npts
    kern = "xpass" if prof["x_ms"] >= prof["y_ms"] else "ypass"
    mean_ms = max(prof["x_ms"], prof["y_ms"])
    achieved = per_launch / (mean_ms * 1e-3) / 1e9
    traffic = measured_traffic(kern, npts)
    ceiling = copy_ceiling(init)

    line = {
        "metric": "2D SS-CN grid-point-steps/s, 1024^2 FP64, % of HBM peak; fwd+adjoint cost ratio",
        "value": value,
        "unit": "grid-point-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": el * 1e3 / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": w.name, "nx": w.nx, "ny": w.ny, "dx": w.dx, "dt": w.dt,
                   "c0": w.c0, "c2": w.c2, "gamma": w.gamma, "so": "gamma p_x Sigma_x",
                   "omega": w.omega, "observables_every": args.obs_every,
                   "initial_state": "256^2 imaginary-time ground state, linearly interpolated"},
        "hbm_frac_step_algorithmic": 2 * bpp * value / (HBM_PEAK_GBS * 1e9),
        "kernels_ms": {"xpass": prof["x_ms"], "ypass": prof["y_ms"], "profiled_steps": prof["steps"],
                       "profile_every": every},
        "roofline": {"bound": "hbm", "kernel": kern, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "algorithmic_bytes_per_launch": per_launch},
        "copy_ceiling": dict(ceiling, kernel_frac_of_copy=achieved / ceiling["GBs"]),
        "observable_samples": len(obs_log),
        "final_observables": {k: obs_log[-1][k] for k in ("N", "M", "E", "rms")},
    }
    progress("kernel timing window and copy ceiling done")
    if not args.no_adjoint and args.dtype == "f64":
        line["adjoint_cost_ratio"] = adjoint_ratio()
        progress("adjoint cost ratio done")
    if not args.no_uso and args.dtype == "f64":
        line["unitary_so"] = unitary_so()
        line["strang_step"] = strang_step()
        line["rashba_step"] = rashba_step()
        progress("unitary-SO, Strang and Rashba legs done")
    if not args.no_batch and args.dtype == "f64":
        line["complex64_step"] = complex64_step()
        progress("complex64 leg done")
    if not args.no_batch:
        line["batch_c4"] = batch_compare()
        progress("batch leg done")
        line["imag_workloads"] = imag_workloads()
        progress("imaginary-time workloads done")
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(w, psi0, args.cpu_seconds)
        progress("CPU baseline done")
    print(json.dumps(line), flush=True)
    g.close()


if __name__ == "__main__":
    main()
