"""Benchmark of the random batch Ewald hot path on one MI355X.

Workload: N = 1e5 ions (+-1) at density 0.1 (L = 100), r_c = 3.5, P = 100
modes per step, alpha from the 1e-4 real-space error estimate, shifted LJ
(eps = 1, sigma = 1, cut 2.5), Langevin kT = 1, gamma = 1, dt = 1e-3, float32
arithmetic with double phases.  Inputs are synthetic and resident on the GPU
before timing starts.

A timed "step" is one pass of the whole hot path: a fresh batch of P modes,
structure factors, the Fourier force, the neighbour list (rebuilt on the
device when particles have moved far enough), the real-space + LJ force and
the Langevin update; the K timed steps are one rbe_step call.  The headline
value is N*P*steps / elapsed seconds over those full steps.  The JSON line also reports MD steps/s, the
Fourier-only pair rate (sample + structure factor + force), per-kernel
durations from HIP events on the library's stream, the ALU roofline of every
kernel of the step (the longest one as "roofline"), and the FP64 CPU oracle
timed on the host.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
                       [--autotune] [--calibrate-copy] [--graphs]
       python bench.py --suite PATH   (N x P sweep, batched vs loop,
                                       forward vs backward, classical Ewald)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "k-space particle–mode pairs/s (N·P) + MD steps/s at N=1e5, P=100, 1 GPU"

# Algorithmic work in FP32 VALU issue slots (an FP64 add/mul/FMA takes 2, a
# transcendental op 4) and the chip's FP32 vector peak: 256 CUs x 128 FP32
# lanes/clock x 2 flop x 2.4 GHz.  One slot counts as 2 flop.
# Per particle-mode pair, with the phase of the exact-wrap FP32 scheme
# (theta = fract(m . s_hi) + m . s_lo: 3 products, 1 fract, 3 FMA, 1 add):
SLOTS_PHASE = 8
SLOTS_RHO = SLOTS_PHASE + 2 * 4 + 2           # phase, sin+cos, 2 FMA into (C, S)
SLOTS_FORCE = SLOTS_PHASE + 2 * 4 + 2 + 3     # phase, sin+cos, cos S - sin C, 3 FMA into F
# Real space, per neighbour-list entry (3 integer differences, 3
# conversions, |d|^2, compare) and per pair inside the cutoff (displacement,
# rsqrt, exp, the erfc rational form with its reciprocal, Coulomb and LJ
# factors, force accumulation); both counted over ordered pairs.
SLOTS_CHECK = 10
SLOTS_PAIR = 6 + 3 + 3 * 4 + 3 + 5 + 9 + 4 + 3 + 6 + 6
PEAK_FP32_TFLOPS = 157.3

# HBM traffic per launch from two rocprofv3 --pmc passes (FETCH_SIZE, then
# WRITE_SIZE, KiB per dispatch, averaged over the launches of the profiled
# run), each multiplied by the ratio of the true size of a 256 MiB device
# copy to what the same counter reads for it.  Valid only for the kernel
# source it was taken on (sha256 prefix); otherwise reported as null.
# "stage" is the time-step variant of k_stage_rho, "stage_fourier" the
# variant of force calls that also draws the modes recorded by rbe_sample_k.
TRAFFIC = {
    "real": {"fetch_kib": 9011.6, "write_kib": 7812.9, "fetch_scale": 2.0, "write_scale": 1.0,
             "src": "bb2bd7dfd861268b"},
    "stage": {"fetch_kib": 3155.2, "write_kib": 7168.7, "fetch_scale": 2.0, "write_scale": 1.0,
              "src": "aefb4ec43f9b949a"},
    "stage_fourier": {"fetch_kib": 916.8, "write_kib": 402.0, "fetch_scale": 2.0, "write_scale": 1.0,
                      "src": "aefb4ec43f9b949a"},
    "kforce": {"fetch_kib": 940.9, "write_kib": 1171.9, "fetch_scale": 2.0, "write_scale": 1.0,
               "src": "aefb4ec43f9b949a"},
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--autotune", action="store_true", help="pick the Fourier tile shapes by timing")
    ap.add_argument("--suite", metavar="PATH", help="run the sweep/batched/gradient/Ewald suite into PATH instead")
    ap.add_argument("--graphs", action="store_true", help="replay the steady-state steps from hipGraphs")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one 256 MiB device copy first (reference for HBM byte counters)")
    return ap.parse_args()


def cpu_baseline(s, modes, budget_s):
    """Time the FP64 oracle's Fourier evaluation (structure factor + force) on
    the metric workload: whole evaluations at N = 1e5, P = 100 repeated until
    the budget is spent, with every host thread, then single-threaded."""
    import oracle as O
    O.build()
    pos = s.pos.astype(np.float32).astype(np.float64)
    q = s.q
    w = O.rbe_weights(s.alpha, s.L, s.p)
    O.rbe_kspace_force(pos[:, :1000], q[:1000], s.L, s.alpha, modes)  # load + warm

    def rate(budget):
        reps, t0 = 0, time.perf_counter()
        while True:
            O.kspace_force(pos, q, s.L, modes, w)
            reps += 1
            el = time.perf_counter() - t0
            if el > budget or reps >= 1000:
                return s.n * s.p * reps / el, reps, el

    threads = O.set_threads(0)
    v, reps, el = rate(budget_s)
    O.set_threads(1)
    v1, reps1, el1 = rate(budget_s / 2)
    O.set_threads(threads)
    return {"value": v, "unit": "pairs/s", "cores": threads, "kind": "oracle",
            "sample": f"{reps} full Fourier evaluations (structure factor + force, FP64) of the N={s.n}, "
                      f"P={s.p} workload in {el:.1f} s on {threads} threads; single-threaded {reps1} "
                      f"in {el1:.1f} s",
            "single_thread_value": v1, "host_cpu": _cpu_model()}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def real_space_counts(s, skin):
    """Ordered pairs within the largest cutoff plus the list skin (the list
    entries a step tests) and within the largest cutoff, for the initial
    configuration."""
    from scipy.spatial import cKDTree
    rmax = max(s.r_cut, s.lj[2] * s.lj[1]) if s.lj[0] > 0 else s.r_cut
    tree = cKDTree(np.mod(s.pos, s.L).T, boxsize=s.L)
    entries = 2 * len(tree.query_pairs(rmax + skin, output_type="ndarray"))
    pairs = 2 * len(tree.query_pairs(rmax, output_type="ndarray"))
    return entries, pairs


def source_sha(name):
    """Hash of a kernel source together with the headers it includes."""
    h = hashlib.sha256()
    for part in (name, "rbe_device.h", "rbe_internal.h", "rbe_roles.h"):
        with open(os.path.join(ROOT, "paper_2010_01559_amd", "csrc", part), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


KERNEL_SOURCE = {"stage": "rbe_kspace.hip", "stage_fourier": "rbe_kspace.hip", "mid": "rbe_kspace.hip",
                 "kforce": "rbe_kspace.hip", "sample": "rbe_kspace.hip", "real": "rbe_real.hip"}


def traffic_for(name):
    t = TRAFFIC.get(name)
    if not t or t["src"] != source_sha(KERNEL_SOURCE[name]):
        return None
    return round((t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"]) * 1024)


# ---------------------------------------------------------------------------
# Suite (--suite PATH): the N x P sweep, batched replicas against a loop of
# single-system calls, the differentiable form, and classical Ewald on the
# same kernels.  Written to PATH as one JSON document.
# ---------------------------------------------------------------------------

def _timed(torch, stream, fn, reps):
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for k in range(reps):
        fn(k)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def _kernel_us(R, ctx, fn, reps):
    R.rbe_profile_enable(ctx, True)
    for k in range(reps):
        fn(k)
    prof = R.rbe_profile_read(ctx)
    R.rbe_profile_enable(ctx, False)
    return {name: 1e3 * ms / n for name, (ms, n) in prof.items() if n}


def _frac(slots, us):
    ach = slots * 2 / (us * 1e-6) / 1e12
    return {"achieved": round(ach, 3), "frac": round(ach / PEAK_FP32_TFLOPS, 4), "avg_launch_us": round(us, 2)}


def suite_np_sweep(torch, R, W, log):
    """N in {1e4, 1e5, 1e6} x P in {50, 100, 200, 500}: Fourier-only pairs/s
    (sample + structure factor + force), MD steps/s, and the ALU roofline of
    the structure-factor and force launches."""
    out = []
    for n in (10000, 100000, 1000000):
        s = W.metric_system() if n == 100000 else W.scaling_system(n, 100)
        for p in (50, 100, 200, 500):
            ctx = R.rbe_create(R.params_from_system(s, R.RBE_FP32, p=p))
            P = R.to_device(s.pos, ctx)
            Q = R.to_device(s.q, ctx)
            V = R.to_device(s.vel, ctx)
            F = torch.zeros_like(P)
            R.rbe_sample_k(ctx, 0)
            R.rbe_kspace_forces(ctx, P, Q, F)
            R.rbe_real_forces(ctx, P, Q, F, accumulate=True)

            def four(k):
                R.rbe_sample_k(ctx, 1000 + k)
                R.rbe_kspace_forces(ctx, P, Q, F)

            four(0)
            k_ms = _timed(torch, ctx.stream, four, 100)
            kus = _kernel_us(R, ctx, four, 50)
            R.rbe_step(ctx, P, V, Q, F, 1, 20)
            st_ms = _timed(torch, ctx.stream, lambda k: R.rbe_step(ctx, P, V, Q, F, 21 + 100 * k, 100), 1) / 100
            pairs = n * p
            row = {"n": n, "p": p, "kspace_pairs_per_s": pairs * 1e3 / k_ms, "kspace_ms": k_ms,
                   "md_steps_per_s": 1e3 / st_ms, "md_pairs_per_s": pairs * 1e3 / st_ms, "md_ms": st_ms,
                   "stage": _frac(pairs * SLOTS_RHO, kus["stage"]), "kforce": _frac(pairs * SLOTS_FORCE, kus["kforce"])}
            log(f"sweep n={n} p={p}: kspace {row['kspace_pairs_per_s']:.3e} pairs/s, "
                f"step {1e3 * st_ms:.1f} us, stage {row['stage']['frac']}, kforce {row['kforce']['frac']}")
            out.append(row)
            del ctx, P, Q, V, F
            torch.cuda.empty_cache()
    return out


def suite_batched(torch, R, W, log, steps=100):
    """64 replicas, N ~ U[500, 20000], 10% divalent: one batched context
    against a loop of 64 single-system contexts, same steps."""
    systems = W.replica_systems()
    params = [R.params_from_system(x, R.RBE_FP32) for x in systems]
    ntot = sum(x.n for x in systems)
    pairs = sum(x.n * x.p for x in systems)
    bctx = R.rbe_batch_create(params)
    cat = lambda a: np.concatenate(a, axis=-1)
    P = R.to_device(cat([x.pos for x in systems]), bctx)
    Q = R.to_device(cat([x.q for x in systems]), bctx)
    V = R.to_device(cat([x.vel for x in systems]), bctx)
    F = torch.zeros_like(P)
    R.rbe_step(bctx, P, V, Q, F, 0, 10)
    b_ms = _timed(torch, bctx.stream, lambda k: R.rbe_step(bctx, P, V, Q, F, 10, steps), 1) / steps
    ctxs, st = [], []
    for x, pr in zip(systems, params):
        c = R.rbe_create(pr)
        t = [R.to_device(x.pos, c), None, R.to_device(x.vel, c), None]
        t[1] = R.to_device(x.q, c)
        t[3] = torch.zeros_like(t[0])
        R.rbe_step(c, t[0], t[2], t[1], t[3], 0, 10)
        ctxs.append(c)
        st.append(t)

    def loop(k):
        for c, t in zip(ctxs, st):
            R.rbe_step(c, t[0], t[2], t[1], t[3], 10, steps)

    l_ms = _timed(torch, ctxs[0].stream, loop, 1) / steps
    row = {"replicas": len(systems), "particles": ntot, "pairs_per_step": pairs,
           "batched": {"ms_per_step": b_ms, "steps_per_s": 1e3 / b_ms, "pairs_per_s": pairs * 1e3 / b_ms},
           "loop": {"ms_per_step": l_ms, "steps_per_s": 1e3 / l_ms, "pairs_per_s": pairs * 1e3 / l_ms},
           "speedup": l_ms / b_ms}
    log(f"batched {b_ms * 1e3:.1f} us/step vs loop {l_ms * 1e3:.1f} us/step")
    return row


def suite_gradient(torch, R, W, log, reps=50):
    """N = 30000 Gaussian charges, P = 200: forces forward only against
    forward + backward of the force-matching loss (autograd over the adjoint)."""
    from paper_2010_01559_amd.autograd import force_matching_loss, rbe_forces
    s = W.gaussian_charge_system()
    ctx = R.rbe_create(R.params_from_system(s, R.RBE_FP32))
    P = R.to_device(s.pos, ctx).requires_grad_()
    Q = R.to_device(s.q, ctx).requires_grad_()
    R.rbe_sample_k(ctx, 5)
    Fref = torch.zeros((3, s.n), dtype=P.dtype, device=P.device)

    def fwd(k):
        with torch.no_grad():
            rbe_forces(ctx, P, Q)

    def fwd_bwd(k):
        P.grad = None
        Q.grad = None
        force_matching_loss(ctx, P, Q, Fref).backward()

    fwd(0)
    fwd_bwd(0)
    f_ms = _timed(torch, ctx.stream, fwd, reps)
    fb_ms = _timed(torch, ctx.stream, fwd_bwd, reps)
    row = {"n": s.n, "p": s.p, "forward_ms": f_ms, "forward_backward_ms": fb_ms, "ratio": fb_ms / f_ms}
    log(f"gradient: forward {f_ms * 1e3:.1f} us, forward+backward {fb_ms * 1e3:.1f} us")
    return row


def suite_ewald(torch, R, W, log, tol=1e-4):
    """Classical Ewald (every mode with exp(-k^2/4 alpha) >= tol, same alpha
    and r_c as the random batch) on the same kernels, against one random
    batch evaluation (P = 100), at growing N and density 0.1."""
    from paper_2010_01559_amd.ewald import ewald_modes, mode_radius2
    out = []
    for n in (1000, 3000, 10000, 30000, 100000):
        s = W.metric_system() if n == 100000 else W.scaling_system(n, 100)
        ctx = R.rbe_create(R.params_from_system(s, R.RBE_FP32))
        P = R.to_device(s.pos, ctx)
        Q = R.to_device(s.q, ctx)
        F = torch.zeros_like(P)
        R.rbe_sample_k(ctx, 0)
        rbe_ms = _timed(torch, ctx.stream, lambda k: (R.rbe_sample_k(ctx, k), R.rbe_kspace_forces(ctx, P, Q, F)),
                        50)
        real_ms = _timed(torch, ctx.stream, lambda k: R.rbe_real_forces(ctx, P, Q, F), 50)
        m, w = ewald_modes(s.alpha, s.L, mode_radius2(s.alpha, s.L, tol))
        R.rbe_reserve_modes(ctx, m.shape[1])
        R.rbe_set_k(ctx, m, w)
        R.rbe_kspace_forces(ctx, P, Q, F)
        ew_ms = _timed(torch, ctx.stream, lambda k: R.rbe_kspace_forces(ctx, P, Q, F), 5)
        row = {"n": n, "box": s.L, "ewald_modes": int(m.shape[1]), "ewald_kspace_ms": ew_ms,
               "ewald_pairs_per_s": n * m.shape[1] * 1e3 / ew_ms, "rbe_kspace_ms": rbe_ms,
               "real_space_ms": real_ms, "ewald_over_rbe": ew_ms / rbe_ms}
        log(f"ewald n={n}: {m.shape[1]} modes {ew_ms:.3f} ms vs rbe {rbe_ms:.4f} ms")
        out.append(row)
        del ctx, P, Q, F
        torch.cuda.empty_cache()
    return out


def run_suite(path):
    import torch

    import paper_2010_01559_amd.rbe as R
    from paper_2010_01559_amd import workloads as W

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    torch.cuda.set_device(0)
    res = {"sweep": suite_np_sweep(torch, R, W, log)}
    res["batched"] = suite_batched(torch, R, W, log)
    res["gradient"] = suite_gradient(torch, R, W, log)
    res["ewald"] = suite_ewald(torch, R, W, log)
    with open(path, "w") as f:
        json.dump(res, f, indent=1)
    log(f"suite written to {path}")


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported: the library runs on a "
              f"single MI355X and has no multi-GPU sharding", file=sys.stderr)
        sys.exit(2)
    if args.suite:
        run_suite(args.suite)
        return
    import torch

    import paper_2010_01559_amd.rbe as R
    from paper_2010_01559_amd import workloads as W

    torch.cuda.set_device(0)
    if args.calibrate_copy:
        a = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    s = W.metric_system()
    params = R.params_from_system(s, R.RBE_FP32)
    ctx = R.rbe_create(params)
    dt = torch.float32
    P = torch.as_tensor(s.pos, dtype=dt, device="cuda").contiguous()
    Q = torch.as_tensor(s.q, dtype=dt, device="cuda").contiguous()
    V = torch.as_tensor(s.vel, dtype=dt, device="cuda").contiguous()
    F = torch.zeros_like(P)
    stream = ctx.stream

    R.rbe_use_graphs(ctx, args.graphs)
    R.rbe_sample_k(ctx, 0)
    tiles = R.rbe_autotune(ctx, P, Q, reps=20) if args.autotune else R.rbe_get_tiles(ctx)
    R.rbe_kspace_forces(ctx, P, Q, F)
    R.rbe_real_forces(ctx, P, Q, F, accumulate=True)

    # ---- full MD steps (one rbe_step call advances all K steps) ----
    R.rbe_step(ctx, P, V, Q, F, 1, args.warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    base = 1 + args.warmup
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    R.rbe_step(ctx, P, V, Q, F, base, args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = e0.elapsed_time(e1) / args.steps
    ms_per_step = max(step_ms, 1e3 * wall / args.steps)

    # ---- Fourier-only evaluations: sample + structure factor + force ----
    nk = max(args.steps, 100)
    for k in range(10):
        R.rbe_sample_k(ctx, 10 ** 6 + k)
        R.rbe_kspace_forces(ctx, P, Q, F)
    torch.cuda.synchronize()
    e0.record(stream)
    for k in range(nk):
        R.rbe_sample_k(ctx, 2 * 10 ** 6 + k)
        R.rbe_kspace_forces(ctx, P, Q, F)
    e1.record(stream)
    torch.cuda.synchronize()
    k_ms = e0.elapsed_time(e1) / nk

    # ---- per-kernel durations with HIP events on the library stream ----
    R.rbe_profile_enable(ctx, True)
    R.rbe_step(ctx, P, V, Q, F, base + args.steps, args.steps)
    prof = R.rbe_profile_read(ctx)
    R.rbe_profile_enable(ctx, False)
    kern = {name: {"avg_us": 1e3 * ms / n, "launches": n} for name, (ms, n) in prof.items() if n}
    step_kernel_us = sum(v["avg_us"] * v["launches"] for v in kern.values()) / args.steps
    # the Fourier kernels alone (structure factor without the fused
    # integrator/binning, and the force pass without the scatter)
    R.rbe_profile_enable(ctx, True)
    for k in range(nk):
        R.rbe_sample_k(ctx, 3 * 10 ** 6 + k)
        R.rbe_kspace_forces(ctx, P, Q, F)
    kprof = R.rbe_profile_read(ctx)
    R.rbe_profile_enable(ctx, False)
    kkern = {name: {"avg_us": 1e3 * ms / n, "launches": n} for name, (ms, n) in kprof.items() if n}

    n, p = s.n, s.p
    pairs = n * p
    cand, nb = real_space_counts(s, params.skin)
    # the force launch of a step also evaluates the Fourier force
    work = {"stage": pairs * SLOTS_RHO, "kforce": pairs * SLOTS_FORCE,
            "real": cand * SLOTS_CHECK + nb * SLOTS_PAIR + pairs * SLOTS_FORCE}
    rooflines = {}
    for name, slots in work.items():
        if name not in kern:
            continue
        us = kern[name]["avg_us"]
        ach = slots * 2 / (us * 1e-6) / 1e12
        rooflines[name] = {"bound": "alu", "achieved": round(ach, 3), "peak": PEAK_FP32_TFLOPS,
                           "unit": "TFLOP/s", "frac": round(ach / PEAK_FP32_TFLOPS, 4),
                           "traffic": traffic_for(name), "avg_launch_us": round(us, 2),
                           "slots_per_launch": int(slots)}
    dom = max(rooflines, key=lambda k: kern[k]["avg_us"])
    roofline = dict(rooflines[dom], kernel=dom)
    fourier = {}
    for name, slots in (("kforce", pairs * SLOTS_FORCE), ("stage", pairs * SLOTS_RHO)):
        us = kkern[name]["avg_us"]
        ach = slots * 2 / (us * 1e-6) / 1e12
        fourier[name] = {"achieved": round(ach, 3), "frac": round(ach / PEAK_FP32_TFLOPS, 4),
                         "avg_launch_us": round(us, 2),
                         "traffic": traffic_for("stage_fourier" if name == "stage" else name)}

    cpu = None
    if not args.no_cpu:
        m = torch.zeros((3, p), dtype=torch.int32, device="cuda")
        R.rbe_sample_k(ctx, 0, m)
        cpu = cpu_baseline(s, m.cpu().numpy(), args.cpu_seconds)

    out = {
        "metric": METRIC,
        "value": pairs * 1e3 / ms_per_step,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": s.name, "n": n, "p": p, "box": s.L, "alpha": round(s.alpha, 6),
                   "r_cut": s.r_cut, "lj": list(s.lj), "dt": s.dt, "precision": "fp32 (fp64 phases)",
                   "tiles": tiles},
        "md_steps_per_s": 1e3 / ms_per_step,
        "kspace_pairs_per_s": pairs * 1e3 / k_ms,
        "kspace_ms": k_ms,
        "step_kernel_us": step_kernel_us,
        "kernels": {k: {"avg_us": round(v["avg_us"], 2), "launches": v["launches"]} for k, v in kern.items()},
        "kspace_kernels": {k: {"avg_us": round(v["avg_us"], 2), "launches": v["launches"]}
                           for k, v in kkern.items()},
        "real_space": {"list_entries": cand, "pairs_in_cutoff": nb},
        "roofline": roofline,
        "rooflines": rooflines,
        "fourier_only_rooflines": fourier,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
