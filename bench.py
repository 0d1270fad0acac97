"""Benchmark of the random batch Ewald hot path on one MI355X.

Workload: N = 1e5 ions (+-1) at density 0.1 (L = 100), r_c = 3.5, P = 100
modes per step, alpha from the 1e-4 real-space error estimate, shifted LJ
(eps = 1, sigma = 1, cut 2.5), Langevin kT = 1, gamma = 1, dt = 1e-3, float32
arithmetic with phases split exactly and double-precision reductions.
Inputs are synthetic and resident on the GPU before timing starts.

A timed "step" is one pass of the whole hot path: a fresh batch of P modes,
structure factors, the Fourier force, the neighbour list (rebuilt on the
device when particles have moved far enough), the real-space + LJ force and
the Langevin update; the K timed steps are one rbe_step call.  The headline
value is N*P*steps / elapsed seconds over those full steps.  The JSON line
also reports MD steps/s, the list builds inside the timed window, the
Fourier-only pair rate (sample + structure factor + force), per-kernel
durations (events carried by the kernels' own dispatches, the same steps
again), the ALU roofline of each kernel from algorithmic operation counts
(the longest one per step as "roofline"), the same work against bounds
calibrated on this device, and the FP64 CPU oracle timed on the host.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
                       [--autotune] [--calibrate-copy] [--graphs]
       python bench.py --calibrate      (device micro-benchmarks only)
       python bench.py --suite PATH     (N x P sweep, batched vs loop,
                                         forward vs backward, classical Ewald)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "k-space particle–mode pairs/s (N·P) + MD steps/s at N=1e5, P=100, 1 GPU"

# Algorithmic work, in FP32 lane operations (an add, multiply, fused
# multiply-add or hardware transcendental each counts one), split into
# (VALU, transcendental).  Per particle-mode pair and pass the phase m.s is
# three multiply-adds and a wrap; the structure factor adds two multiply-adds
# into (C, S), the force cos(th) S - sin(th) C and three multiply-adds into F
# (paper Sec. 3.1, eq. 3.6, with rho of eq. 2.7).  Real space: every list
# entry is a distance test (3 differences, |d|^2, compare, select); a pair
# inside the cutoff adds rsqrt, exp and a reciprocal, r and beta r, the
# erfc polynomial, G(r), the charge product, the LJ term and three force
# components (eq. 2.11, eq. 4.1).  Implementation extras (the exact phase
# split, fixed-point sums) are not counted.
OPS = {
    "rho_pair": (6, 2),
    "force_pair": (9, 2),
    "list_entry": (8, 0),
    "cutoff_pair": (22, 3),
}
PEAK_FP32_TFLOPS = 157.3   # MI355X FP32 vector peak (published)
WARMUP_EVALS = 5000        # device warm-up before the warmup steps (GPU clocks): ~0.1 s
PEAK_HBM_GBS = 8000.0

# HBM traffic per launch from two rocprofv3 --pmc passes (FETCH_SIZE, then
# WRITE_SIZE, KiB per dispatch, averaged over the launches of the profiled
# run), each multiplied by the ratio of the true size of a 256 MiB device
# copy to what the same counter reads for it.  Valid only for the kernel
# source it was taken on (sha256 prefix); otherwise reported as null.
# k_real_step: the list-pass launches of the profiled run (the rebuild step's
# cell pass, which reads several times more, is left out, as the timed window
# of the N = 1e5 run holds no rebuild); the staging launches of steps after
# the first of a call; the Fourier-only launches at N = 1e5.
TRAFFIC = {
    "real": {"src": "eec603a65a2ee666", "fetch_kib": 8589.8, "write_kib": 6187.7, "fetch_scale": 2.000,
             "write_scale": 1.000},
    "stage": {"src": "adaeb3e7b6491e46", "fetch_kib": 3012.7, "write_kib": 6995.3, "fetch_scale": 2.000,
              "write_scale": 1.000},
    "stage_fourier": {"src": "adaeb3e7b6491e46", "fetch_kib": 875.8, "write_kib": 400.0, "fetch_scale": 2.000,
                      "write_scale": 1.000},
    "kforce": {"src": "adaeb3e7b6491e46", "fetch_kib": 840.8, "write_kib": 1171.9, "fetch_scale": 2.000,
               "write_scale": 1.000},
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
    ap.add_argument("--suite-parts", default="sweep,batched,gradient,ewald,n_t",
                    help="comma-separated parts of the suite to run")
    ap.add_argument("--calibrate", action="store_true", help="print the device micro-benchmarks and exit")
    ap.add_argument("--tune", metavar="PATH",
                    help="autotune the benchmark configurations and append the tile cache entries to PATH")
    ap.add_argument("--graphs", action="store_true", help="replay the steady-state steps from hipGraphs")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one 256 MiB device copy first (reference for HBM byte counters)")
    return ap.parse_args()


def calibration(R, reps=5):
    """Device micro-benchmarks of the library (rbe_calibrate): rates of the
    hardware sine/cosine, non-packed FP32 and FP64 FMA, and a device copy."""
    return {name: R.rbe_calibrate(k, reps) for k, name in R.CALIBRATION_KINDS.items()}


def kspace_bound_pairs_per_s(cal):
    """Pairs/s of one Fourier evaluation (structure factor + force) if its
    algorithmic work ran at the calibrated rates, transcendental and VALU
    issue not overlapping."""
    valu = OPS["rho_pair"][0] + OPS["force_pair"][0]
    trans = OPS["rho_pair"][1] + OPS["force_pair"][1]
    return 1.0 / (trans / cal["sin_cos_lane_ops_per_s"] + valu / cal["fp32_fma_lane_ops_per_s"])


def alu_roofline(units, us, cal=None, traffic=None):
    """units: {OPS key: count per launch}; us: average launch duration."""
    valu = sum(OPS[k][0] * n for k, n in units.items())
    trans = sum(OPS[k][1] * n for k, n in units.items())
    ops = valu + trans
    ach = ops / (us * 1e-6) / 1e12
    out = {"bound": "alu", "achieved": round(ach, 3), "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
           "frac": round(ach / PEAK_FP32_TFLOPS, 4), "traffic": traffic, "avg_launch_us": round(us, 2),
           "ops_per_launch": int(ops), "units": {k: int(n) for k, n in units.items()}}
    if cal:
        bound_us = 1e6 * (trans / cal["sin_cos_lane_ops_per_s"] + valu / cal["fp32_fma_lane_ops_per_s"])
        out["calibrated"] = {"bound_us": round(bound_us, 2), "frac": round(bound_us / us, 4)}
    return out


def cpu_baseline(s, budget_s):
    """Time the FP64 oracle on the metric workload: whole MD steps (a fresh
    mode sample, structure factor and Fourier force, real space on the
    oracle's linked cells, BAOAB) repeated until the budget is spent, with
    every host thread, then single-threaded; and the Fourier evaluation
    alone."""
    import oracle as O
    O.build()
    pos = s.pos.astype(np.float32).astype(np.float64)
    vel = s.vel.astype(np.float32).astype(np.float64)
    q = s.q.astype(np.float64)
    sysd = O.make_sys(s.n, s.p, s.L, s.alpha, s.r_cut, s.coulomb, s.lj, s.kT, s.gamma, s.dt, s.mass, s.seed)
    F = O.total_force(sysd, pos, q, 0)

    def md_rate(budget, first):
        steps, t0 = 0, time.perf_counter()
        while True:
            O.baoab_step(sysd, pos, vel, q, F, first + steps)
            steps += 1
            el = time.perf_counter() - t0
            if el > budget or steps >= 500:
                return s.n * s.p * steps / el, steps, el

    modes, _ = O.sample_modes(s.alpha, s.L, s.p, s.seed, 0)
    w = O.rbe_weights(s.alpha, s.L, s.p)

    def fourier_rate(budget):
        reps, t0 = 0, time.perf_counter()
        while True:
            O.kspace_force(pos, q, s.L, modes, w)
            reps += 1
            el = time.perf_counter() - t0
            if el > budget or reps >= 1000:
                return s.n * s.p * reps / el, reps, el

    threads = O.set_threads(0)
    v, steps, el = md_rate(budget_s, 1)
    vf, reps, elf = fourier_rate(budget_s / 3)
    O.set_threads(1)
    v1, steps1, el1 = md_rate(budget_s / 3, 1 + steps)
    O.set_threads(threads)
    return {"value": v, "unit": "pairs/s", "cores": threads, "kind": "oracle",
            "sample": f"{steps} full MD steps (mode sample, structure factor and Fourier force, linked-cell "
                      f"real space + LJ, BAOAB; FP64) of the N={s.n}, P={s.p} workload in {el:.1f} s on "
                      f"{threads} threads; single-threaded {steps1} steps in {el1:.1f} s; Fourier evaluation "
                      f"alone {reps} times in {elf:.1f} s on {threads} threads",
            "single_thread_value": v1, "fourier_only_value": vf, "md_steps_per_s": steps / el,
            "host_cpu": _cpu_model()}


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

def suite_np_sweep(torch, R, W, log, cal):
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
                   "kspace_frac_of_calibrated_bound": pairs * 1e3 / k_ms / kspace_bound_pairs_per_s(cal),
                   "md_steps_per_s": 1e3 / st_ms, "md_pairs_per_s": pairs * 1e3 / st_ms, "md_ms": st_ms,
                   "stage": alu_roofline({"rho_pair": pairs}, kus["stage"], cal),
                   "kforce": alu_roofline({"force_pair": pairs}, kus["kforce"], cal)}
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
    row = {"replicas": len(systems), "particles": ntot, "pairs_per_step": pairs, "tiles": R.rbe_get_tiles(bctx),
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
    from paper_2010_01559_amd.ewald import mode_radius2, set_ewald
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
        m2 = mode_radius2(s.alpha, s.L, tol)
        nm = set_ewald(ctx, m2)
        R.rbe_kspace_forces(ctx, P, Q, F)
        ew_ms = _timed(torch, ctx.stream, lambda k: R.rbe_kspace_forces(ctx, P, Q, F), 5)
        row = {"n": n, "box": s.L, "ewald_modes": nm, "ewald_kspace_ms": ew_ms,
               "ewald_pairs_per_s": n * nm * 1e3 / ew_ms, "rbe_kspace_ms": rbe_ms,
               "real_space_ms": real_ms, "ewald_over_rbe": ew_ms / rbe_ms}
        if n in (1000, 10000):
            # the FP64 oracle's classical Ewald Fourier force on the host, on
            # the oracle's own enumeration of the same mode ball
            import oracle as O
            pos, q = s.pos.astype(np.float32).astype(np.float64), s.q
            m, w = O.ewald_modes(s.alpha, s.L, m2)
            t0 = time.perf_counter()
            O.kspace_force(pos, q, s.L, m, w)
            row["oracle_ewald_kspace_ms"] = 1e3 * (time.perf_counter() - t0)
            row["oracle_threads"] = O.set_threads(0)
        log(f"ewald n={n}: {nm} modes {ew_ms:.3f} ms vs rbe {rbe_ms:.4f} ms")
        out.append(row)
        del ctx, P, Q, F
        torch.cuda.empty_cache()
    return out


def suite_nt(torch, R, W, log, s_acc=3.0, reps=3):
    """Per-evaluation force time against N (the paper's per-step timing
    figure, Sec. 4.1), on the GPU.  Classical Ewald runs on the same kernels
    with alpha re-balanced as the box grows (Sec. 2: r_c = s/sqrt(alpha),
    k_c = 2 s sqrt(alpha), and sqrt(alpha) ~ N^(1/6)/L balances the real and
    Fourier costs for O(N^(3/2)) in all): s = 3 (exp(-s^2) ~ 1e-4), the
    constant of alpha ~ N^(-1/3) at density 0.1 fixed by the fastest total
    over a scan at N = 1e4.  The random batch evaluation keeps alpha = 0.6633,
    r_c = 3.5 and P = 100 (a fresh sample each time).  Coulomb only, cell
    list rebuilt per call (no skin), FP32."""
    from paper_2010_01559_amd.ewald import set_ewald

    def ewald_parts(sy, alpha):
        rc = s_acc / math.sqrt(alpha)
        mc = s_acc * math.sqrt(alpha) * sy.L / math.pi   # k_c L / (2 pi)
        ctx = R.rbe_create(R.params_from_system(sy, R.RBE_FP32, alpha=alpha, r_cut=rc, lj_eps=0.0, skin=0.0))
        P = R.to_device(sy.pos, ctx)
        Q = R.to_device(sy.q, ctx)
        F = torch.zeros_like(P)
        R.rbe_real_forces(ctx, P, Q, F)
        real_ms = _timed(torch, ctx.stream, lambda k: R.rbe_real_forces(ctx, P, Q, F), reps)
        nm = set_ewald(ctx, int(math.floor(mc * mc)))
        R.rbe_kspace_forces(ctx, P, Q, F)
        four_ms = _timed(torch, ctx.stream, lambda k: R.rbe_kspace_forces(ctx, P, Q, F), reps)
        ctx.close()
        del P, Q, F
        torch.cuda.empty_cache()
        return {"alpha": alpha, "r_cut": rc, "modes": nm, "real_ms": real_ms, "kspace_ms": four_ms,
                "total_ms": real_ms + four_ms}

    n0 = 10000
    s0 = W.scaling_system(n0, 100)
    scan = [ewald_parts(s0, a) for a in (0.05, 0.07, 0.1, 0.14, 0.2)]
    a0 = min(scan, key=lambda r: r["total_ms"])["alpha"]
    log(f"n-t: alpha scan at N = {n0}: " + ", ".join(f"{r['alpha']}: {r['total_ms']:.3f} ms" for r in scan))
    rows = []
    for n in (1000, 3000, 10000, 30000, 100000, 300000, 1000000):
        sy = W.metric_system() if n == 100000 else W.scaling_system(n, 100)
        alpha = max(a0 * (n / n0) ** (-1.0 / 3.0), 4.0 * s_acc * s_acc / (sy.L * sy.L))   # r_c <= L/2
        ew = ewald_parts(sy, alpha)
        ctx = R.rbe_create(R.params_from_system(sy, R.RBE_FP32, lj_eps=0.0, skin=0.0))
        P = R.to_device(sy.pos, ctx)
        Q = R.to_device(sy.q, ctx)
        F = torch.zeros_like(P)

        def rbe(k):
            R.rbe_sample_k(ctx, 100 + k)
            R.rbe_kspace_forces(ctx, P, Q, F)
            R.rbe_real_forces(ctx, P, Q, F, accumulate=True)

        rbe(0)
        rbe_ms = _timed(torch, ctx.stream, rbe, max(reps, 10))
        ctx.close()
        del P, Q, F
        torch.cuda.empty_cache()
        row = {"n": n, "box": sy.L, "ewald": ew, "rbe_ms": rbe_ms, "ewald_over_rbe": ew["total_ms"] / rbe_ms}
        log(f"n-t n={n}: ewald {ew['total_ms']:.3f} ms (alpha {alpha:.4f}, {ew['modes']} modes, r_c "
            f"{ew['r_cut']:.2f}) vs rbe {rbe_ms:.4f} ms")
        rows.append(row)
    big = [r for r in rows if r["n"] >= 10000]
    ln = np.log([r["n"] for r in big])
    slope_e = float(np.polyfit(ln, np.log([r["ewald"]["total_ms"] for r in big]), 1)[0])
    slope_r = float(np.polyfit(ln, np.log([r["rbe_ms"] for r in big]), 1)[0])
    log(f"n-t slopes over N >= 1e4: ewald {slope_e:.3f}, rbe {slope_r:.3f}")
    return {"alpha_scan": scan, "alpha_at_1e4": a0, "rows": rows,
            "slope_ewald": slope_e, "slope_rbe": slope_r, "fit_range": "N >= 1e4"}


def run_suite(path, parts):
    import torch

    import paper_2010_01559_amd.rbe as R
    from paper_2010_01559_amd import workloads as W

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    torch.cuda.set_device(0)
    cal = calibration(R)
    log(f"calibration: {cal}")
    res = {"calibration": cal}
    if "sweep" in parts:
        res["sweep"] = suite_np_sweep(torch, R, W, log, cal)
    if "batched" in parts:
        res["batched"] = suite_batched(torch, R, W, log)
    if "gradient" in parts:
        res["gradient"] = suite_gradient(torch, R, W, log)
    if "ewald" in parts:
        res["ewald"] = suite_ewald(torch, R, W, log)
    if "n_t" in parts:
        res["n_t"] = suite_nt(torch, R, W, log)
    with open(path, "w") as f:
        json.dump(res, f, indent=1)
    log(f"suite written to {path}")


def run_tune(path):
    """rbe_autotune on the configurations the benchmark and its suite time:
    the N x P sweep, the 64 batched replicas, the differentiable form and the
    3000-ion electrolyte.  Each result is appended to the tile cache at
    PATH (the library writes it); the Fourier evaluation time with the
    default and the tuned shapes is printed."""
    os.environ["RBE_TUNE_CACHE"] = path
    import torch

    import paper_2010_01559_amd.rbe as R
    from paper_2010_01559_amd import workloads as W

    torch.cuda.set_device(0)
    cases = [("electrolyte", [W.langevin_electrolyte()]), ("gradient", [W.gaussian_charge_system()]),
             ("replicas", W.replica_systems())]
    for n in (10000, 100000, 1000000):
        for p in (50, 100, 200, 500):
            cases.append((f"sweep n={n} p={p}", [W.metric_system() if n == 100000 else W.scaling_system(n, 100)]))
            cases[-1][1][0].p = p
    for name, systems in cases:
        ctx = R.rbe_batch_create([R.params_from_system(x, R.RBE_FP32) for x in systems])
        cat = lambda a: np.ascontiguousarray(np.concatenate(a, axis=-1))
        P = R.to_device(cat([x.pos for x in systems]), ctx)
        Q = R.to_device(cat([x.q for x in systems]), ctx)
        F = torch.zeros_like(P)
        R.rbe_sample_k(ctx, 0)

        def four(k):
            R.rbe_sample_k(ctx, 10 + k)
            R.rbe_kspace_forces(ctx, P, Q, F)

        four(0)
        before, t0 = _timed(torch, ctx.stream, four, 20), R.rbe_get_tiles(ctx)
        R.rbe_sample_k(ctx, 0)
        best = R.rbe_autotune(ctx, P, Q, reps=20)
        four(0)
        after = _timed(torch, ctx.stream, four, 20)
        print(json.dumps({"case": name, "default": t0, "default_ms": before, "tuned": best, "tuned_ms": after}),
              flush=True)
        ctx.close()
        del P, Q, F
        torch.cuda.empty_cache()


def kspace_at_scale(torch, R, W, cal, n=1000000, p=200, reps=30):
    """Fourier evaluations (sample + structure factor + force) at N = 1e6,
    P = 200, the largest sweep size, where the launch and tail latencies that
    dominate N = 1e5 are amortised: pairs/s against the calibrated bound and
    the ALU roofline of its two passes (durations from dispatch events)."""
    s = W.scaling_system(n, p)
    ctx = R.rbe_create(R.params_from_system(s, R.RBE_FP32))
    P = R.to_device(s.pos, ctx)
    Q = R.to_device(s.q, ctx)
    F = torch.zeros_like(P)

    def four(k):
        R.rbe_sample_k(ctx, 5000 + k)
        R.rbe_kspace_forces(ctx, P, Q, F)

    four(0)
    ms = _timed(torch, ctx.stream, four, reps)
    kus = _kernel_us(R, ctx, four, reps)
    pairs = n * p
    out = {"n": n, "p": p, "kspace_ms": ms, "kspace_pairs_per_s": pairs * 1e3 / ms,
           "kspace_frac_of_calibrated_bound": pairs * 1e3 / ms / kspace_bound_pairs_per_s(cal),
           "kernels_us": {k: round(v, 2) for k, v in kus.items()},
           "stage": alu_roofline({"rho_pair": pairs}, kus["stage"], cal),
           "kforce": alu_roofline({"force_pair": pairs}, kus["kforce"], cal)}
    ctx.close()
    del P, Q, F
    torch.cuda.empty_cache()
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported: the library runs on a "
              f"single MI355X and has no multi-GPU sharding", file=sys.stderr)
        sys.exit(2)
    if args.suite:
        run_suite(args.suite, set(args.suite_parts.split(",")))
        return
    if args.tune:
        run_tune(args.tune)
        return
    import torch

    import paper_2010_01559_amd.rbe as R
    from paper_2010_01559_amd import workloads as W

    torch.cuda.set_device(0)
    if args.calibrate:
        print(json.dumps({"device": torch.cuda.get_device_name(0), "calibration": calibration(R)}))
        return
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

    # ---- device warm-up: after the host-side set-up the GPU idles and its
    # clocks drop; a short window timed from there reads about 7% slow
    # (measured: 42.0 µs per step by events for 20 steps from idle, 39.3
    # after 100 ms of work).  A fixed number of Fourier-only evaluations on
    # the same context (about 0.1 s), into a scratch force buffer, runs before
    # the warmup steps; the MD state is not touched. ----
    F_scratch = torch.zeros_like(P)
    torch.cuda.synchronize()
    t_w = time.perf_counter()
    for k_w in range(WARMUP_EVALS):
        R.rbe_sample_k(ctx, 3 * 10 ** 6 + k_w)
        R.rbe_kspace_forces(ctx, P, Q, F_scratch)
    torch.cuda.synchronize()
    warm_ms = 1e3 * (time.perf_counter() - t_w)
    del F_scratch

    # ---- full MD steps (one rbe_step call advances all K steps) ----
    R.rbe_step(ctx, P, V, Q, F, 1, args.warmup)
    builds0 = R.rbe_list_builds(ctx)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    base = 1 + args.warmup
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    R.rbe_step(ctx, P, V, Q, F, base, args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    builds_window = R.rbe_list_builds(ctx) - builds0
    R.rbe_check(ctx)
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

    # ---- per-kernel durations: events on the kernels' own dispatches ----
    # (the same number of steps again, continuing the trajectory)
    R.rbe_profile_enable(ctx, True)
    b1 = R.rbe_list_builds(ctx)
    R.rbe_step(ctx, P, V, Q, F, base + args.steps, args.steps)
    prof = R.rbe_profile_read(ctx)
    builds_prof = R.rbe_list_builds(ctx) - b1
    R.rbe_profile_enable(ctx, False)
    kern = {name: {"avg_us": 1e3 * ms / n, "launches": n, "us_per_step": 1e3 * ms / args.steps}
            for name, (ms, n) in prof.items() if n}
    step_kernel_us = sum(v["us_per_step"] for v in kern.values())
    R.rbe_profile_enable(ctx, True)
    for k in range(nk):
        R.rbe_sample_k(ctx, 3 * 10 ** 6 + k)
        R.rbe_kspace_forces(ctx, P, Q, F)
    kprof = R.rbe_profile_read(ctx)
    R.rbe_profile_enable(ctx, False)
    kkern = {name: {"avg_us": 1e3 * ms / n, "launches": n} for name, (ms, n) in kprof.items() if n}

    cal = calibration(R)
    n, p = s.n, s.p
    pairs = n * p
    entries, nb = real_space_counts(s, params.skin)
    # work of one launch of each kernel of the step; the force launch of a
    # step also evaluates the Fourier force
    work = {"stage": {"rho_pair": pairs},
            "real": {"force_pair": pairs, "list_entry": entries, "cutoff_pair": nb}}
    rooflines = {name: alu_roofline(units, kern[name]["avg_us"], cal, traffic_for(name))
                 for name, units in work.items() if name in kern}
    dom = max(kern, key=lambda k: kern[k]["us_per_step"])
    roofline = dict(rooflines[dom], kernel=dom) if dom in rooflines else None
    fourier = {"stage": alu_roofline({"rho_pair": pairs}, kkern["stage"]["avg_us"], cal,
                                     traffic_for("stage_fourier")),
               "kforce": alu_roofline({"force_pair": pairs}, kkern["kforce"]["avg_us"], cal, traffic_for("kforce"))}
    kbound = kspace_bound_pairs_per_s(cal)

    at_scale = kspace_at_scale(torch, R, W, cal)
    cpu = None if args.no_cpu else cpu_baseline(s, args.cpu_seconds)

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
                   "r_cut": s.r_cut, "lj": list(s.lj), "dt": s.dt,
                   "precision": "fp32 (exact split phases, fp64 reductions)", "tiles": tiles},
        "md_steps_per_s": 1e3 / ms_per_step,
        "step_ms_events_wall": [round(step_ms, 6), round(1e3 * wall / args.steps, 6)],
        "device_warmup": {"ms": round(warm_ms, 1), "work": f"{WARMUP_EVALS} Fourier-only evaluations (sample + structure "
                                                            "factor + force) on the same context into a scratch buffer, "
                                                            "before the warmup steps"},
        "list_builds": {"timed_window": builds_window, "profiled_window": builds_prof, "steps": args.steps},
        "kspace_pairs_per_s": pairs * 1e3 / k_ms,
        "kspace_ms": k_ms,
        "kspace_bound_pairs_per_s": kbound,
        "kspace_frac_of_calibrated_bound": pairs * 1e3 / k_ms / kbound,
        "step_kernel_us": step_kernel_us,
        "kernels": {k: {"avg_us": round(v["avg_us"], 2), "launches": v["launches"],
                        "us_per_step": round(v["us_per_step"], 2)} for k, v in kern.items()},
        "kspace_kernels": {k: {"avg_us": round(v["avg_us"], 2), "launches": v["launches"]}
                           for k, v in kkern.items()},
        "real_space": {"list_entries": entries, "pairs_in_cutoff": nb},
        "calibration": cal,
        "roofline": roofline,
        "rooflines": rooflines,
        "fourier_only_rooflines": fourier,
        "kspace_at_scale": at_scale,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
