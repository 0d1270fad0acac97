"""Helpers for the GPU tests: build a context and device tensors from a
synthetic system, and compare with the oracle."""
import numpy as np

import paper_2010_01559_amd.rbe as R


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def make_ctx(sys, precision=R.RBE_FP64, **over):
    p = R.params_from_system(sys, precision, **over)
    return R.rbe_create(p)


def device_state(ctx, sys, pos=None):
    import torch
    dt = torch.float64 if ctx.precision == R.RBE_FP64 else torch.float32
    pos = sys.pos if pos is None else pos
    P = torch.as_tensor(np.ascontiguousarray(pos), dtype=dt, device="cuda").contiguous()
    Q = torch.as_tensor(sys.q, dtype=dt, device="cuda").contiguous()
    V = torch.as_tensor(np.ascontiguousarray(sys.vel), dtype=dt, device="cuda").contiguous()
    F = torch.zeros((3, sys.n), dtype=dt, device="cuda")
    return P, Q, V, F


def host(t):
    return t.detach().double().cpu().numpy()


def rounded(sys, precision):
    """Positions/charges as the GPU sees them (float32 rounding for FP32)."""
    if precision == R.RBE_FP32:
        return sys.pos.astype(np.float32).astype(np.float64), sys.q.astype(np.float32).astype(np.float64)
    return sys.pos, sys.q


# Trajectory checks.  FP32 positions are stored in single precision after
# every step, which alone moves a coordinate by up to half an ulp of the box
# side per step; over the short horizons of the tests that is well below
# 2e-3 of the distance the particles travel, the bound used for the
# position error over the displacement from the start.  Velocities carry the
# same relative rounding (~6e-8 per step).  (The position bound, 2e-3, is
# about three times the storage rounding of a box of side 226 over 20 steps
# of 0.002.)  The force the step leaves is
# checked against the oracle evaluated at the GPU's own final positions, so
# its tolerance is the force tolerance itself.
TRAJ_TOL = {R.RBE_FP64: dict(pos=1e-9, vel=1e-10, force=1e-11),
            R.RBE_FP32: dict(pos=2e-3, vel=2e-5, force=1e-5)}


def min_image(d, L):
    return d - L * np.round(d / L)


def displacement_error(P, po, p_start, L):
    """|| GPU - oracle || over || oracle - start || (minimum image)."""
    dp = min_image(host(P) - po, L)
    moved = min_image(po - p_start, L)
    return float(np.linalg.norm(dp) / np.linalg.norm(moved))


def check_trajectory(prec, P, V, F, po, vo, p_start, L, force_at_gpu_positions, scale=1.0):
    """Asserts the three trajectory bounds; force_at_gpu_positions(pos) is the
    oracle's force at the given positions with the last step's modes."""
    tol = TRAJ_TOL[prec]
    e_pos = displacement_error(P, po, p_start, L)
    e_vel = rel_l2(host(V), vo)
    e_f = rel_l2(host(F), force_at_gpu_positions(host(P)))
    assert e_pos <= scale * tol["pos"], ("position", e_pos)
    assert e_vel <= scale * tol["vel"], ("velocity", e_vel)
    assert e_f <= tol["force"], ("force", e_f)
    return e_pos, e_vel, e_f
