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
