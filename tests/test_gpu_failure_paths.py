"""Failure handling of the device-side list rebuild, forced from the host.

The rebuild inside a time step (Algorithm 1 of Sec. 3.1 on the neighbour
list) orders its binning, scan and scatter blocks with bounded waits.  A wait
bound of zero, set from the host, makes every wait give up at once: every
kernel still runs to its end, no access leaves its system's slots, the error
surfaces as RBE_ERR_TIMEOUT at the next check, and once the bound is back
the context repairs itself and steps exactly as a fresh one.  No test here
makes a kernel fault, trap or hang."""
import numpy as np
import pytest

import paper_2010_01559_amd.rbe as R
from paper_2010_01559_amd import workloads as W
from gpu_util import device_state, host, make_ctx

pytestmark = pytest.mark.gpu


def _initial(ctx, s):
    P, Q, V, F = device_state(ctx, s)
    R.rbe_sample_k(ctx, 0)
    R.rbe_kspace_forces(ctx, P, Q, F)
    R.rbe_real_forces(ctx, P, Q, F, accumulate=True)
    return P, Q, V, F


@pytest.mark.parametrize("prec", [R.RBE_FP32, R.RBE_FP64])
def test_rebuild_timeout_is_reported_and_repaired(prec):
    s = W.langevin_electrolyte()
    ctx = make_ctx(s, prec)
    P, Q, V, F = _initial(ctx, s)
    P0, V0, F0 = P.clone(), V.clone(), F.clone()
    R.rbe_set_wait_limit(ctx, 0)
    R.rbe_step(ctx, P, V, Q, F, 1, 3)   # the first step rebuilds; its waits give up
    st, builds = R.rbe_list_builds(ctx, allow_status=(R.RBE_OK, R.RBE_ERR_TIMEOUT))
    assert st == R.RBE_ERR_TIMEOUT and builds == 0
    assert R.rbe_check_status(ctx) == R.RBE_OK          # reported once, then cleared
    R.rbe_step(ctx, P, V, Q, F, 4, 1)
    st, e = R.rbe_energy(ctx, P, Q, V, allow_status=(R.RBE_ERR_TIMEOUT,))
    assert st == R.RBE_ERR_TIMEOUT and e[0]["timeout"] == 1
    # back to the default bound: the same start steps as in a fresh context
    R.rbe_set_wait_limit(ctx, 1 << 24)
    P.copy_(P0)
    V.copy_(V0)
    F.copy_(F0)
    R.rbe_step(ctx, P, V, Q, F, 1, 6)
    R.rbe_check(ctx)
    assert R.rbe_list_builds(ctx) >= 1
    ref = make_ctx(s, prec)
    P2, V2, F2 = P0.clone(), V0.clone(), F0.clone()
    R.rbe_step(ref, P2, V2, Q, F2, 1, 6)
    R.rbe_check(ref)
    for a, b in ((P, P2), (V, V2), (F, F2)):
        if prec == R.RBE_FP32:
            # single-precision pair sums are exact, so the order of partners
            # inside a cell (atomic counters) does not show
            assert np.array_equal(host(a), host(b))
        else:
            # double-precision pair sums follow that order: rounding only
            assert np.abs(host(a) - host(b)).max() <= 1e-12 * np.abs(host(b)).max()


def test_wait_limit_rejects_negative_values():
    s = W.small_fp64()
    ctx = make_ctx(s, R.RBE_FP64)
    with pytest.raises(R.RBEError) as e:
        R.rbe_set_wait_limit(ctx, -1)
    assert e.value.status == R.RBE_ERR_INVALID


def test_non_finite_position_is_reported_by_check():
    s = W.langevin_electrolyte()
    ctx = make_ctx(s, R.RBE_FP32)
    P, Q, V, F = _initial(ctx, s)
    R.rbe_check(ctx)
    P[0, 7] = float("nan")
    R.rbe_sample_k(ctx, 1)
    R.rbe_kspace_forces(ctx, P, Q, F)
    assert R.rbe_check_status(ctx) == R.RBE_ERR_NONFINITE
    assert R.rbe_check_status(ctx) == R.RBE_OK


def test_overlap_beyond_the_exact_range_is_reported():
    """Two ions pressed into each other's LJ wall (r = 0.3 sigma, a pair force
    near 3e8): the single-precision pair sums would leave the range in which
    they are exact, and rbe_check reports RBE_ERR_NONFINITE instead of
    returning silently rounded forces; the same system at its drawn positions
    reports nothing."""
    s = W.langevin_electrolyte()
    ctx = make_ctx(s, R.RBE_FP32)
    P, Q, V, F = device_state(ctx, s)
    R.rbe_real_forces(ctx, P, Q, F)
    assert R.rbe_check_status(ctx) == R.RBE_OK
    P[:, 1] = P[:, 0]
    P[0, 1] = (P[0, 0] + 0.3) % s.L
    R.rbe_real_forces(ctx, P, Q, F)
    assert R.rbe_check_status(ctx) == R.RBE_ERR_NONFINITE
    assert "2^20" in R.lib().rbe_last_error(ctx.handle).decode()
    assert R.rbe_check_status(ctx) == R.RBE_OK
