"""Classical Ewald on the random batch Ewald kernels (the comparator).

Classical Ewald keeps every mode 0 < |m|^2 <= mmax2 of the Fourier sum
(eq. 2.9, second term, truncated as in Sec. 2.2), each with the weight
exp(-k^2 / (4 alpha)), k = 2 pi |m| / L; the random batch weight S/p is the
sampled counterpart of the same sum (Sec. 3.1).  The library enumerates the
list and its weights (rbe_ewald_modes) and makes it active on a context
(rbe_set_k_ewald); the structure-factor and force kernels then evaluate that
deterministic sum.  This module only forwards to those entry points.
"""
from __future__ import annotations

from . import rbe as R


def mode_radius2(alpha: float, L: float, tol: float) -> int:
    """Largest |m|^2 whose Gaussian factor exp(-pi^2 |m|^2 / (alpha L^2)) is
    at least tol (rbe_ewald_radius2)."""
    return R.rbe_ewald_radius2(alpha, L, tol)


def ewald_modes(alpha: float, L: float, mmax2: int):
    """All integer modes with 0 < |m|^2 <= mmax2 and their weights
    (rbe_ewald_modes): (modes int32 [3, nm], weights float64 [nm])."""
    return R.rbe_ewald_modes(alpha, L, mmax2)


def set_ewald(ctx, mmax2: int) -> int:
    """Make the classical Ewald list active on a single-system context
    (rbe_set_k_ewald); returns the number of modes."""
    return R.rbe_set_k_ewald(ctx, mmax2)
