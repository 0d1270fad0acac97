"""Mode lists for classical Ewald on the random batch Ewald kernels.

Classical Ewald keeps every mode 0 < |k| <= k_c of the Fourier sum (paper
eq. 2.9, second term, truncated as in Sec. 2.2).  Passed to ``rbe_set_k``
with per-mode weights, the library's structure-factor and force kernels then
evaluate that deterministic sum instead of a random batch.  In the library's
convention the force of a mode list is

    F_i = -q_i * coulomb * sum_l w_l * 2 m_l / (L^2 |m_l|^2) * Im(e^{-i theta_il} rho_l),

so the Ewald weight of mode m is exp(-k^2 / (4 alpha)) with k = 2 pi |m| / L
(the RBE weight S/p is the sampled counterpart of the same sum, Sec. 3.1).
"""
from __future__ import annotations

import math

import numpy as np


def mode_radius2(alpha: float, L: float, tol: float) -> int:
    """Largest |m|^2 whose Gaussian factor exp(-pi^2 |m|^2 / (alpha L^2)) is
    at least tol."""
    return int(math.floor(math.log(1.0 / tol) * alpha * L * L / (math.pi * math.pi)))


def ewald_modes(alpha: float, L: float, mmax2: int):
    """All integer modes with 0 < |m|^2 <= mmax2 (a ball, every sign) and their
    weights; returns (modes int32 [3, nm], weights float64 [nm])."""
    R = int(math.isqrt(mmax2))
    r = np.arange(-R, R + 1, dtype=np.int64)
    mx, my, mz = np.meshgrid(r, r, r, indexing="ij")
    m2 = mx * mx + my * my + mz * mz
    keep = (m2 > 0) & (m2 <= mmax2)
    modes = np.stack([mx[keep], my[keep], mz[keep]]).astype(np.int32)
    w = np.exp(-(math.pi * math.pi / (alpha * L * L)) * m2[keep].astype(np.float64))
    return np.ascontiguousarray(modes), w
