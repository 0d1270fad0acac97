"""Observables of the paper's electrolyte validation (Sec. 4.1).

* Pair correlations g_++, g_+-, g_-- from the library's pair counts
  (``rbe_pair_histogram``), normalised by the ideal-gas count of each shell.
* The charge density around a cation, q (n_+ g_++(r) - n_- g_+-(r)) with
  n_+/- the number densities of the two species: the quantity the
  Debye-Hueckel theory of the appendix predicts, -kappa^2 eps phi(r); the
  paper calls it the charge-charge correlation rho(r) = g_++ - g_+-, whose
  DH line ln(r |rho|) = -kappa r + ln(kappa^2 q e^{kappa a} / (4 pi (1 + kappa a)))
  is the line for this charge density.
* Potential energy per particle and pressure of eq. (4.3):
  E_pot = (E_Coul + E_LJ) / N and P = 2/(3V) (sum m v^2/2 - vir), with
  vir = (1/2) sum_{i<j} r_ij . F_ij including the Fourier part.

Host arithmetic on results the GPU library returns; no kernel work here.
"""
from __future__ import annotations

import math

import numpy as np

from . import rbe as R


def pair_counts(ctx, pos, q, r_max, nbins, counts=None):
    """Adds one configuration's pair counts to counts (device int64
    [R, 3, nbins], allocated zeroed when None) and returns it."""
    import torch
    if counts is None:
        counts = torch.zeros((ctx.R, 3, int(nbins)), dtype=torch.int64, device="cuda")
    R.rbe_pair_histogram(ctx, pos, q, r_max, nbins, counts)
    return counts


def pair_correlations(counts, n_plus, n_minus, L, r_max, samples=1):
    """(r, g_++, g_+-, g_--) from counts [3, nbins] accumulated over `samples`
    configurations of one system with n_plus cations and n_minus anions."""
    counts = np.asarray(counts, np.float64)
    nbins = counts.shape[-1]
    dr = r_max / nbins
    edges = np.arange(nbins + 1) * dr
    shell = 4.0 * math.pi / 3.0 * (edges[1:] ** 3 - edges[:-1] ** 3)
    V = L ** 3
    pairs = np.array([n_plus * (n_plus - 1) / 2.0, float(n_plus) * n_minus, n_minus * (n_minus - 1) / 2.0])
    ideal = pairs[:, None] * shell[None, :] / V * samples
    g = counts / ideal
    r = 0.5 * (edges[1:] + edges[:-1])
    return r, g[0], g[1], g[2]


def charge_density_around_cation(g_pp, g_pm, n_plus, n_minus, L, q=1.0):
    """q (n_+ g_++ - n_- g_+-): net charge density at distance r from a cation."""
    V = L ** 3
    return q * (n_plus / V * np.asarray(g_pp) - n_minus / V * np.asarray(g_pm))


def debye_huckel(density, a, q=1.0, kT=1.0, eps=1.0 / (4.0 * math.pi)):
    """(kappa, intercept) of the DH line ln(r |rho(r)|) = -kappa r + intercept
    for a symmetric electrolyte of total number density `density`, charges
    +-q, contact distance a, permittivity eps (1/(4 pi) in the paper's reduced
    units, where the potential of a charge is q/r)."""
    kappa = math.sqrt(q * q * density / (eps * kT))
    intercept = math.log(kappa * kappa * q * math.exp(kappa * a) / (4.0 * math.pi * (1.0 + kappa * a)))
    return kappa, intercept


def potential_energy_per_particle(e, n):
    """E_pot of eq. (4.3) from an rbe_energy dictionary."""
    return (e["e_kspace"] + e["e_self"] + e["e_real"] + e["e_lj"]) / n


def pressure(e, L):
    """P of eq. (4.3) from an rbe_energy dictionary (velocities given)."""
    vir = 0.5 * (e["virial"] + e["virial_kspace"])
    return 2.0 / (3.0 * L ** 3) * (e["e_kin"] - vir)
