"""Seeded synthetic inputs shaped like the paper's primitive-model electrolytes.

This module is shared by the tests, the benchmark and the smoke check.  It
draws positions, charges and velocities only; it contains none of the random
batch Ewald arithmetic.

Recipes (Sec. 4 of arXiv:2010.01559 describes primitive-model ions in a cubic
periodic box in reduced units):

* positions: independent uniform points in [0, L)^3; every point that lies
  closer than ``dmin`` (periodic minimum image) to a lower-indexed point is
  drawn again, until no such pair is left;
* charges: ``+1`` for the first half and ``-1`` for the second half of a 1:1
  electrolyte; optional divalent ``+2`` counter-ions balanced by extra ``-1``
  ions; or Gaussian charges shifted to zero net charge;
* velocities: Maxwell-Boltzmann at temperature kT for mass m.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
from scipy.spatial import cKDTree

DEFAULT_SEED = 20101559


def box_for_density(n: int, density: float) -> float:
    """Side of the cubic box holding n particles at number density n/L^3."""
    return (n / density) ** (1.0 / 3.0)


def alpha_for_real_space_error(density: float, r_cut: float, tol: float = 1e-4) -> float:
    """Splitting parameter whose Kolafa-Perram real-space RMS force estimate
    2 sqrt(density / r_cut) exp(-alpha r_cut^2) equals ``tol`` (unit charges)."""
    return (math.log(2.0 * math.sqrt(density / r_cut)) - math.log(tol)) / (r_cut * r_cut)


def positions(n: int, L: float, rng: np.random.Generator, dmin: float = 0.8, max_rounds: int = 1000) -> np.ndarray:
    """[3, n] float64 positions in [0, L) with no periodic pair closer than dmin."""
    pts = rng.random((n, 3)) * L
    if dmin <= 0.0 or n < 2:
        return np.ascontiguousarray(pts.T)
    for _ in range(max_rounds):
        tree = cKDTree(pts, boxsize=L)
        pairs = tree.query_pairs(dmin, output_type="ndarray")
        if pairs.size == 0:
            return np.ascontiguousarray(pts.T)
        redo = np.unique(np.maximum(pairs[:, 0], pairs[:, 1]))
        pts[redo] = rng.random((redo.size, 3)) * L
        # guard against points that landed exactly on L after scaling
        pts[pts >= L] = 0.0
    raise RuntimeError("could not place particles without overlaps; density too high for dmin")


def electrolyte_charges(n: int, divalent_fraction: float = 0.0) -> np.ndarray:
    """Charges of an electroneutral electrolyte.

    Without divalent ions: n/2 cations (+1) then n/2 anions (-1) (n even).
    With divalent fraction f: n2 = round(f n) ions of +2; the remaining
    n - n2 ions split into n_plus = (n - 3 n2)/2 cations (+1) and
    n_minus = n_plus + 2 n2 anions (-1); if n - n2 is odd, n2 is raised by one.
    """
    if divalent_fraction <= 0.0:
        if n % 2:
            raise ValueError("a 1:1 electrolyte needs an even particle count")
        return np.concatenate([np.ones(n // 2), -np.ones(n // 2)])
    n2 = int(round(divalent_fraction * n))
    if (n - n2) % 2:
        n2 += 1
    n_plus = (n - 3 * n2) // 2
    n_minus = n_plus + 2 * n2
    if n_plus < 0:
        raise ValueError("too many divalent ions for neutrality")
    q = np.concatenate([np.ones(n_plus), 2.0 * np.ones(n2), -np.ones(n_minus)])
    assert q.shape[0] == n and abs(q.sum()) < 1e-9
    return q


def gaussian_charges(n: int, rng: np.random.Generator, sigma: float = 0.5) -> np.ndarray:
    """N(0, sigma^2) charges shifted to zero net charge."""
    q = rng.normal(0.0, sigma, n)
    return q - q.mean()


def velocities(n: int, rng: np.random.Generator, kT: float = 1.0, mass: float = 1.0) -> np.ndarray:
    return np.ascontiguousarray(rng.normal(0.0, math.sqrt(kT / mass), (3, n)))


@dataclass
class System:
    """One synthetic system: inputs plus the method's parameters."""
    name: str
    n: int
    L: float
    alpha: float
    r_cut: float
    p: int
    pos: np.ndarray          # [3, n] float64
    q: np.ndarray            # [n] float64
    vel: np.ndarray          # [3, n] float64
    seed: int
    coulomb: float = 1.0
    lj: tuple = (0.0, 1.0, 2.5)   # (epsilon, sigma, cutoff); epsilon 0 disables
    kT: float = 1.0
    gamma: float = 1.0
    dt: float = 1e-3
    mass: float = 1.0
    extra: dict = field(default_factory=dict)


def electrolyte_system(name: str, n: int, density: float, alpha: float, r_cut: float, p: int, seed: int,
                       lj=(1.0, 1.0, 2.5), divalent_fraction: float = 0.0, dmin: float = 0.8,
                       L: float | None = None, **kw) -> System:
    rng = np.random.default_rng(seed)
    L = box_for_density(n, density) if L is None else L
    pos = positions(n, L, rng, dmin)
    q = electrolyte_charges(n, divalent_fraction)
    vel = velocities(n, rng, kw.get("kT", 1.0), kw.get("mass", 1.0))
    return System(name, n, L, alpha, r_cut, p, pos, q, vel, seed, lj=lj, **kw)


# -- the workloads used by the tests and the benchmark ------------------------

def small_fp64(seed: int = DEFAULT_SEED) -> System:
    """L=10, N=200 (+1 for the first 100, -1 for the rest), min distance 0.8,
    alpha=1, r_c=3.5, P=100; Coulomb only."""
    return electrolyte_system("rbe-small-n200-p100", 200, 200 / 1000.0, 1.0, 3.5, 100, seed,
                              lj=(0.0, 1.0, 2.5), L=10.0)


def langevin_electrolyte(seed: int = DEFAULT_SEED + 1) -> System:
    """N=3000 +-1 ions at density 0.1, alpha=0.5, r_c=3.5, P=100, shifted LJ
    (eps=1, sigma=1, cut 2.5), kT=1, gamma=1, dt=1e-3."""
    return electrolyte_system("electrolyte-n3000-p100", 3000, 0.1, 0.5, 3.5, 100, seed)


def scaling_system(n: int, p: int, seed: int = DEFAULT_SEED + 2) -> System:
    """+-1 ions at density 0.1, r_c=3.5, alpha from the 1e-4 real-space error
    estimate, LJ and Langevin parameters as in the 3000-ion electrolyte."""
    a = alpha_for_real_space_error(0.1, 3.5)
    return electrolyte_system(f"electrolyte-n{n}-p{p}", n, 0.1, a, 3.5, p, seed)


def metric_system(seed: int = DEFAULT_SEED) -> System:
    """The headline workload: N=1e5 +-1 ions at density 0.1 (L=100), r_c=3.5,
    P=100, alpha from the 1e-4 real-space error estimate."""
    a = alpha_for_real_space_error(0.1, 3.5)
    return electrolyte_system("electrolyte-n100000-p100", 100000, 0.1, a, 3.5, 100, seed, L=100.0)


def replica_systems(R: int = 64, nmin: int = 500, nmax: int = 20000, seed: int = DEFAULT_SEED + 3,
                    p: int = 100, divalent_fraction: float = 0.1) -> list:
    """R independent electrolytes with N ~ U[nmin, nmax], +-1 ions plus 10%
    divalent +2 counter-ions, each at density 0.1 in its own box, own seed."""
    rng = np.random.default_rng(seed)
    ns = rng.integers(nmin, nmax + 1, size=R)
    a = alpha_for_real_space_error(0.1, 3.5)
    out = []
    for r, n in enumerate(ns):
        out.append(electrolyte_system(f"replica{r}-n{int(n)}", int(n), 0.1, a, 3.5, p, seed + 1000 + r,
                                      divalent_fraction=divalent_fraction))
    return out


def gaussian_charge_system(n: int = 30000, seed: int = DEFAULT_SEED + 4, p: int = 200, alpha: float = 0.5,
                           density: float = 0.1) -> System:
    """Ions at density 0.1 with N(0, 0.5^2) charges shifted to zero net charge;
    alpha=0.5, r_c=3.5, P=200; Coulomb only."""
    rng = np.random.default_rng(seed)
    L = box_for_density(n, density)
    pos = positions(n, L, rng, 0.8)
    q = gaussian_charges(n, rng, 0.5)
    vel = velocities(n, rng)
    return System(f"gaussq-n{n}-p{p}", n, L, alpha, 3.5, p, pos, q, vel, seed, lj=(0.0, 1.0, 2.5))


def colloid_system(n_salt: int = 0, seed: int = DEFAULT_SEED + 5, p: int = 100) -> System:
    """The charge-inversion setup of Sec. 4.2 (after Lenz and Holm), lengths
    in Angstrom and energies in k_B T: one colloid of diameter 100 with a
    central charge -300 fixed at the centre of a periodic box of side 225.8,
    200 trivalent counterions (+3), 300 + n_salt monovalent coions (-1) and
    n_salt monovalent counterions (+1), all ions of diameter 4; Coulomb
    prefactor l_B = 7.1; shifted LJ with sigma = 1, epsilon = 1 and the cutoff
    R_c = 2^(1/6) on r - r_off, r_off = (d_i + d_j)/2 - sigma; alpha = 0.0072,
    r_c = 40, p = 100 (the random batch row of Table 4).  n_salt = 1300 is
    the 196 mM case.  The colloid is particle 0 and does not move; ions are
    uniform in the box, redrawn while closer than 52.5 to the colloid centre
    or 4 to a lower-indexed ion (periodic minimum image)."""
    L, d_col, d_ion = 225.8, 100.0, 4.0
    n_ion = 200 + (300 + n_salt) + n_salt
    n = 1 + n_ion
    rng = np.random.default_rng(seed)
    centre = np.full(3, 0.5 * L)
    pts = np.empty((n, 3))
    pts[0] = centre
    contact = 0.5 * (d_col + d_ion) + 0.5
    todo = np.arange(1, n)
    while todo.size:
        pts[todo] = rng.random((todo.size, 3)) * L
        d = pts[todo] - centre
        d -= L * np.round(d / L)
        bad = np.sqrt((d * d).sum(1)) < contact
        tree = cKDTree(pts[1:], boxsize=L)
        pairs = tree.query_pairs(d_ion, output_type="ndarray") + 1
        redo = set(todo[bad].tolist())
        if pairs.size:
            redo |= set(np.maximum(pairs[:, 0], pairs[:, 1]).tolist())
        todo = np.array(sorted(redo), dtype=int)
    pts[pts >= L] = 0.0
    q = np.concatenate([[-300.0], np.full(200, 3.0), np.full(300 + n_salt, -1.0), np.full(n_salt, 1.0)])
    assert abs(q.sum()) < 1e-9
    diam = np.full(n, d_ion)
    diam[0] = d_col
    vel = velocities(n, rng)
    vel[:, 0] = 0.0
    return System(f"colloid-n{n}-p{p}", n, L, 0.0072, 40.0, p, np.ascontiguousarray(pts.T), q, vel, seed,
                  coulomb=7.1, lj=(1.0, 1.0, 2.0 ** (1.0 / 6.0)), dt=0.002,
                  extra={"diameter": diam, "n_fixed": 1})
