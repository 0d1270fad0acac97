"""Pins of the oracle's normaliser, random numbers and mode samplers.

Paper: Sec. 3.1, eqs. (3.1)-(3.5).  Nothing here needs a GPU.
"""
import math

import numpy as np
import pytest
from scipy import stats

import oracle as O
from conftest import read_golden


# -- H and S: eqs. (3.1)-(3.2) -------------------------------------------------

@pytest.mark.parametrize("alpha,L", [(1.0, 10.0), (0.5, 31.07232505953859), (0.6633, 100.0),
                                      (0.05, 3.0), (0.3, 2.0), (2.0, 1.5)])
def test_H_direct_equals_poisson_dual(alpha, L):
    # the two sides of eq. (3.2) are independent series; small alpha L^2 makes
    # the dual side need several terms, large alpha L^2 the direct side
    hd, hp = O.H_direct(alpha, L), O.H_dual(alpha, L)
    assert abs(hd - hp) <= 2e-14 * hd


def test_H_closed_form_small_box():
    # alpha L^2 = 100: the dual series is 1 + 2 e^-100 + ..., i.e. sqrt(100/pi) to FP64
    assert O.H_direct(1.0, 10.0) == pytest.approx(math.sqrt(100.0 / math.pi), rel=1e-15)


@pytest.mark.parametrize("alpha,L,mmax", [(1.0, 3.0, 12), (0.4, 5.0, 16), (2.0, 2.0, 10)])
def test_S_equals_lattice_sum(alpha, L, mmax):
    # eq. (3.1): S = sum over k != 0 of exp(-k^2/4alpha) equals H^3 - 1
    assert O.S(alpha, L) == pytest.approx(O.S_bruteforce(alpha, L, mmax), rel=1e-13)


def test_paper_truncated_H():
    # the truncation at m = +-1 of the dual series (Sec. 3.1) is exact to FP64
    # once alpha L^2 >> 1
    for alpha, L in [(1.0, 10.0), (0.5, 31.07)]:
        approx = math.sqrt(alpha * L * L / math.pi) * (1.0 + 2.0 * math.exp(-alpha * L * L))
        assert O.H_direct(alpha, L) == pytest.approx(approx, rel=1e-14)


# -- Philox4x32-10 ----------------------------------------------------------------

def test_philox_known_answers():
    for row in read_golden("philox4x32_10_kat.txt"):
        v = [int(x, 16) for x in row]
        out = O.philox(v[0:4], v[4:6])
        assert [int(x) for x in out] == v[6:10]


# -- exact i.i.d. sampler: eq. (3.3) ---------------------------------------------

def _pmf_1d(alpha, L, M):
    m = np.arange(-M, M + 1)
    w = np.exp(-math.pi ** 2 * m * m / (alpha * L * L))
    return m, w / w.sum()


def test_cdf_table_shape():
    alpha, L = 1.0, 10.0
    cdf = O.mode_cdf(alpha, L)
    M = O.mode_range(alpha, L)
    assert cdf.shape == (2 * M + 1,)
    assert np.all(np.diff(cdf) >= 0) and cdf[-1] == 1.0
    _, pmf = _pmf_1d(alpha, L, M)
    assert np.allclose(np.diff(np.concatenate([[0.0], cdf])), pmf, atol=1e-16)


def _draw_many(alpha, L, nsteps, p, seed=7, sampler=None):
    out = []
    for s in range(nsteps):
        if sampler is None:
            m, _ = O.sample_modes(alpha, L, p, seed, s)
        else:
            m = sampler(s)
        out.append(m)
    return np.concatenate(out, axis=1)


def _second_moment_z(alpha, L, modes):
    """z-score of the sample mean of m_d^2 against its exact value under P_k
    conditioned on m != 0: E[m_x^2] / (1 - P(0)^3) (m_x^2 vanishes on m = 0)."""
    M = O.mode_range(alpha, L)
    mv, pmf = _pmf_1d(alpha, L, M)
    exact = (pmf * mv * mv).sum() / (1.0 - pmf[M] ** 3)
    x = (modes.astype(np.float64) ** 2).ravel()
    return (x.mean() - exact) / (x.std() / math.sqrt(x.size))


def _marginal_and_shell_chi2(alpha, L, modes):
    """chi^2 p-values of the x-marginal and of the |m|^2 shell histogram of the
    target distribution P_k conditioned on m != 0 (eq. 3.3)."""
    M = O.mode_range(alpha, L)
    mv, pmf = _pmf_1d(alpha, L, M)
    p0 = pmf[M]
    # marginal of m_x given the 3-vector is non-zero
    marg = pmf * (1.0 - np.where(mv == 0, p0 * p0, 0.0)) / (1.0 - p0 ** 3)
    ntot = modes.shape[1]
    cnt = np.array([(modes[0] == v).sum() for v in mv], float)
    exp_ = marg * ntot
    keep = exp_ > 5
    chi_m = ((cnt[keep] - exp_[keep]) ** 2 / exp_[keep]).sum()
    pm = stats.chi2.sf(chi_m, keep.sum() - 1)
    # shells |m|^2 by enumeration of the 3-D lattice
    R = min(M, 40)
    g = np.arange(-R, R + 1)
    w1 = np.exp(-math.pi ** 2 * g * g / (alpha * L * L))
    W = w1[:, None, None] * w1[None, :, None] * w1[None, None, :]
    m2 = g[:, None, None] ** 2 + g[None, :, None] ** 2 + g[None, None, :] ** 2
    W[R, R, R] = 0.0
    W /= W.sum()
    shells = np.bincount(m2.ravel(), weights=W.ravel())
    obs = np.bincount((modes.astype(np.int64) ** 2).sum(0), minlength=shells.size)[: shells.size]
    e = shells * ntot
    keep = e > 5
    chi_s = ((obs[keep] - e[keep]) ** 2 / e[keep]).sum()
    ps = stats.chi2.sf(chi_s, keep.sum() - 1)
    return pm, ps


@pytest.mark.parametrize("alpha,L", [(1.0, 10.0), (0.3, 5.0)])
def test_exact_sampler_chi2(alpha, L):
    modes = _draw_many(alpha, L, 400, 500)
    assert not np.any((modes == 0).all(axis=0)), "the zero mode must be discarded"
    pm, ps = _marginal_and_shell_chi2(alpha, L, modes)
    assert pm > 1e-4 and ps > 1e-4, (pm, ps)
    assert abs(_second_moment_z(alpha, L, modes)) < 5
    # symmetric components
    M = O.mode_range(alpha, L)
    mv, pmf = _pmf_1d(alpha, L, M)
    for d in range(3):
        assert abs(modes[d].mean()) < 5 * math.sqrt((pmf * mv * mv).sum() / modes.shape[1])


def test_exact_sampler_is_inverse_cdf_of_its_uniforms():
    alpha, L, seed, step = 1.0, 10.0, 99, 3
    modes, rej = O.sample_modes(alpha, L, 64, seed, step)
    cdf = O.mode_cdf(alpha, L)
    M = O.mode_range(alpha, L)
    for l in range(64):
        # find the accepted attempt: the first with a non-zero vector
        for a in range(50):
            u = O.sample_uniforms(seed, step, l, a)
            m = np.searchsorted(cdf, u, side="right") - M
            if np.any(m != 0):
                break
        assert np.array_equal(m, modes[:, l])


def test_sampler_depends_on_seed_and_step():
    a = O.sample_modes(1.0, 10.0, 100, 1, 0)[0]
    b = O.sample_modes(1.0, 10.0, 100, 1, 1)[0]
    c = O.sample_modes(1.0, 10.0, 100, 2, 0)[0]
    d = O.sample_modes(1.0, 10.0, 100, 1, 0)[0]
    assert np.array_equal(a, d)
    assert not np.array_equal(a, b) and not np.array_equal(a, c)


# -- the paper's Metropolis-Hastings variant: eqs. (3.4)-(3.5) --------------------

def test_mh_proposal_mass_matches_rounded_gaussian():
    alpha, L = 1.0, 10.0
    sd = math.sqrt(alpha * L * L / (2 * math.pi ** 2))
    for m in range(0, 12):
        lo, hi = (m - 0.5) / sd, (m + 0.5) / sd
        ref = stats.norm.cdf(hi) - stats.norm.cdf(lo)
        if m == 0:
            ref = stats.norm.cdf(0.5 / sd) - stats.norm.cdf(-0.5 / sd)
        assert O.mh_proposal_mass(alpha, L, m) == pytest.approx(ref, rel=1e-9, abs=1e-300)
        assert O.mh_proposal_mass(alpha, L, -m) == O.mh_proposal_mass(alpha, L, m)


def _mh_draws(alpha, L, nsteps, p, skip_accept=False):
    st = np.zeros(3, np.int32)
    out = []
    for s in range(nsteps):
        m, st, _ = O.sample_modes_mh(alpha, L, p, 11, s, st, skip_accept)
        out.append(m)
    return np.concatenate(out, axis=1)


def test_mh_sampler_targets_P_k():
    alpha, L = 1.0, 10.0
    modes = _mh_draws(alpha, L, 400, 500)
    assert not np.any((modes == 0).all(axis=0))
    pm, ps = _marginal_and_shell_chi2(alpha, L, modes)
    assert pm > 1e-4 and ps > 1e-4, (pm, ps)
    # successive MH states are correlated (a rejection repeats the state), so
    # the z bound is looser than for i.i.d. draws
    assert abs(_second_moment_z(alpha, L, modes)) < 6


def test_mh_without_acceptance_is_caught():
    # planted mistake: accepting every proposal samples the rounded Gaussian
    # of eq. (3.5) instead of P(m) of eq. (3.4); the chi^2 pins must see it
    alpha, L = 1.0, 10.0
    modes = _mh_draws(alpha, L, 400, 500, skip_accept=True)
    pm, ps = _marginal_and_shell_chi2(alpha, L, modes)
    # the rounded Gaussian has variance sigma^2 + 1/12: about 1.6% too large at
    # alpha L^2 = 100, which the second-moment test resolves at ~9 sigma
    assert min(pm, ps) < 1e-2
    assert _second_moment_z(alpha, L, modes) > 6
