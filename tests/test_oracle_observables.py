"""CPU pins of the oracle's observables (Sec. 4.1: eq. 4.3 and the
charge-charge correlation): pair counts against an independent numpy
enumeration and a rock-salt lattice with known shells; the virial sums
against the scaling derivative of the energies and against the Ewald trace
identity (for a pure Coulomb system the total virial equals minus the total
electrostatic energy, whatever the splitting)."""
import numpy as np
import pytest

import oracle as O


def _numpy_counts(pos, q, L, r_max, nbins):
    n = q.shape[0]
    i, j = np.triu_indices(n, 1)
    d = pos[:, j] - pos[:, i]
    d -= L * np.round(d / L)
    r = np.sqrt((d * d).sum(0))
    keep = r < r_max
    b = np.floor(r[keep] / (r_max / nbins)).astype(int)
    cls = 2 - ((q[i[keep]] > 0).astype(int) + (q[j[keep]] > 0).astype(int))
    out = np.zeros((3, nbins), np.int64)
    np.add.at(out, (cls, b), 1)
    return out


def test_pair_histogram_matches_numpy():
    rng = np.random.default_rng(3)
    L = 7.0
    pos = rng.random((3, 150)) * L
    q = np.where(rng.random(150) < 0.5, 1.0, -1.0)
    for r_max, nb in ((3.5, 70), (2.0, 13)):
        assert np.array_equal(O.pair_histogram(pos, q, L, r_max, nb), _numpy_counts(pos, q, L, r_max, nb))


def test_pair_histogram_rock_salt_shells():
    g = np.arange(4.0)
    x, y, z = np.meshgrid(g, g, g, indexing="ij")
    pos = np.stack([x.ravel(), y.ravel(), z.ravel()])
    q = np.where((x + y + z).ravel() % 2 == 0, 1.0, -1.0)
    c = O.pair_histogram(pos, q, 4.0, 2.0, 200)
    r = (np.arange(200) + 0.5) * 0.01

    def shell(r0):
        sel = np.abs(r - r0) < 0.011
        return c[:, sel].sum(1)

    assert shell(1.0).tolist() == [0, 192, 0]           # 6 opposite-charge neighbours each
    assert shell(np.sqrt(2)).tolist() == [192, 0, 192]  # 12 like-charge neighbours each
    assert shell(np.sqrt(3)).tolist() == [0, 256, 0]    # 8 opposite-charge neighbours each
    assert c.sum() == 192 + 384 + 256                   # distance 2 = L/2 lies outside r < r_max


def _system(n=40, L=8.0, seed=5):
    rng = np.random.default_rng(seed)
    pos = rng.random((3, n)) * L
    q = rng.normal(size=n)
    q -= q.mean()
    return pos, q, L


def test_pair_virial_is_the_scaling_derivative():
    """r_ij . F_ij summed over pairs equals d U / d lambda for positions and
    box scaled by lambda at fixed splitting (real-space and LJ parts)."""
    pos, q, L = _system()
    alpha, rc, lj = 2.5, 4.0, (1.0, 0.4, 2.0)
    wr, wl = O.pair_virial(pos, q, L, alpha, rc, 1.0, lj)
    h = 1e-6

    def energies(lam):
        _, er, el = O.real_force(lam * pos, q, lam * L, alpha, rc, 1.0, lj)
        return er.sum(), el.sum()

    up, um = energies(1 + h), energies(1 - h)
    assert wr == pytest.approx((up[0] - um[0]) / (2 * h), rel=1e-7)
    assert wl == pytest.approx((up[1] - um[1]) / (2 * h), rel=1e-6, abs=1e-9)


def test_kspace_virial_is_the_scaling_derivative():
    pos, q, L = _system()
    alpha = 1.0
    m, w = O.ewald_modes(alpha, L, 60)
    wk = O.kspace_virial(pos, q, L, alpha, m, w)
    h = 1e-6

    def ek(lam):
        # weights exp(-k^2/4 alpha) follow the scaled box
        _, wl = O.ewald_modes(alpha, lam * L, 60)
        return O.kspace_energy(lam * pos, q, lam * L, m, wl)

    assert wk == pytest.approx((ek(1 + h) - ek(1 - h)) / (2 * h), rel=1e-7)


def test_virial_trace_identity_for_converged_ewald():
    pos, q, L = _system()
    alpha, rc = 2.5, 4.0
    wr, _ = O.pair_virial(pos, q, L, alpha, rc)
    m, w = O.ewald_modes(alpha, L, 700)
    wk = O.kspace_virial(pos, q, L, alpha, m, w)
    _, er, _ = O.real_force(pos, q, L, alpha, rc)
    utot = er.sum() + O.kspace_energy(pos, q, L, m, w) + O.self_energy(q, alpha)
    scale = abs(wr) + abs(wk) + abs(utot)
    assert abs(wr + wk + utot) <= 1e-12 * scale
