"""CPU: the package's classical-Ewald mode list (used by the comparator)
equals the oracle's enumeration of 0 < |m|^2 <= mmax2 with weights
exp(-k^2 / (4 alpha)) (paper eq. 2.9, second term)."""
import math

import numpy as np

import oracle as O
from paper_2010_01559_amd.ewald import ewald_modes, mode_radius2


def _key(m):
    return np.lexsort(m[::-1])


def test_modes_and_weights_match_oracle():
    for alpha, L, m2 in ((0.6633, 21.5, 40), (1.0, 10.0, 100), (0.5, 31.07, 17)):
        m, w = ewald_modes(alpha, L, m2)
        mo, wo = O.ewald_modes(alpha, L, m2)
        assert m.shape == mo.shape
        a, b = _key(m), _key(mo)
        assert np.array_equal(m[:, a], mo[:, b])
        assert np.allclose(w[a], wo[b], rtol=1e-14, atol=0)


def test_radius_from_tolerance():
    alpha, L, tol = 0.6633, 46.416, 1e-4
    m2 = mode_radius2(alpha, L, tol)
    f = lambda k2: math.exp(-math.pi ** 2 * k2 / (alpha * L * L))
    assert f(m2) >= tol > f(m2 + 1)
