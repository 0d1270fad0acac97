"""CPU: the library's classical-Ewald mode list (rbe_ewald_modes, used by the
comparator through rbe_set_k_ewald) equals the oracle's enumeration of
0 < |m|^2 <= mmax2 with weights exp(-k^2 / (4 alpha)) (eq. 2.9, second term),
and rbe_ewald_radius2 is the largest |m|^2 whose weight is still >= tol."""
import math

import numpy as np
import pytest

import oracle as O
import paper_2010_01559_amd.rbe as R
from paper_2010_01559_amd.ewald import ewald_modes, mode_radius2


def _key(m):
    return np.lexsort(m[::-1])


def test_modes_and_weights_match_oracle():
    for alpha, L, m2 in ((0.6633, 21.5, 40), (1.0, 10.0, 100), (0.5, 31.07, 17), (0.3, 8.0, 1)):
        m, w = ewald_modes(alpha, L, m2)
        mo, wo = O.ewald_modes(alpha, L, m2)
        assert m.shape == mo.shape
        a, b = _key(m), _key(mo)
        assert np.array_equal(m[:, a], mo[:, b])
        assert np.allclose(w[a], wo[b], rtol=1e-14, atol=0)


def test_mode_order_and_count():
    # m_x outermost, m_z innermost, each from -floor(sqrt(mmax2)); the ball
    # of radius^2 2 holds the 6 axis and 12 face-diagonal vectors
    m, w = ewald_modes(1.0, 10.0, 2)
    assert m.shape == (3, 18)
    assert np.array_equal(m[:, 0], [-1, -1, 0]) and np.array_equal(m[:, -1], [1, 1, 0])
    assert all(tuple(m[:, i]) < tuple(m[:, i + 1]) for i in range(17))
    assert np.allclose(w[m[0] ** 2 + m[1] ** 2 + m[2] ** 2 == 1], math.exp(-math.pi ** 2 / 100.0), rtol=1e-15)


def test_radius_from_tolerance():
    for alpha, L, tol in ((0.6633, 46.416, 1e-4), (0.55, 10.0, 1e-8), (2.0, 5.0, 0.5)):
        m2 = mode_radius2(alpha, L, tol)
        f = lambda k2: math.exp(-math.pi ** 2 * k2 / (alpha * L * L))
        assert f(m2) >= tol > f(m2 + 1)


def test_bad_arguments_are_rejected():
    for args in ((0.0, 10.0, 1e-4), (1.0, -1.0, 1e-4), (1.0, 10.0, 1.5), (1.0, 1e6, 1e-300)):
        with pytest.raises(R.RBEError):
            R.rbe_ewald_radius2(*args)
    with pytest.raises(R.RBEError):
        R.rbe_ewald_modes(1.0, 10.0, 0)
