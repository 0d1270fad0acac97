"""Fit of the scaled complementary error function used by the real-space
kernels in single precision.

erfc(x) = exp(-x^2) * h(x), and h(x) = sum_k c_k t^(k+1) with t = 1 / (1 + p x)
for x >= 0 -- the form of Abramowitz & Stegun 7.1.26, refitted here to a
higher degree so that the *relative* error of erfc stays near single-precision
rounding over the whole range the kernels use (beta r <= X_MAX).  The fit is
a weighted least-squares solve iterated towards equal-ripple relative error
(Lawson's algorithm); it uses only numpy and scipy.special.erfc (as the
reference in double precision).

Run ``python fit_erfc.py`` to print the coefficient table pasted into
rbe_real.hip and the achieved maximum relative error.
"""
import numpy as np
from scipy.special import erfc, erfcx

P = 0.47047        # scale of t; any value near 0.3-0.5 works
DEGREE = 9
X_MAX = 8.0


def design(x):
    t = 1.0 / (1.0 + P * x)
    return np.stack([t ** (k + 1) for k in range(DEGREE)], axis=1)


def fit():
    x = np.concatenate([np.linspace(0.0, X_MAX, 20001), np.linspace(0.0, 1.0, 2001)])
    h = erfcx(x)                       # erfc(x) exp(x^2), accurate in double
    A = design(x)
    w = np.ones_like(x)
    for _ in range(60):
        Aw = A * (w / h)[:, None]
        c, *_ = np.linalg.lstsq(Aw, w, rcond=None)
        rel = np.abs(A @ c - h) / h
        w = w * (rel / rel.max() + 1e-3) ** 0.5
        w /= w.max()
    return c


def evaluate(c, x):
    t = 1.0 / (1.0 + P * x)
    s = 0.0
    for k in reversed(range(DEGREE)):
        s = s * t + c[k]
    return s * t * np.exp(-x * x)


if __name__ == "__main__":
    c = fit()
    x = np.linspace(0.0, X_MAX, 400001)
    rel = np.abs(evaluate(c, x) - erfc(x)) / erfc(x)
    print(f"// p = {P!r}; degree {DEGREE}; max relative error on [0, {X_MAX}] = {rel.max():.3e} (double)")
    print(f"    float s = {c[-1]:.9e}f;")
    for k in reversed(range(DEGREE - 1)):
        print(f"    s = fmaf(s, t, {c[k]:.9e}f);")
