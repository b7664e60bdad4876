"""Derives the polynomial of the seed proposer's normal CDF (norm_cdf in
mlp_kernels.hpp): for u >= 0 write erfc(u) = t exp(-u^2 + P(t)) with
t = 1 / (1 + u / 2), so that P(t) = ln(erfc(u) / t) + u^2 is smooth on
t in [0, 1] (P(0) = -ln(2 sqrt(pi)) from the asymptotic series of erfc), and
interpolate P at 200 Chebyshev nodes by a degree-9 polynomial (the classical
construction, e.g. Numerical Recipes Sec. 6.2).  Prints the power-basis
coefficients and the largest |error of P| on a fine grid, which is the
largest relative error of erfc in exact arithmetic (about 1.0e-7).

Run: python norm_cdf_fit.py
"""
from math import erfc, log, pi, sqrt

import numpy as np

DEG = 9


def p_exact(t: float) -> float:
    if t == 0.0:
        return -log(2.0 * sqrt(pi))
    u = 2.0 * (1.0 / t - 1.0)
    if u > 26.0:   # erfc underflows in double: asymptotic series
        s = 1 - 1 / (2 * u * u) + 3 / (4 * u ** 4) - 15 / (8 * u ** 6) + 105 / (16 * u ** 8)
        return log(s / (u * sqrt(pi) * t))
    return log(erfc(u) / t) + u * u


def fit(deg: int = DEG):
    k = np.arange(200)
    x = 0.5 - 0.5 * np.cos(np.pi * (k + 0.5) / 200)
    cheb = np.polynomial.chebyshev.Chebyshev.fit(x, [p_exact(v) for v in x], deg, domain=[0, 1])
    poly = cheb.convert(kind=np.polynomial.Polynomial, domain=[-1, 1], window=[-1, 1])
    grid = np.linspace(0.0, 1.0, 20001)
    err = float(np.max(np.abs(np.array([p_exact(v) for v in grid]) - poly(grid))))
    return list(poly.coef), err


if __name__ == "__main__":
    coef, err = fit()
    for i, c in enumerate(coef):
        print(f"c{i} = {c:.17g}")
    print(f"max |P error| = {err:.3e}")
