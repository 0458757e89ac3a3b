"""Pins of the strip oracle (Sec. 4.3, multidomain spectral collocation).

* The differentiation and interpolation matrices are exact on polynomials of degree < n.
* A manufactured solution on the annulus between two circles (v = (r - a)(b - r) g(theta), which
  vanishes on both, f = Lap v in closed form) is recovered to spectral accuracy, and the error
  decreases as the radial resolution grows.
* f = 0 gives v = 0; the solution is linear in f.
"""
import numpy as np
import pytest

from oracle import strip


def test_matrices_exact_on_polynomials():
    x = strip.cheb2(12)
    D = strip.diff_matrix(x)
    rng = np.random.default_rng(0)
    c = rng.standard_normal(12)
    p = np.polynomial.Polynomial(c)
    assert np.max(np.abs(D @ p(x) - p.deriv()(x))) < 1e-11 * np.max(np.abs(p.deriv()(x)))
    s, _ = np.polynomial.legendre.leggauss(12)
    E = strip.interp_matrix(s, x)
    assert np.max(np.abs(E @ p(s) - p(x))) < 1e-12 * np.max(np.abs(p(x)))


def _annulus(n_panel, n_gl, R):
    s, _ = np.polynomial.legendre.leggauss(n_gl)
    h = np.pi / n_panel
    th = (2 * h * np.arange(n_panel))[:, None] + h * (s[None, :] + 1)
    return np.stack([R * np.cos(th), R * np.sin(th)], axis=2)


def _manufactured(a, b):
    # v = phi(r) g(theta), phi = (r - a)(b - r) e^(2r): zero on both circles, not a polynomial in r
    def parts(p):
        r, th = np.hypot(p[:, 0], p[:, 1]), np.arctan2(p[:, 1], p[:, 0])
        e = np.exp(2 * r)
        q, q1 = (r - a) * (b - r), (a + b) - 2 * r
        phi = q * e
        phi1 = (q1 + 2 * q) * e
        phi2 = (-2.0 + 4 * q1 + 4 * q) * e
        g = 1 + 0.3 * np.cos(3 * th) + 0.2 * np.sin(2 * th)
        g2 = -2.7 * np.cos(3 * th) - 0.8 * np.sin(2 * th)
        return r, phi, phi1, phi2, g, g2

    def v(p):
        _, phi, _, _, g, _ = parts(p)
        return phi * g

    def f(p):
        r, phi, phi1, phi2, g, g2 = parts(p)
        return g * (phi2 + phi1 / r) + phi * g2 / (r * r)

    return v, f


def test_manufactured_solution_on_annulus():
    a, b = 0.75, 0.9  # Gamma~ inside, Gamma outside
    v, f = _manufactured(a, b)
    errs = []
    for n_r in (4, 6, 10, 16):
        sol, X = strip.solve(_annulus(12, 16, b), _annulus(12, 16, a), f, q=16, n_r=n_r)
        ve = v(X.reshape(-1, 2))
        errs.append(np.max(np.abs(sol.reshape(-1) - ve)) / np.max(np.abs(ve)))
    assert errs[0] > errs[1] > errs[2]  # spectral convergence across the strip
    assert errs[-1] < 1e-12  # saturates near 1.5e-14 (rounding of the row-equilibrated solve)


def test_zero_and_linearity():
    a, b = 0.75, 0.9
    gam, gamt = _annulus(8, 16, b), _annulus(8, 16, a)
    z, _ = strip.solve(gam, gamt, lambda p: np.zeros(p.shape[0]), q=12, n_r=10)
    assert np.max(np.abs(z)) == 0.0
    f1 = lambda p: np.sin(3 * p[:, 0]) * p[:, 1]
    f2 = lambda p: np.exp(p[:, 0] - p[:, 1])
    s1, _ = strip.solve(gam, gamt, f1, q=12, n_r=10)
    s2, _ = strip.solve(gam, gamt, f2, q=12, n_r=10)
    s12, _ = strip.solve(gam, gamt, lambda p: 2 * f1(p) - f2(p), q=12, n_r=10)
    assert np.max(np.abs(s12 - (2 * s1 - s2))) < 1e-13 * np.max(np.abs(s12))  # row-scaled condition number about 1e2


def test_full_size_manufactured_and_zero_boundary():
    # 56 thin elements at 24 x 16 (the size of the benchmark strip): the row norms span seven
    # decades here, and the solve must still hold the boundary rows at zero and the manufactured
    # solution to near rounding
    a, b = 0.85, 0.9
    v, f = _manufactured(a, b)
    sol, X = strip.solve(_annulus(56, 16, b), _annulus(56, 16, a), f, q=24, n_r=16)
    ve = v(X.reshape(-1, 2)).reshape(sol.shape)
    assert np.max(np.abs(sol - ve)) < 1e-12 * np.max(np.abs(ve))
    assert np.max(np.abs(sol[:, 0])) < 1e-15 and np.max(np.abs(sol[:, -1])) < 1e-15
