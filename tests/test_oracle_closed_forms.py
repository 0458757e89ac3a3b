"""Pins for the closed forms: each checked against SciPy quadrature (an independent library
routine) or a defining differential identity."""
import numpy as np
from scipy import integrate

from oracle import closed_forms as cf


def _G(r):
    return -np.log(r) / (2 * np.pi)


def _square_by_quadpack(x, y, a1, b1, a2, b2):
    # split at the target so any singularity sits on a corner of each piece
    xs = sorted({a1, b1} | ({x} if a1 < x < b1 else set()))
    ys = sorted({a2, b2} | ({y} if a2 < y < b2 else set()))
    tot = 0.0
    for xa, xb in zip(xs[:-1], xs[1:]):
        for ya, yb in zip(ys[:-1], ys[1:]):
            v, _ = integrate.dblquad(lambda t, s: _G(np.hypot(x - s, y - t)), xa, xb, ya, yb,
                                     epsabs=1e-14, epsrel=1e-13)
            tot += v
    return tot


def test_square_potential_matches_quadpack():
    for (x, y) in [(0.3, -0.2), (0.999, 0.5), (1.2, 0.1), (-2.5, 3.0), (-1.0, 1.0)]:
        ref = _square_by_quadpack(x, y, -1.0, 1.0, -1.0, 1.0)
        assert abs(cf.square_potential(x, y, -1, 1, -1, 1) - ref) < 1e-12


def test_square_potential_poisson():
    h = 1e-3
    for (x, y, inside) in [(0.2, 0.3, True), (1.7, -0.4, False)]:
        lap = (cf.square_potential(x + h, y, -1, 1, -1, 1) + cf.square_potential(x - h, y, -1, 1, -1, 1)
               + cf.square_potential(x, y + h, -1, 1, -1, 1) + cf.square_potential(x, y - h, -1, 1, -1, 1)
               - 4 * cf.square_potential(x, y, -1, 1, -1, 1)) / h ** 2
        assert abs(-lap - (1.0 if inside else 0.0)) < 1e-5


def test_gaussian_potential_matches_radial_quadrature():
    sig, A = 0.13, 0.7
    f = lambda rho: A * np.exp(-rho ** 2 / (2 * sig ** 2))
    for r in [0.0, 1e-4, 0.05, 0.2, 0.9]:
        # u(r) = -int_0^inf rho f(rho) log max(r, rho) d rho
        inner = integrate.quad(lambda p: p * f(p) * np.log(r), 0, r, epsabs=1e-17, epsrel=1e-14)[0] if r > 0 else 0.0
        cuts = [r + k * sig for k in (0, 1, 2, 4, 8, 16, 40)]  # finite pieces; tail beyond 40 sigma < 1e-300
        outer = sum(integrate.quad(lambda p: p * f(p) * np.log(p), a, b, epsabs=1e-17, epsrel=1e-14, limit=200)[0]
                    for a, b in zip(cuts[:-1], cuts[1:]))
        ref = -(inner + outer)
        got = cf.gaussian_potential(r, 0.0, 0.0, 0.0, sig, A)
        assert abs(got - ref) < 1e-14


def test_ein_series_matches_exp1_branch():
    # the small-t series and E1(t) + log t + gamma must agree where both are accurate
    from scipy import special

    for t in (0.05, 0.2, 0.45):
        series = cf.ein(np.array([t]))[0]
        closed = special.exp1(t) + np.log(t) + cf.EULER_GAMMA
        assert abs(series - closed) < 1e-15
    # Ein(t) = int_0^t (1 - e^-s)/s ds
    ref = integrate.quad(lambda s: -np.expm1(-s) / s, 0, 0.7, epsabs=1e-17, epsrel=1e-15)[0]
    assert abs(cf.ein(np.array([0.7]))[0] - ref) < 1e-15


def test_exterior_tail_small_for_centred_narrow_source():
    v = cf.gaussian_exterior_tail(0.1, -0.2, 0.0, 0.0, 0.1, 1.0)
    assert abs(v) < 1e-18
