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


def _breakpoints(lo, hi, focus, d, step):
    # panel ends on [lo, hi]: graded geometrically (ratio 2) away from the point of the interval
    # nearest the target, plus a uniform grid of the given step
    pts = {lo, hi}
    k = -1
    while d * 2.0 ** k < hi - lo:
        for v in (focus - d * 2.0 ** k, focus + d * 2.0 ** k):
            if lo < v < hi:
                pts.add(v)
        k += 1
    n = int(np.ceil((hi - lo) / step))
    pts.update(float(v) for v in np.linspace(lo, hi, n + 1)[1:-1])
    return np.array(sorted(pts))


def _composite_gauss(bp, ng=24):
    t, w = np.polynomial.legendre.leggauss(ng)
    a, b = bp[:-1, None], bp[1:, None]
    return (0.5 * (a + b) + 0.5 * (b - a) * t).ravel(), (0.5 * (b - a) * w).ravel()


def _tail_cartesian(x, y, cx, cy, sig, amp, reach=14.0):
    """The exterior tail by brute force in Cartesian coordinates: the complement of [-1,1]^2 cut
    into four rectangles (left and right strips, and the top and bottom pieces between them),
    each clipped to the square of half-side 14 sigma about the centre (exp(-98) beyond), and
    integrated by tensor composite 24-point Gauss-Legendre rules graded towards the target."""
    d = min(1.0 - abs(x), 1.0 - abs(y))
    X0, X1, Y0, Y1 = cx - reach * sig, cx + reach * sig, cy - reach * sig, cy + reach * sig
    tot = 0.0
    for a1, b1, a2, b2 in ((X0, -1.0, Y0, Y1), (1.0, X1, Y0, Y1), (-1.0, 1.0, 1.0, Y1), (-1.0, 1.0, Y0, -1.0)):
        if b1 <= a1 or b2 <= a2:
            continue
        xs, wx = _composite_gauss(_breakpoints(a1, b1, min(max(x, a1), b1), d, sig / 2))
        ys, wy = _composite_gauss(_breakpoints(a2, b2, min(max(y, a2), b2), d, sig / 2))
        dx, dy = x - xs[:, None], y - ys[None, :]
        g = _G(np.sqrt(dx * dx + dy * dy)) * amp * np.exp(
            -((xs[:, None] - cx) ** 2 + (ys[None, :] - cy) ** 2) / (2 * sig * sig))
        tot += wx @ g @ wy
    return tot


def test_exterior_tail_matches_cartesian_brute_force():
    # the polar-coordinate tail against an independent Cartesian quadrature, at targets inside
    # and near the edges and corners of the root, for sources with up to 9 % of their mass outside
    # (config 1's worst case: sigma = 0.3 centred at (0.5, 0.5))
    cases = [(0.2, -0.1, 0.5, 0.5, 0.3, 1.0), (0.9, 0.95, 0.5, 0.5, 0.3, -0.7), (0.0, 0.0, 0.5, 0.5, 0.3, 1.0),
             (-0.99, 0.3, -0.4, 0.3, 0.25, 0.6), (0.6, -0.999, 0.6, -0.7, 0.2, 1.3)]
    for x, y, cx, cy, s, a in cases:
        ref = _tail_cartesian(x, y, cx, cy, s, a)
        got = cf.gaussian_exterior_tail(x, y, cx, cy, s, a)
        assert abs(ref) > 1e-4  # a tail that vanishes could not tell a wrong routine from a right one
        assert abs(got - ref) <= 1e-13 * abs(ref), (x, y, got, ref)


def test_exterior_tail_completes_the_whole_plane_potential():
    # the whole-plane potential minus the exterior tail is the potential of the part inside the
    # root: check it at a target against a Cartesian quadrature of the inside, split at the target
    x, y, cx, cy, s, a = 0.3, -0.45, 0.5, 0.5, 0.3, 1.0
    inside = 0.0
    for a1, b1 in ((-1.0, x), (x, 1.0)):
        for a2, b2 in ((-1.0, y), (y, 1.0)):
            xs, wx = _composite_gauss(_breakpoints(a1, b1, x, 1e-6, s / 4))
            ys, wy = _composite_gauss(_breakpoints(a2, b2, y, 1e-6, s / 4))
            dx, dy = x - xs[:, None], y - ys[None, :]
            g = _G(np.sqrt(dx * dx + dy * dy)) * a * np.exp(
                -((xs[:, None] - cx) ** 2 + (ys[None, :] - cy) ** 2) / (2 * s * s))
            inside += wx @ g @ wy
    whole = cf.gaussian_potential(x, y, cx, cy, s, a)
    assert abs(whole - cf.gaussian_exterior_tail(x, y, cx, cy, s, a) - inside) <= 1e-13 * abs(inside)
