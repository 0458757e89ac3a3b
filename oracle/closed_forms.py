"""Closed-form potentials used to pin the oracle (test infrastructure only).

Kernel: G(r) = -(1/2pi) log|r|, the free-space Laplace Green's function of the
introduction (Sec. 1, the convolution approach), with the sign that makes -Lap u = f.

* ``square_potential``: u(x) = int_{[a1,b1]x[a2,b2]} G(x - y) dy for a uniform unit
  density. With F(X,Y) = XY log(X^2+Y^2) - 3XY + X^2 atan(Y/X) + Y^2 atan(X/Y) one has
  d^2F/dXdY = log(X^2+Y^2), so the integral is -(1/4pi) times the signed corner sum
  of F at (x - corner). ``square_gradient`` differentiates that sum term by term.
* ``gaussian_potential``: whole-plane potential of f = A exp(-|y-c|^2/(2 sigma^2)).
  Circle averages of log|x-y| give u(r) = -int_0^inf rho f(rho) log max(r, rho) d rho,
  which integrates to u(r) = -(A sigma^2/2) [log(2 sigma^2) - gamma + Ein(r^2/(2 sigma^2))],
  Ein(t) = E1(t) + log t + gamma (entire; series for small t).
* ``gaussian_exterior_tail``: int over R^2 minus the root box of G(x-y) f(y) dy, by nested
  adaptive quadrature in polar coordinates about x (SciPy QUADPACK).

The Gaussian source follows the synthetic workloads (Gaussian bumps as in the
raindrop and cell-bleb examples, Sec. 5.1 and 5.4); sigma is the standard deviation.
"""
import numpy as np
from scipy import integrate, special

EULER_GAMMA = 0.57721566490153286060651209008240243


def _F(X, Y):
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    r2 = X * X + Y * Y
    with np.errstate(divide="ignore", invalid="ignore"):
        t1 = np.where(r2 > 0, X * Y * np.log(np.where(r2 > 0, r2, 1.0)), 0.0)
        t3 = np.where(X != 0, X * X * np.arctan(Y / np.where(X != 0, X, 1.0)), 0.0)
        t4 = np.where(Y != 0, Y * Y * np.arctan(X / np.where(Y != 0, Y, 1.0)), 0.0)
    return t1 - 3.0 * X * Y + t3 + t4


def square_potential(x, y, a1, b1, a2, b2):
    """int_{[a1,b1]x[a2,b2]} -(1/2pi) log|(x,y) - s| ds  for uniform unit density."""
    X1, X2 = x - b1, x - a1
    Y1, Y2 = y - b2, y - a2
    s = _F(X2, Y2) - _F(X1, Y2) - _F(X2, Y1) + _F(X1, Y1)
    return -s / (4.0 * np.pi)


def _dF(X, Y):
    """(dF/dX, dF/dY) of F above: dF/dX = Y log(X^2+Y^2) - 2Y + 2X atan(Y/X) (symmetric in Y)."""
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    r2 = X * X + Y * Y
    with np.errstate(divide="ignore", invalid="ignore"):
        lg = np.where(r2 > 0, np.log(np.where(r2 > 0, r2, 1.0)), 0.0)
        ax = np.where(X != 0, np.arctan(Y / np.where(X != 0, X, 1.0)), 0.0)
        ay = np.where(Y != 0, np.arctan(X / np.where(Y != 0, Y, 1.0)), 0.0)
    return Y * lg - 2.0 * Y + 2.0 * X * ax, X * lg - 2.0 * X + 2.0 * Y * ay


def square_gradient(x, y, a1, b1, a2, b2):
    """Gradient of ``square_potential`` in (x, y): the same signed corner sum of dF."""
    X1, X2 = x - b1, x - a1
    Y1, Y2 = y - b2, y - a2
    gx = np.zeros(np.broadcast(x, y).shape)
    gy = np.zeros_like(gx)
    for (X, Y, sgn) in ((X2, Y2, 1.0), (X1, Y2, -1.0), (X2, Y1, -1.0), (X1, Y1, 1.0)):
        dx, dy = _dF(X, Y)
        gx = gx + sgn * dx
        gy = gy + sgn * dy
    return -gx / (4.0 * np.pi), -gy / (4.0 * np.pi)


def ein(t):
    """Ein(t) = int_0^t (1 - e^{-s})/s ds = E1(t) + log t + gamma, for t >= 0."""
    t = np.asarray(t, dtype=np.float64)
    out = np.empty_like(t)
    small = t < 0.5
    ts = t[small]
    # alternating series sum_{k>=1} (-1)^{k+1} t^k / (k k!)
    acc = np.zeros_like(ts)
    term = np.ones_like(ts)
    for k in range(1, 40):
        term = term * ts / k
        acc += (-1) ** (k + 1) * term / k
    out[small] = acc
    tl = t[~small]
    out[~small] = special.exp1(tl) + np.log(tl) + EULER_GAMMA
    return out


def gaussian_potential(x, y, cx, cy, sigma, amp):
    """Whole-plane potential of amp*exp(-|s-c|^2/(2 sigma^2)) at (x, y)."""
    r2 = (np.asarray(x) - cx) ** 2 + (np.asarray(y) - cy) ** 2
    t = r2 / (2.0 * sigma * sigma)
    return -(amp * sigma * sigma / 2.0) * (np.log(2.0 * sigma * sigma) - EULER_GAMMA + ein(t))


def gaussian_exterior_tail(x, y, cx, cy, sigma, amp, root=(-1.0, 1.0), epsabs=1e-15, epsrel=1e-13):
    """int_{R^2 \\ [root]^2} G((x,y) - s) amp exp(-|s-c|^2/(2 sigma^2)) ds for (x,y) inside.

    Polar coordinates about the target: for direction theta the ray leaves the box at
    R(theta); the radial integral of r log r g(r) over [R, inf) is done in closed form of the
    Gaussian profile by QUADPACK, the angular one split at the four corner directions.
    """
    lo, hi = root
    corners = [(hi, hi), (lo, hi), (lo, lo), (hi, lo)]
    ang = sorted(np.mod(np.arctan2(cy_ - y, cx_ - x), 2 * np.pi) for cx_, cy_ in corners)
    bx, by = x - cx, y - cy
    q2 = bx * bx + by * by

    def exit_radius(th):
        c, s = np.cos(th), np.sin(th)
        rs = []
        if c > 0:
            rs.append((hi - x) / c)
        elif c < 0:
            rs.append((lo - x) / c)
        if s > 0:
            rs.append((hi - y) / s)
        elif s < 0:
            rs.append((lo - y) / s)
        return min(rs)

    def radial(th):
        c, s = np.cos(th), np.sin(th)
        b = bx * c + by * s  # |x - c + r e|^2 = r^2 + 2 r b + q2
        R = exit_radius(th)
        f = lambda r: r * np.log(r) * np.exp(-(r * r + 2 * r * b + q2) / (2 * sigma * sigma))
        val, _ = integrate.quad(f, R, np.inf, epsabs=epsabs, epsrel=epsrel, limit=200)
        return val

    total = 0.0
    edges = ang + [ang[0] + 2 * np.pi]
    for a0, a1 in zip(edges[:-1], edges[1:]):
        v, _ = integrate.quad(radial, a0, a1, epsabs=epsabs, epsrel=epsrel, limit=200)
        total += v
    return -(amp / (2 * np.pi)) * total
