"""Strip solve by multidomain spectral collocation (oracle; test infrastructure only).

Sec. 4.3 solves Lap v = f in the thin strip between the boundary Gamma and the fictitious curve
Gamma~ with v = 0 on both. Element k is bounded by panel k of Gamma, panel k of Gamma~ and the
straight segments joining their endpoints. Its grid is the curvilinear tensor product

    X_ij = (1 + r_i)/2 x~_j + (1 - r_i)/2 x_j,

x_j and x~_j the panels' points at second-kind Chebyshev nodes (obtained from the panels'
Gauss-Legendre nodes by polynomial interpolation), r_i second-kind Chebyshev nodes across the
strip (r = -1 on Gamma, r = +1 on Gamma~). Derivatives: spectral differentiation along each grid
direction, the inverse-map chain rule, D_X = M[xi_x] D_xi + M[eta_x] D_eta (and Y), and the
Laplacian D_X^2 + D_Y^2. Rows: Dirichlet at the nodes on Gamma and Gamma~; the PDE at interior
nodes; on the edges shared with the neighbours, continuity of the value (rows of the left edge)
and of the derivative along the interface normal (rows of the right edge), periodic around the
strip.

Conventions of this implementation (the paper fixes the scheme, not the indexing): ascending
node orders, so j = 0 is a panel's start and j = q - 1 its end, which meets the next panel's
start; element unknowns ordered (i, j) with j fastest; the interface normal is the unit normal
of the segment from Gamma's to Gamma~'s shared endpoint, oriented along increasing j.

Everything is written out plainly (barycentric weights and differentiation matrices from their
definitions, a dense global matrix, numpy.linalg.solve). Before the solve every row is divided by
its 1-norm: this changes no solution of the system, but without it the spread of row norms (1
for boundary rows, up to about 1e7 for Laplacian rows on thin elements) costs the dense LU up to
five digits (4e-9 against a manufactured solution at 56 panels, 24 x 16; 4e-14 with the
scaling). Pinned by tests/test_oracle_strip.py.
"""
import numpy as np


def cheb2(n):
    """Second-kind Chebyshev points on [-1, 1], ascending."""
    return -np.cos(np.pi * np.arange(n) / (n - 1))


def bary_weights(x):
    x = np.asarray(x, dtype=np.float64)
    w = np.ones(x.size)
    for j in range(x.size):
        for k in range(x.size):
            if k != j:
                w[j] /= (x[j] - x[k])
    return w


def diff_matrix(x):
    """D[i, j] = l_j'(x_i) for the Lagrange basis on the points x."""
    x = np.asarray(x, dtype=np.float64)
    w = bary_weights(x)
    n = x.size
    D = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            if i != j:
                D[i, j] = (w[j] / w[i]) / (x[i] - x[j])
        D[i, i] = -np.sum(D[i])
    return D


def interp_matrix(x_from, x_to):
    """E[a, b] = l_b(x_to[a]) for the Lagrange basis on x_from (barycentric second form)."""
    x_from = np.asarray(x_from, dtype=np.float64)
    w = bary_weights(x_from)
    E = np.zeros((len(x_to), x_from.size))
    for a, t in enumerate(x_to):
        d = t - x_from
        hit = np.nonzero(d == 0)[0]
        if hit.size:
            E[a, hit[0]] = 1.0
            continue
        c = w / d
        E[a] = c / c.sum()
    return E


def element_grids(gamma, gamma_t, q, n_r):
    """gamma, gamma_t: (n_panel, n_gl, 2) Gauss-Legendre nodes of the panels of Gamma and
    Gamma~ (same parametrisation direction). Returns X (n_panel, n_r, q, 2)."""
    gamma = np.asarray(gamma, dtype=np.float64)
    gamma_t = np.asarray(gamma_t, dtype=np.float64)
    n_gl = gamma.shape[1]
    s_gl, _ = np.polynomial.legendre.leggauss(n_gl)
    E = interp_matrix(s_gl, cheb2(q))
    r = cheb2(n_r)
    X = np.empty((gamma.shape[0], n_r, q, 2))
    for k in range(gamma.shape[0]):
        xc = E @ gamma[k]
        xt = E @ gamma_t[k]
        for i in range(n_r):
            X[k, i] = 0.5 * (1 + r[i]) * xt + 0.5 * (1 - r[i]) * xc
    return X


def element_operators(Xk):
    """(DX, DY) of one element grid Xk (n_r, q, 2), each (B, B) with B = n_r q, (i, j) j fastest."""
    n_r, q, _ = Xk.shape
    Dq = diff_matrix(cheb2(q))
    Dr = diff_matrix(cheb2(n_r))
    Dxi = np.kron(np.eye(n_r), Dq)    # along j
    Deta = np.kron(Dr, np.eye(q))     # along i
    x = Xk[:, :, 0].reshape(-1)
    y = Xk[:, :, 1].reshape(-1)
    x_xi, y_xi = Dxi @ x, Dxi @ y
    x_eta, y_eta = Deta @ x, Deta @ y
    J = x_xi * y_eta - x_eta * y_xi
    xi_x, xi_y = y_eta / J, -x_eta / J
    eta_x, eta_y = -y_xi / J, x_xi / J
    DX = xi_x[:, None] * Dxi + eta_x[:, None] * Deta
    DY = xi_y[:, None] * Dxi + eta_y[:, None] * Deta
    return DX, DY, (x_xi, y_xi)


def assemble(X):
    """Global matrix A (dense, N = n_panel * n_r * q) and the mask of PDE rows."""
    n, n_r, q, _ = X.shape
    B = n_r * q
    A = np.zeros((n * B, n * B))
    pde = np.zeros(n * B, dtype=bool)
    ops = [element_operators(X[k]) for k in range(n)]
    for k in range(n):
        DX, DY, (x_xi, y_xi) = ops[k]
        L = DX @ DX + DY @ DY
        kp, km = (k + 1) % n, (k - 1) % n
        for i in range(n_r):
            for j in range(q):
                row = k * B + i * q + j
                loc = i * q + j
                if i == 0 or i == n_r - 1:
                    A[row, row] = 1.0
                elif j == 0:  # value continuity with the previous element's last column
                    A[row, row] = 1.0
                    A[row, km * B + i * q + (q - 1)] -= 1.0
                elif j == q - 1:  # normal-derivative continuity with the next element's first column
                    P, Pt = X[k, 0, q - 1], X[k, n_r - 1, q - 1]
                    t = (Pt - P) / np.linalg.norm(Pt - P)
                    nv = np.array([t[1], -t[0]])
                    if nv[0] * x_xi[loc] + nv[1] * y_xi[loc] < 0:
                        nv = -nv
                    DXn, DYn, _ = ops[kp]
                    A[row, k * B:(k + 1) * B] += nv[0] * DX[loc] + nv[1] * DY[loc]
                    A[row, kp * B:(kp + 1) * B] -= nv[0] * DXn[i * q] + nv[1] * DYn[i * q]
                else:
                    A[row, k * B:(k + 1) * B] = L[loc]
                    pde[row] = True
    return A, pde


def solve(gamma, gamma_t, f, q=16, n_r=16):
    """v at every element node (n_panel, n_r, q) for Lap v = f, v = 0 on Gamma and Gamma~.
    f maps an (m, 2) array of points to m values."""
    X = element_grids(gamma, gamma_t, q, n_r)
    A, pde = assemble(X)
    b = np.where(pde, f(X.reshape(-1, 2)), 0.0)
    s = 1.0 / np.abs(A).sum(axis=1)  # row equilibration
    return np.linalg.solve(A * s[:, None], b * s).reshape(X.shape[:3]), X
