"""Layer potentials of the glue step, by direct summation (oracle; test infrastructure only).

Sec. 4.4 repairs the jumps of the piecewise particular solution across the fictitious
interface with the harmonic function v_glue = S[sigma] - D[tau], where on that curve

    S[sigma](x) = int Phi(x, y) sigma(y) ds_y,    D[tau](x) = int dPhi(x, y)/dn_y tau(y) ds_y,

Phi(x, y) = (1/2pi) log(1/|x - y|) the free-space fundamental solution of -Lap (the same
kernel as the volume potential), n_y the unit normal at y. The solution is then evaluated at
every quadtree node with an FMM (end of Sec. 4.4, and the evaluation timing of Sec. 5).

With the curve discretised by quadrature nodes y_j, weights w_j (arc length included) and
unit normals n_j, the discrete layer potential at a point x is the plain sum

    V(x) = sum_j w_j [ sigma_j Phi(x, y_j) - tau_j dPhi(x, y_j)/dn_y ]
         = -(1/2pi) sum_j w_j [ sigma_j log|x - y_j| + tau_j n_j . (x - y_j) / |x - y_j|^2 ],

since dPhi/dn_y = (1/2pi) n_y . (x - y) / |x - y|^2. ``layer_potential`` evaluates exactly
that, in FP64, target by target (chunked). It is the plain definition of what the FMM
approximates, pinned by tests/test_oracle_layer.py against closed forms on a circle, Green's
representation formula on a panel-discretised star, and a finite-difference check of the
dipole orientation.
"""
import numpy as np

INV_2PI = 1.0 / (2.0 * np.pi)


def layer_potential(targets, nodes, weights, normals, sigma, tau, chunk=4096):
    """V at each target: sum over nodes of w [sigma Phi - tau dPhi/dn_y] (see module doc).

    targets (n, 2), nodes (m, 2), weights (m,), normals (m, 2) unit, sigma and tau (m,).
    A target that coincides with a node gives a non-finite value (the sum is undefined there).
    """
    targets = np.asarray(targets, dtype=np.float64).reshape(-1, 2)
    nodes = np.asarray(nodes, dtype=np.float64).reshape(-1, 2)
    q = np.asarray(weights, dtype=np.float64) * np.asarray(sigma, dtype=np.float64)
    d = np.asarray(weights, dtype=np.float64) * np.asarray(tau, dtype=np.float64)
    nx, ny = np.asarray(normals, dtype=np.float64).reshape(-1, 2).T
    out = np.empty(targets.shape[0])
    for a in range(0, targets.shape[0], chunk):
        t = targets[a:a + chunk]
        dx = t[:, 0:1] - nodes[None, :, 0]
        dy = t[:, 1:2] - nodes[None, :, 1]
        r2 = dx * dx + dy * dy
        s_part = 0.5 * np.log(r2) @ q
        d_part = ((dx * nx[None, :] + dy * ny[None, :]) / r2) @ d
        out[a:a + chunk] = -INV_2PI * (s_part + d_part)
    return out


def leaf_targets(centres, levels, p=16):
    """All leaf nodes of a tree in the volume code's layout: (n_leaves * p * p, 2), leaves in
    the given order, then y index, then x index (first-kind Chebyshev points, ascending)."""
    i = np.arange(1, p + 1)
    t = -np.cos((2 * i - 1) * np.pi / (2 * p))
    X, Y = np.meshgrid(t, t, indexing="xy")
    s = 2.0 ** (-np.asarray(levels, dtype=np.float64))
    c = np.asarray(centres, dtype=np.float64)
    x = c[:, 0:1] + s[:, None] * X.reshape(1, -1)
    y = c[:, 1:2] + s[:, None] * Y.reshape(1, -1)
    return np.stack([x.reshape(-1), y.reshape(-1)], axis=1)
