"""Pins of the layer-potential oracle (direct sum of S[sigma] - D[tau], Sec. 4.4).

* Circle of radius R, trapezoid rule: the single layer of a unit density is -R log R inside
  and -R log|x| outside (mean-value property of log), the double layer of a unit density is
  -1 inside and 0 outside (Gauss's theorem for the dipole kernel with outward normals).
* Green's representation formula on the panel-discretised star curve: for a function h
  harmonic inside, S[dh/dn] - D[h] equals h inside and 0 outside.
* The dipole term equals a centred finite difference of two opposite charges along the normal
  (orientation and sign of the normal derivative).
* The leaf-target layout matches the node convention of the volume code.
"""
import numpy as np
import pytest

from oracle import layer, nodes
from workloads import gen


def _circle(R, m):
    th = 2 * np.pi * np.arange(m) / m
    y = np.stack([R * np.cos(th), R * np.sin(th)], axis=1)
    nrm = np.stack([np.cos(th), np.sin(th)], axis=1)
    w = np.full(m, 2 * np.pi * R / m)
    return y, w, nrm


def test_circle_single_and_double_layer_closed_forms():
    R = 0.6
    y, w, nrm = _circle(R, 400)
    rng = np.random.default_rng(3)
    inside = rng.uniform(-0.3, 0.3, (50, 2))
    ang = rng.uniform(0, 2 * np.pi, 50)
    rad = rng.uniform(0.95, 2.0, 50)
    outside = np.stack([rad * np.cos(ang), rad * np.sin(ang)], axis=1)
    one, zero = np.ones(len(w)), np.zeros(len(w))
    s_in = layer.layer_potential(inside, y, w, nrm, one, zero)
    s_out = layer.layer_potential(outside, y, w, nrm, one, zero)
    assert np.max(np.abs(s_in - (-R * np.log(R)))) < 1e-13
    assert np.max(np.abs(s_out - (-R * np.log(np.hypot(outside[:, 0], outside[:, 1]))))) < 1e-13
    # V = S - D, so a unit tau gives -D: +1 inside, 0 outside
    d_in = layer.layer_potential(inside, y, w, nrm, zero, one)
    d_out = layer.layer_potential(outside, y, w, nrm, zero, one)
    assert np.max(np.abs(d_in - 1.0)) < 1e-13
    assert np.max(np.abs(d_out)) < 1e-13


def _harmonic(x, y):
    h = x ** 3 - 3 * x * y * y + 0.3 * x - 0.2 * y + 1.0
    hx = 3 * x * x - 3 * y * y + 0.3
    hy = -6 * x * y - 0.2
    return h, hx, hy


def test_green_representation_on_star_panels():
    c = gen.star_curve(n_panels=128, order=24)
    h, hx, hy = _harmonic(c.nodes[:, 0], c.nodes[:, 1])
    dhdn = hx * c.normals[:, 0] + hy * c.normals[:, 1]
    rng = np.random.default_rng(5)
    # inside: well within the star (r < 0.9 * min radius); outside: beyond the box [-1,1]^2 edge region
    ang = rng.uniform(0, 2 * np.pi, 80)
    rin = rng.uniform(0, 0.9 * 0.95 * 0.7 * 0.7, 80)
    tin = np.stack([rin * np.cos(ang), rin * np.sin(ang)], axis=1)
    rout = rng.uniform(1.0, 1.4, 80)
    tout = np.stack([rout * np.cos(ang), rout * np.sin(ang)], axis=1)
    vin = layer.layer_potential(tin, c.nodes, c.weights, c.normals, dhdn, h)
    vout = layer.layer_potential(tout, c.nodes, c.weights, c.normals, dhdn, h)
    hin = _harmonic(tin[:, 0], tin[:, 1])[0]
    assert np.max(np.abs(vin - hin)) < 1e-12 * np.max(np.abs(hin))
    assert np.max(np.abs(vout)) < 1e-12 * np.max(np.abs(hin))


def test_dipole_is_the_normal_difference_of_two_charges():
    c = gen.star_curve(n_panels=16, order=8, seed=2)
    j = 37
    y, w, nrm = c.nodes[j:j + 1], c.weights[j:j + 1], c.normals[j:j + 1]
    eps = 1e-4
    rng = np.random.default_rng(9)
    t = rng.uniform(-1, 1, (40, 2))
    t = t[np.hypot(t[:, 0] - y[0, 0], t[:, 1] - y[0, 1]) > 0.2]
    dip = layer.layer_potential(t, y, w, nrm, [0.0], [1.0])
    plus = layer.layer_potential(t, y + 0.5 * eps * nrm, w, nrm, [1.0 / eps], [0.0])
    minus = layer.layer_potential(t, y - 0.5 * eps * nrm, w, nrm, [1.0 / eps], [0.0])
    # S(y + eps n/2) - S(y - eps n/2) ~ eps dPhi/dn_y, and V = -D for the dipole part
    assert np.max(np.abs(dip + (plus - minus))) < 1e-7 * np.max(np.abs(dip))


def test_leaf_target_layout():
    centres = np.array([[0.25, -0.75], [-0.5, 0.5]])
    levels = np.array([2, 1])
    t = layer.leaf_targets(centres, levels)
    ref = np.concatenate([nodes.leaf_nodes(centres[0], 0.25), nodes.leaf_nodes(centres[1], 0.5)])
    assert np.array_equal(t, ref)


def test_empty_and_coincident():
    c = gen.star_curve(n_panels=4, order=4)
    out = layer.layer_potential(np.zeros((0, 2)), c.nodes, c.weights, c.normals, c.sigma, c.tau)
    assert out.shape == (0,)
    z = layer.layer_potential(np.array([[0.1, 0.2]]), np.zeros((0, 2)), [], np.zeros((0, 2)), [], [])
    assert z.shape == (1,) and z[0] == 0.0
    with np.errstate(divide="ignore", invalid="ignore"):
        v = layer.layer_potential(c.nodes[:1], c.nodes, c.weights, c.normals, c.sigma, c.tau)
    assert not np.isfinite(v[0])
