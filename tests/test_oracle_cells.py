"""Pins of the cell-side oracle (incident volume fraction, modified incident
pressure, relaxation weight and blending) against closed forms and
properties that hold by construction of the formulas in the paper."""
import numpy as np

from oracle import cells


def test_alpha_limits_and_linearity():
    zc = np.array([0.0, 0.0, 0.0, 0.0, 0.0, -5.0, 5.0])
    dz = np.full(7, 0.2)
    eta = np.array([-0.1, 0.1, 0.0, 0.05, -0.2, 0.0, 0.0])
    a = cells.incident_alpha(eta, zc, dz)
    # interface at the bottom face, top face, centre, three quarters up;
    # a cell entirely above the surface, one deep below, one high above
    assert np.allclose(a, [0.0, 1.0, 0.5, 0.75, 0.0, 1.0, 0.0], atol=1e-15)


def test_alpha_is_the_submerged_height_fraction():
    rng = np.random.default_rng(0)
    zc = rng.uniform(-1, 1, 500)
    dz = rng.uniform(0.01, 0.3, 500)
    eta = rng.uniform(-1, 1, 500)
    a = cells.incident_alpha(eta, zc, dz)
    # brute force: the share of 20001 equally spaced sample heights below eta
    s = (np.arange(20001) + 0.5) / 20001
    z = (zc - dz / 2)[:, None] + dz[:, None] * s[None, :]
    assert np.abs(a - np.mean(z < eta[:, None], axis=1)).max() < 1e-4


def test_pstar_in_water_air_and_mixture():
    p = np.array([2.0, 2.0, 2.0])
    a = np.array([1.0, 0.0, 0.25])
    ps = cells.pstar(p, a, 1000.0, 1.2)
    assert np.allclose(ps, [2.0, 2.0 * 1.2 / 1000.0, 2.0 * (250.0 + 0.75 * 1.2) / 1000.0], rtol=1e-15)


def test_relax_weight_closed_form_and_smoothness():
    x = np.array([-0.5, 0.0, 0.25, 0.5, 1.0, 1.5])
    w = cells.relax_weight(x)
    assert np.allclose(w, [0.0, 0.0, 0.15625, 0.5, 1.0, 1.0], atol=1e-15)
    # zero slope at both ends of the zone, symmetric about x = 1/2
    h = 1e-6
    assert abs(cells.relax_weight(np.array([h]))[0]) < 1e-11
    assert abs(1.0 - cells.relax_weight(np.array([1.0 - h]))[0]) < 1e-11
    t = np.linspace(0, 1, 101)
    assert np.allclose(cells.relax_weight(t) + cells.relax_weight(1.0 - t), 1.0, atol=1e-15)


def test_relax_blends_towards_the_incident_field():
    x = np.array([0.0, 1.0, 0.5])
    ai = np.array([0.3, 0.3, 0.3])
    ac = np.array([0.9, 0.9, 0.9])
    uc = np.array([[1.0, 1.0, 1.0], [2.0, 2.0, 2.0], [-1.0, -1.0, -1.0]])
    a, u = cells.relax(x, ai, ac, uc)
    assert np.allclose(a, [0.9, 0.3, 0.6], atol=1e-15)
    assert np.allclose(u, [[1.0, 0.0, 0.5], [2.0, 0.0, 1.0], [-1.0, 0.0, -0.5]], atol=1e-15)
