"""Pins of the planner-side IG reference (Eq. 3 IDW, orientation factor, c_I); no GPU."""

import math

import numpy as np

from oracle import idw as I
from workloads import look_at


def test_idw_two_samples_closed_form():
    pos = np.array([[0.0, 0, 0], [3.0, 0, 0]])
    g = np.array([2.0, 5.0])
    # query at x=1: distances 1 and 2 -> weights 1 and 1/4 (p = 2)
    assert math.isclose(I.idw_one([1.0, 0, 0], pos, g, 2.0), (2.0 + 5.0 / 4) / 1.25, rel_tol=1e-15)
    # p = 1: weights 1 and 1/2
    assert math.isclose(I.idw_one([1.0, 0, 0], pos, g, 1.0), (2.0 + 2.5) / 1.5, rel_tol=1e-15)
    # midpoint: equal weights for any p
    assert math.isclose(I.idw_one([1.5, 0, 0], pos, g, 3.0), 3.5, rel_tol=1e-15)


def test_idw_coincident_and_constant_field():
    pos = np.array([[0.0, 0, 0], [1.0, 1, 1], [1.0, 1, 1], [2.0, 0, 5]])
    g = np.array([1.0, 4.0, 6.0, 9.0])
    assert I.idw_one([1.0, 1, 1], pos, g) == 5.0          # mean of the two coincident samples
    rng = np.random.default_rng(0)
    P = rng.normal(size=(50, 3))
    for p in (0.5, 2.0, 4.0):
        assert math.isclose(I.idw_one(rng.normal(size=3), P, np.full(50, 7.25), p), 7.25, rel_tol=1e-12)


def test_interpolate_buffer_weights_are_harmonic():
    """N_B identical IDs: G = value * sum_u 1/(N_B - u) = value * H(N_B); newest weighs 1."""
    rng = np.random.default_rng(1)
    pos = rng.normal(size=(20, 3))
    ig = rng.uniform(1, 5, size=20)
    q = rng.normal(size=3)
    one = I.idw_one(q, pos, ig)
    for nb in (1, 3, 10):
        G = I.interpolate(q, np.repeat(pos[None], nb, 0), np.repeat(ig[None], nb, 0))
        assert math.isclose(G, one * sum(1.0 / k for k in range(1, nb + 1)), rel_tol=1e-13)
    # only the newest ID carries information: G equals its IDW
    ids = np.zeros((4, 20)); ids[3] = ig
    assert math.isclose(I.interpolate(q, np.repeat(pos[None], 4, 0), ids), one, rel_tol=1e-13)


def test_orientation_factor_cases():
    poi = np.array([0.0, 0.0, 0.0])
    t45 = math.tan(math.radians(35))
    cam = look_at(np.array([[0.0, -2.0, 0.0]]), poi)[0]
    assert math.isclose(I.orientation_factor(cam, poi, t45, t45), 1.0, rel_tol=1e-6)
    away = look_at(np.array([[0.0, -2.0, 0.0]]), np.array([0.0, -4.0, 0.0]))[0]
    assert I.orientation_factor(away, poi, t45, t45) == 0.0
    # camera looking 30 degrees to the side of the PoI (in the horizontal plane)
    target = np.array([2.0 * math.tan(math.radians(30)), 0.0, 0.0])
    side = look_at(np.array([[0.0, -2.0, 0.0]]), target)[0]
    assert math.isclose(I.orientation_factor(side, poi, t45, t45), math.cos(math.radians(30)), rel_tol=1e-6)
    assert I.orientation_factor(side, poi, math.tan(math.radians(25)), t45) == 0.0


def test_horizon_cost_closed_form():
    poi = np.zeros(3)
    pos = np.array([[0.0, -1.0, 0.0], [0.0, -3.0, 0.0]])
    ids_pos = pos[None]
    ids_ig = np.array([[2.0, 2.0]])
    poses = look_at(np.array([[0.0, -2.0, 0.0], [0.0, -1.5, 0.0]]), poi)
    G, O, c = I.horizon_cost(poses, poi, 1.0, 1.0, ids_pos, ids_ig, w_i=25.0)
    assert np.allclose(G, 2.0) and np.allclose(O, 1.0, rtol=1e-6)
    assert math.isclose(c, 2 * 25.0 / (2.0 + 1e-7), rel_tol=1e-6)
