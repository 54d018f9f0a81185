"""Pins of the keyframe-strategy oracle (Sec. 4.2): the overlap count and the
relative motion, against closed forms and a per-pixel brute force."""
import math

import numpy as np

from oracle import strategies
from paper_1709_03763_amd import synth

INTR = synth.Intrinsics(64, 48, 52.5, 52.5, 31.5, 23.5)


def _rot(axis, ang):
    w = np.zeros(3)
    w[axis] = ang
    return synth.se3_exp(np.concatenate([np.zeros(3), w]))[0]


def test_identity_sees_every_valid_pixel():
    rng = np.random.default_rng(0)
    z = rng.uniform(0.5, 3.5, (48, 64)).astype(np.float32)
    z[rng.random((48, 64)) < 0.2] = 0.0
    R, t = _rot(1, 0.3), np.array([0.2, -0.1, 1.0])
    valid, visible = strategies.overlap(z, INTR, R, t, R, t)
    assert valid == int((z > 0).sum()) and visible == valid


def test_sideways_shift_of_a_plane():
    # plane at 2 m; the reference camera sits dx to the right: points move
    # fx dx / Z = 10.25 px to the left, so columns u >= 10 stay visible
    Z = 2.0
    dx = 10.25 * Z / INTR.fx
    z = np.full((48, 64), Z, np.float32)
    valid, visible = strategies.overlap(z, INTR, np.eye(3), np.zeros(3), np.eye(3), np.array([dx, 0, 0]))
    assert valid == 64 * 48
    assert visible == (64 - 10) * 48
    # and to the left: columns u <= 53 - ... shift +10.25: u + 10.25 <= 63.5 -> u <= 53
    valid, visible = strategies.overlap(z, INTR, np.eye(3), np.zeros(3), np.eye(3), np.array([-dx, 0, 0]))
    assert visible == 54 * 48


def test_turned_around_sees_nothing():
    z = np.full((48, 64), 1.5, np.float32)
    valid, visible = strategies.overlap(z, INTR, np.eye(3), np.zeros(3), _rot(1, math.pi), np.zeros(3))
    assert valid == 64 * 48 and visible == 0


def test_depth_range_defines_validity():
    z = np.array([[0.0, 0.29, 0.3, 2.0, 4.0, 4.01, np.inf, np.nan]], np.float32)
    intr = synth.Intrinsics(8, 1, 5.0, 5.0, 3.5, 0.0)
    valid, visible = strategies.overlap(z, intr, np.eye(3), np.zeros(3), np.eye(3), np.zeros(3))
    assert valid == 3 and visible == 3


def test_vectorised_count_equals_brute_force():
    rng = np.random.default_rng(4)
    intr = synth.Intrinsics(12, 9, 10.0, 11.0, 5.5, 4.0)
    for trial in range(6):
        z = rng.uniform(0.2, 4.2, (9, 12)).astype(np.float32)
        R, t = synth.se3_exp(rng.normal(0, 0.3, 6))
        Rr, tr = synth.se3_exp(rng.normal(0, 0.3, 6))
        assert strategies.overlap(z, intr, R, t, Rr, tr) == strategies.overlap_brute(z, intr, R, t, Rr, tr)


def test_relative_motion_closed_forms():
    Rk, tk = _rot(2, 0.4), np.array([1.0, 2.0, 0.5])
    for axis, ang in ((0, 0.1), (1, 1.2), (2, 3.0), (0, 1e-9)):
        R = Rk @ _rot(axis, ang)
        t = tk + Rk @ np.array([0.3, 0.0, 0.4])
        dt, dr = strategies.relative_motion(Rk, tk, R, t)
        assert abs(dt - 0.5) < 1e-12
        assert abs(dr - ang) < 1e-9
