"""Pins of the oracle's keyframe selection (Sec. 4.3, Eq. 3, Fig. 4)."""
import json
import math
import os

import numpy as np
import pytest

from oracle import selection as sel

GOLD = os.path.join(os.path.dirname(__file__), "golden", "fig4_selection.json")


def _rot(roll, pitch, yaw):
    cr, sr, cp, sp, cy, sy = (math.cos(roll), math.sin(roll), math.cos(pitch), math.sin(pitch),
                              math.cos(yaw), math.sin(yaw))
    Rx = np.array([[1, 0, 0], [0, cr, -sr], [0, sr, cr]])
    Ry = np.array([[cp, 0, sp], [0, 1, 0], [-sp, 0, cp]])
    Rz = np.array([[cy, -sy, 0], [sy, cy, 0], [0, 0, 1]])
    return Rz @ Ry @ Rx


def test_fig4_window_sums_and_eq3():
    g = json.load(open(GOLD))
    d = np.array(g["distance"], float)
    sums = sel.window_sums(d, g["m"])
    assert sums.tolist() == g["window_sums"]
    chosen = sel.select(d, g["m"], sel.EQ3)
    assert [i + 1 for i in chosen] == g["eq3_frames_1based"]
    assert chosen[0] + 1 == g["eq3_start_1based"]
    assert sum(d[chosen]) == g["eq3_window_sum"]


def test_fig4_top_m():
    g = json.load(open(GOLD))
    d = np.array(g["distance"], float)
    chosen = sel.select(d, g["m"], sel.TOPM)
    assert [i + 1 for i in chosen] == g["topm_frames_1based"]


def test_eq3_ties_pick_smallest_start_and_short_lists():
    assert sel.select([1, 1, 1, 1], 2, sel.EQ3) == [0, 1]
    assert sel.select([0, 2, 0, 2, 0], 1, sel.EQ3) == [1]
    assert sel.select([3.0, 1.0], 5, sel.EQ3) == [0, 1]  # K < m: all
    assert sel.select([0.5, 0.0, 0.7, 0.0], 9, sel.ALL_ORDERED) == [2, 0]


def test_euler_roundtrip():
    rng = np.random.default_rng(0)
    for _ in range(200):
        r, p, y = rng.uniform(-3.1, 3.1), rng.uniform(-1.5, 1.5), rng.uniform(-3.1, 3.1)
        e = sel.euler_zyx(_rot(r, p, y))
        assert np.allclose(e, [r, p, y], atol=1e-12)


def test_distance_closed_forms():
    I = np.eye(3)
    # pure translation
    assert sel.pose_distance(I, [0, 0, 0], I, [0.3, -0.4, 0.0]) == pytest.approx(0.5, abs=1e-15)
    # pure yaw by theta: the angle part is scaled by 2
    th = 0.1
    assert sel.pose_distance(I, [0, 0, 0], _rot(0, 0, th), [0, 0, 0]) == pytest.approx(2 * th, abs=1e-14)
    # roll and pitch scale identically
    assert sel.pose_distance(_rot(0.05, 0, 0), [0, 0, 0], _rot(0, -0.02, 0), [0, 0, 0]) == pytest.approx(
        2 * math.hypot(0.05, 0.02), abs=1e-14)
    # combined
    d = sel.pose_distance(I, [1, 2, 3], _rot(0, 0, th), [1, 2, 3.2])
    assert d == pytest.approx(math.sqrt((2 * th) ** 2 + 0.2**2), abs=1e-14)
    # wrap-around: yaw 179 deg vs -179 deg is a 2 deg change
    a, b = math.radians(179.0), math.radians(-179.0)
    assert sel.pose_distance(_rot(0, 0, a), [0, 0, 0], _rot(0, 0, b), [0, 0, 0]) == pytest.approx(
        2 * math.radians(2.0), abs=1e-12)


def test_topm_differs_from_eq3_on_spread_changes():
    d = np.zeros(20)
    d[[2, 9, 17]] = [5, 6, 7]
    d[11:14] = 4
    assert sel.select(d, 3, sel.TOPM) == [17, 9, 2]
    assert sel.select(d, 3, sel.EQ3) == [11, 12, 13]
