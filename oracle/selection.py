"""Keyframe selection for re-integration (Sec. 4.3) — oracle side, NumPy.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Pose change of keyframe i between its integration pose T_i and its updated
pose T_i': ||s o t_i - s o t_i'|| where t_i stacks the Euler rotation angles
and the translation and s = (2, 2, 2, 1, 1, 1) (Sec. 4.3).  Euler angles are
read as Z-Y-X (yaw, pitch, roll), R = Rz(yaw) Ry(pitch) Rx(roll); angle
differences are wrapped to (-pi, pi].

Modes:
  EQ3          the m most-moved *consecutive* keyframes, Eq. (3); ties go to
               the smallest start j; all keyframes when K < m; processed in
               ascending index order ("successively", Sec. 4.3)
  TOPM         the m most-moved keyframes (the comparison strategy the paper
               attributes to BundleFusion, Sec. 4.3 and Fig. 4), in descending
               distance, ties to the lower index
  ALL_ORDERED  every keyframe whose pose changed, in descending distance
"""
from __future__ import annotations

import math

import numpy as np

EQ3, TOPM, ALL_ORDERED = 0, 1, 2
S = np.array([2.0, 2.0, 2.0, 1.0, 1.0, 1.0])


def euler_zyx(R) -> np.ndarray:
    """(roll, pitch, yaw) with R = Rz(yaw) Ry(pitch) Rx(roll)."""
    R = np.asarray(R, float).reshape(3, 3)
    yaw = math.atan2(R[1, 0], R[0, 0])
    pitch = math.atan2(-R[2, 0], math.hypot(R[0, 0], R[1, 0]))
    roll = math.atan2(R[2, 1], R[2, 2])
    return np.array([roll, pitch, yaw])


def wrap(d: float) -> float:
    """Wrap an angle difference in (-2 pi, 2 pi) to (-pi, pi]."""
    if d > math.pi:
        d -= 2 * math.pi
    elif d <= -math.pi:
        d += 2 * math.pi
    return d


def pose_distance(R0, t0, R1, t1) -> float:
    e0, e1 = euler_zyx(R0), euler_zyx(R1)
    de = np.array([wrap(float(e0[k]) - float(e1[k])) for k in range(3)])
    dt = np.asarray(t0, float) - np.asarray(t1, float)
    v = S * np.concatenate([de, dt])
    acc = 0.0
    for k in range(6):  # sequential sum of squares, in component order
        acc += float(v[k]) * float(v[k])
    return math.sqrt(acc)


def distances(R0, t0, R1, t1) -> np.ndarray:
    return np.array([pose_distance(R0[i], t0[i], R1[i], t1[i]) for i in range(len(R0))])


def window_sums(dist, m):
    """sum_{i=j}^{j+m-1} dist_i for every admissible start j (0-based)."""
    dist = np.asarray(dist, float)
    K = len(dist)
    return np.array([sum(float(x) for x in dist[j:j + m]) for j in range(K - m + 1)])


def select(dist, m, mode) -> list[int]:
    """Keyframe indices (0-based) in processing order."""
    dist = np.asarray(dist, float)
    K = len(dist)
    if mode == EQ3:
        if K <= m:
            return list(range(K))
        sums = window_sums(dist, m)
        j = int(np.argmax(sums))  # first maximum = smallest j
        return list(range(j, j + m))
    order = sorted(range(K), key=lambda i: (-dist[i], i))
    if mode == TOPM:
        return order[:m]
    if mode == ALL_ORDERED:
        return [i for i in order if dist[i] > 0]
    raise ValueError(mode)
