"""Keyframe strategies of Sec. 4.2 — test infrastructure (the oracle).

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline may use
this module; the product path never does.

* Distance strategy: a new keyframe starts when the relative pose between
  the current frame and the keyframe's first frame exceeds a translational
  or rotational threshold.  `relative_motion` gives (translation norm,
  rotation angle) of T_kf^-1 T_frame.
* Overlap strategy: a new keyframe starts when the share of the frame's
  pixels that are visible in the keyframe's view drops below a threshold.
  `overlap` counts (valid, visible) pixels in FP64 in the written order the
  GPU kernel also follows: camera point (((u - cx) / fx) Z, ((v - cy) / fy) Z,
  Z); world point R p + t row by row; reference point R_ref^T (w - t_ref)
  column by column; visible if its depth is positive and its nearest pixel
  floor(((fx x) / z + cx) + 1/2) (likewise y) lies inside the image.
"""
from __future__ import annotations

import math

import numpy as np


def _f32(x):
    return np.float64(np.float32(x))


def overlap(depth, intr, R, t, R_ref, t_ref, z_min=0.3, z_max=4.0):
    """(valid, visible) pixel counts of `depth` (H, W) seen from pose (R, t)
    against the reference view (R_ref, t_ref).  Intrinsics are taken in FP32
    (as the C ABI stores them) and widened to FP64."""
    z32 = np.asarray(depth, np.float32)
    H, W = z32.shape
    fx, fy, cx, cy = _f32(intr.fx), _f32(intr.fy), _f32(intr.cx), _f32(intr.cy)
    R = np.asarray(R, np.float64).reshape(3, 3)
    t = np.asarray(t, np.float64).reshape(3)
    Rr = np.asarray(R_ref, np.float64).reshape(3, 3)
    tr = np.asarray(t_ref, np.float64).reshape(3)
    valid = (z32 >= np.float32(z_min)) & (z32 <= np.float32(z_max))
    v, u = np.nonzero(valid)
    z = z32[v, u].astype(np.float64)
    u = u.astype(np.float64)
    v = v.astype(np.float64)
    p0 = ((u - cx) / fx) * z
    p1 = ((v - cy) / fy) * z
    p2 = z
    w = [((R[r, 0] * p0 + R[r, 1] * p1) + R[r, 2] * p2) + t[r] for r in range(3)]
    d = [w[r] - tr[r] for r in range(3)]
    q = [(Rr[0, c] * d[0] + Rr[1, c] * d[1]) + Rr[2, c] * d[2] for c in range(3)]
    front = q[2] > 0.0
    with np.errstate(divide="ignore", invalid="ignore"):
        fu = np.floor(((fx * q[0]) / q[2] + cx) + 0.5)
        fv = np.floor(((fy * q[1]) / q[2] + cy) + 0.5)
    inside = front & (fu >= 0.0) & (fu <= W - 1) & (fv >= 0.0) & (fv <= H - 1)
    return int(valid.sum()), int(inside.sum())


def overlap_brute(depth, intr, R, t, R_ref, t_ref, z_min=0.3, z_max=4.0):
    """The same count, one pixel at a time in plain Python (small images)."""
    z32 = np.asarray(depth, np.float32)
    H, W = z32.shape
    fx, fy, cx, cy = (float(_f32(a)) for a in (intr.fx, intr.fy, intr.cx, intr.cy))
    R = np.asarray(R, np.float64).reshape(3, 3)
    Rr = np.asarray(R_ref, np.float64).reshape(3, 3)
    valid = visible = 0
    for v in range(H):
        for u in range(W):
            zf = z32[v, u]
            if not (zf >= np.float32(z_min) and zf <= np.float32(z_max)):
                continue
            valid += 1
            z = float(zf)
            p = (((u - cx) / fx) * z, ((v - cy) / fy) * z, z)
            w = [((R[r, 0] * p[0] + R[r, 1] * p[1]) + R[r, 2] * p[2]) + t[r] for r in range(3)]
            d = [w[r] - t_ref[r] for r in range(3)]
            q = [(Rr[0, c] * d[0] + Rr[1, c] * d[1]) + Rr[2, c] * d[2] for c in range(3)]
            if not q[2] > 0.0:
                continue
            pu = math.floor(((fx * q[0]) / q[2] + cx) + 0.5)
            pv = math.floor(((fy * q[1]) / q[2] + cy) + 0.5)
            if 0 <= pu <= W - 1 and 0 <= pv <= H - 1:
                visible += 1
    return valid, visible


def relative_motion(R_kf, t_kf, R, t):
    """(translation norm, rotation angle in radians) of T_kf^-1 T."""
    R_kf = np.asarray(R_kf, np.float64).reshape(3, 3)
    R = np.asarray(R, np.float64).reshape(3, 3)
    Rrel = R_kf.T @ R
    trel = R_kf.T @ (np.asarray(t, np.float64) - np.asarray(t_kf, np.float64))
    # angle = atan2(sin, cos): R - R^T = 2 sin(theta) [axis]x, trace = 1 + 2 cos(theta)
    sin_t = math.sqrt((Rrel[2, 1] - Rrel[1, 2]) ** 2 + (Rrel[0, 2] - Rrel[2, 0]) ** 2 +
                      (Rrel[1, 0] - Rrel[0, 1]) ** 2) / 2.0
    cos_t = (Rrel[0, 0] + Rrel[1, 1] + Rrel[2, 2] - 1.0) / 2.0
    return float(np.linalg.norm(trel)), math.atan2(sin_t, cos_t)
