"""Online surface correction session (Sec. 4.1 "System Pipeline" and Sec. 4.3
"Re-integration strategy"): host-side control over the library's calls.

Frames arrive with pose estimates and are collected into the current
keyframe.  Sec. 4.2's strategies decide when a keyframe is complete: after
kappa frames (constant size), when the current frame's motion relative to
the keyframe's first frame exceeds a translation or rotation threshold
(distance), or when the share of the frame's valid pixels visible in the
keyframe's first view falls below a threshold (overlap, counted on the GPU
by `sc_overlap`); a keyframe never exceeds 64 frames.  A complete
keyframe is fused (Eq. 1 and the colour median, `kf_fuse`), packed, and
integrated into the volume at its current pose estimate, which becomes its
integration pose (with integrate_every = k > 1, finished keyframes are held
and integrated k at a time by one batched call, `tsdf_integrate_batch`, and
before every pose-graph update and the final pass: the same volume, bit for
bit, at those points).  A pose-graph update supplies new estimates for every
keyframe so far; the update re-integrates the selected keyframes (by default
the m most-moved consecutive keyframes, Eq. 3) in one batched pass, and
only those take the new pose as their integration pose.  The final pass
re-integrates every keyframe whose integration pose differs from its latest
estimate.  Every step runs in the library's kernels; this module only
decides which call to make.
"""
from __future__ import annotations

import numpy as np
import torch

from . import scsurf


MAX_FRAMES = 64  # frames one keyframe may fuse


class OnlineSession:
    def __init__(self, vol: scsurf.Volume, intr, kappa: int, m: int, mode: int = scsurf.SEL_EQ3, stream=None,
                 strategy: str = "const", max_trans: float = 0.1, max_rot: float = 0.0873,
                 min_overlap: float = 0.8, z_min: float = 0.3, z_max: float = 4.0,
                 stream_radius: float | None = None, integrate_every: int = 1):
        if kappa < 1 or m < 1:
            raise ValueError("kappa and m must be positive")
        if integrate_every < 1:
            raise ValueError("integrate_every must be positive")
        if integrate_every > 1 and stream_radius is not None:
            raise ValueError("held integrations and streaming do not mix: streaming moves the sphere per keyframe")
        if strategy not in ("const", "dist", "overlap"):
            raise ValueError(f"unknown keyframe strategy {strategy!r}")
        self.vol, self.intr, self.kappa, self.m, self.mode, self.stream = vol, intr, kappa, m, mode, stream
        self.strategy, self.max_trans, self.max_rot, self.min_overlap = strategy, max_trans, max_rot, min_overlap
        self.z_min, self.z_max = z_min, z_max
        # streaming sphere (Sec. 3): blocks farther than this from the camera
        # are kept on the host; every operation streams in what it needs
        self.stream_radius = stream_radius
        if stream_radius is not None:
            vol.stream_enable(True)
        self.keyframe_sizes: list[int] = []
        self._depth, self._rgb, self._R, self._t = [], [], [], []
        self.keyframes: list[scsurf.Keyframe] = []
        self.R_int = np.zeros((0, 3, 3))  # integration poses
        self.t_int = np.zeros((0, 3))
        self.R_new = np.zeros((0, 3, 3))  # latest estimates
        self.t_new = np.zeros((0, 3))
        self._kset = None
        self.reintegrated = 0  # keyframe re-integrations performed (de + re counted once)
        self.integrate_every = integrate_every
        self._pending: list[int] = []  # finished keyframes not yet integrated

    @property
    def n_keyframes(self) -> int:
        return len(self.keyframes)

    def _starts_new_keyframe(self, depth, R, t) -> bool:
        if not self._depth:
            return False
        if len(self._depth) >= MAX_FRAMES:
            return True
        if self.strategy == "dist":
            dt, dr = scsurf.relative_motion(self._R[0], self._t[0], R, t)
            return dt > self.max_trans or dr > self.max_rot
        if self.strategy == "overlap":
            valid, visible = scsurf.overlap(depth, self.intr, R, t, self._R[0], self._t[0], self.z_min, self.z_max,
                                            self.stream)
            return valid > 0 and visible < self.min_overlap * valid
        return False

    def add_frame(self, depth: torch.Tensor, rgb: torch.Tensor, R, t):
        """One RGB-D frame (device tensors, depth (H,W) f32, rgb (H,W,3) u8)
        with its pose estimate (camera to world).  Returns the index of the
        keyframe completed and integrated by this frame, or None.  With the
        distance and overlap strategies the frame that starts a new keyframe
        completes the previous one."""
        done = None
        R = np.asarray(R, np.float64)
        t = np.asarray(t, np.float64)
        if self.strategy != "const" and self._starts_new_keyframe(depth, R, t):
            done = self._finish_keyframe()
        self._depth.append(depth)
        self._rgb.append(rgb)
        self._R.append(R)
        self._t.append(t)
        if self.strategy == "const" and len(self._depth) >= min(self.kappa, MAX_FRAMES):
            done = self._finish_keyframe()
        return done

    def flush(self):
        """Completes the current keyframe if it holds frames; returns its index
        or None."""
        return self._finish_keyframe() if self._depth else None

    def _finish_keyframe(self):
        z = torch.stack(self._depth)
        c = torch.stack(self._rgb)
        R, t = np.array(self._R), np.array(self._t)
        kf = scsurf.kf_fuse(z, c, R, t, self.intr, stream=self.stream)
        kf = scsurf.keyframe_pack(kf, stream=self.stream)
        self.keyframe_sizes.append(len(R))
        self._depth, self._rgb, self._R, self._t = [], [], [], []
        if self.stream_radius is not None:
            self.vol.stream_out(t[0], self.stream_radius, stream=self.stream)
        if self.integrate_every == 1:
            self.vol.integrate(kf, self.intr, R[0], t[0], stream=self.stream)
        else:
            self._pending.append(self.n_keyframes)
        self.keyframes.append(kf)
        self._kset = None
        self.R_int = np.concatenate([self.R_int, R[:1]])
        self.t_int = np.concatenate([self.t_int, t[:1]])
        self.R_new = np.concatenate([self.R_new, R[:1]])
        self.t_new = np.concatenate([self.t_new, t[:1]])
        if len(self._pending) >= self.integrate_every:
            self.integrate_pending()
        return self.n_keyframes - 1

    def integrate_pending(self):
        """Integrates the finished keyframes held so far (integrate_every > 1)
        at their integration poses, in order, in one batched call."""
        if self._pending:
            idx = self._pending
            self.vol.integrate_batch([self.keyframes[i] for i in idx], self.intr, self.R_int[idx], self.t_int[idx],
                                     stream=self.stream)
            self._pending = []

    def _keyframe_set(self):
        if self._kset is None or len(self._kset) != self.n_keyframes:
            self._kset = scsurf.KeyframeSet(self.keyframes)
        return self._kset

    def pose_update(self, R, t):
        """New pose estimates for the keyframes so far ((K,3,3), (K,3)).
        Re-integrates the selected keyframes; returns their indices in
        processing order."""
        R = np.asarray(R, np.float64).reshape(-1, 3, 3)
        t = np.asarray(t, np.float64).reshape(-1, 3)
        if len(R) != self.n_keyframes:
            raise ValueError(f"{len(R)} poses for {self.n_keyframes} keyframes")
        self.R_new, self.t_new = R.copy(), t.copy()
        if self.n_keyframes == 0:
            return []
        self.integrate_pending()
        if self.stream_radius is not None:
            # Sec. 4.3: the sphere around the first selected keyframe's
            # integration pose; what the update needs beyond it streams in
            sel, _ = scsurf.select((self.R_int, self.t_int), (self.R_new, self.t_new), self.m, self.mode)
            if sel:
                self.vol.stream_out(self.t_int[sel[0]], self.stream_radius, stream=self.stream)
        order, (Ri, ti) = self.vol.reintegrate_batch(self._keyframe_set(), self.intr, (self.R_int, self.t_int),
                                                      (self.R_new, self.t_new), self.m, self.mode, self.stream)
        self.R_int, self.t_int = Ri, ti
        self.reintegrated += len(order)
        return order

    def final_pass(self):
        """Completes the current keyframe, then re-integrates every keyframe
        whose integration pose differs from its latest estimate, most-moved
        first.  Returns their indices."""
        self.flush()
        self.integrate_pending()
        if self.n_keyframes == 0:
            return []
        order, (Ri, ti) = self.vol.reintegrate_batch(self._keyframe_set(), self.intr, (self.R_int, self.t_int),
                                                      (self.R_new, self.t_new), self.n_keyframes,
                                                      scsurf.SEL_ALL_ORDERED, self.stream)
        self.R_int, self.t_int = Ri, ti
        self.reintegrated += len(order)
        return order


def drifting_estimates(R, t, seed, rho_step=0.002, phi_step_deg=0.1):
    """Synthetic tracking: pose estimates of keyframes whose error grows as a
    seeded random walk in se(3) (rho_step m and phi_step_deg per keyframe),
    applied as T_est = T_true Exp(drift)."""
    rng = np.random.default_rng(seed)
    K = len(R)
    steps = np.concatenate([rng.normal(0, rho_step, (K, 3)), rng.normal(0, np.radians(phi_step_deg), (K, 3))], 1)
    drift = np.cumsum(steps, axis=0)
    return drift


def corrected(R, t, drift, frac):
    """Poses T_true Exp(frac * drift): a pose-graph update that removes
    (1 - frac) of each keyframe's drift."""
    from .synth import compose, se3_exp
    Rn, tn = np.empty_like(R), np.empty_like(t)
    for k in range(len(R)):
        dR, dt = se3_exp(frac * drift[k])
        Rn[k], tn[k] = compose(R[k], t[k], dR, dt)
    return Rn, tn
