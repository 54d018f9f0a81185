"""Host-side pieces of the online session (no GPU): the synthetic drift and
pose-graph correction used by the online loop's tests and benchmark."""
import numpy as np

from paper_1709_03763_amd import scsurf, online, synth


def _poses(n, seed=0):
    rng = np.random.default_rng(seed)
    R, t = [], []
    for _ in range(n):
        Ri, ti = synth.se3_exp(np.concatenate([rng.normal(0, 1, 3), rng.normal(0, 0.5, 3)]))
        R.append(Ri)
        t.append(ti)
    return np.array(R), np.array(t)


def test_correction_endpoints():
    R, t = _poses(6)
    drift = online.drifting_estimates(R, t, seed=3)
    R0, t0 = online.corrected(R, t, drift, 0.0)
    np.testing.assert_allclose(R0, R, atol=1e-15)
    np.testing.assert_allclose(t0, t, atol=1e-15)
    R1, t1 = online.corrected(R, t, drift, 1.0)
    for k in range(len(R)):
        dR, dt = synth.se3_exp(drift[k])
        np.testing.assert_allclose(R1[k], R[k] @ dR, atol=1e-14)
        np.testing.assert_allclose(t1[k], R[k] @ dt + t[k], atol=1e-14)


def test_drift_is_a_random_walk():
    R, t = _poses(200)
    drift = online.drifting_estimates(R, t, seed=5, rho_step=0.002, phi_step_deg=0.1)
    steps = np.diff(drift, axis=0)
    assert abs(steps[:, :3].std() - 0.002) < 2e-4
    assert abs(steps[:, 3:].std() - np.radians(0.1)) < 2e-4
    # the error grows along the trajectory
    assert np.linalg.norm(drift[-20:, :3], axis=1).mean() > np.linalg.norm(drift[:20, :3], axis=1).mean()


def test_halving_corrections_shrink_the_pose_change():
    R, t = _poses(8)
    drift = online.drifting_estimates(R, t, seed=7)
    a = online.corrected(R, t, drift, 0.5)
    b = online.corrected(R, t, drift, 0.25)
    da = np.linalg.norm(a[1] - t, axis=1)
    db = np.linalg.norm(b[1] - t, axis=1)
    assert np.all(db <= da + 1e-12)


class _Recorder(online.OnlineSession):
    """A session whose keyframe completion only records the frames it holds,
    so the grouping logic runs without a device."""

    def _finish_keyframe(self):
        self.keyframe_sizes.append(len(self._R))
        self._depth, self._rgb, self._R, self._t = [], [], [], []
        return len(self.keyframe_sizes) - 1


def _feed(sess, R, t):
    done = [sess.add_frame(None, None, R[f], t[f]) for f in range(len(R))]
    sess.flush()
    return done


def test_constant_strategy_groups_kappa_frames_capped_at_64():
    R, t = _poses(23)
    s = _Recorder(None, None, 5, 1)
    done = _feed(s, R, t)
    assert s.keyframe_sizes == [5, 5, 5, 5, 3]
    assert [k for k in done if k is not None] == [0, 1, 2, 3]
    R, t = _poses(150, seed=2)
    s = _Recorder(None, None, 100, 1)
    _feed(s, R, t)
    assert s.keyframe_sizes == [64, 64, 22]


def test_distance_strategy_splits_at_thresholds():
    # a camera moving 1 cm per frame along x, turning 1 deg per frame about z
    n = 40
    R = np.array([synth.se3_exp(np.array([0, 0, 0, 0, 0, np.radians(1.0 * f)]))[0] for f in range(n)])
    t = np.array([[0.01 * f, 0, 0] for f in range(n)])
    s = _Recorder(None, None, 5, 1, strategy="dist", max_trans=0.045, max_rot=np.radians(100.0))
    _feed(s, R, t)
    assert s.keyframe_sizes == [5] * 8  # 5 cm > 4.5 cm starts the next keyframe
    s = _Recorder(None, None, 5, 1, strategy="dist", max_trans=10.0, max_rot=np.radians(2.5))
    _feed(s, R, t)
    assert s.keyframe_sizes[:-1] == [3] * 13 and s.keyframe_sizes[-1] == 1
    # a keyframe never exceeds 64 frames, even when the camera stands still
    R0 = np.repeat(np.eye(3)[None], 130, 0)
    s = _Recorder(None, None, 5, 1, strategy="dist")
    _feed(s, R0, np.zeros((130, 3)))
    assert s.keyframe_sizes == [64, 64, 2]


def test_relative_motion_closed_forms():
    for ang in (0.0, 0.3, 1.0, 2.5, np.pi - 1e-9):
        axis = np.array([1.0, -2.0, 0.5]) / np.linalg.norm([1.0, -2.0, 0.5])
        Ra, ta = synth.se3_exp(np.array([0.1, 0.2, 0.3, 0.4, -0.2, 0.9]))
        dR, dt = synth.se3_exp(np.concatenate([[0, 0, 0], ang * axis]))
        Rb, tb = synth.compose(Ra, ta, dR, np.array([0.3, 0.0, -0.4]))
        d, a = scsurf.relative_motion(Ra, ta, Rb, tb)
        assert abs(d - 0.5) < 1e-12 and abs(a - ang) < 1e-9


def test_unknown_strategy_is_rejected():
    import pytest
    with pytest.raises(ValueError):
        online.OnlineSession(None, None, 5, 1, strategy="dvo")


def test_held_integrations_are_validated():
    import pytest
    with pytest.raises(ValueError):
        online.OnlineSession(None, None, 5, 3, integrate_every=0)
    with pytest.raises(ValueError):
        online.OnlineSession(None, None, 5, 3, integrate_every=4, stream_radius=2.0)


class _CallLog:
    """A volume stand-in that records the session's calls."""

    def __init__(self):
        self.calls = []

    def integrate(self, kf, intr, R, t, stream=None):
        self.calls.append(("integrate", kf))

    def integrate_batch(self, kfs, intr, R, t, stream=None):
        assert len(kfs) == len(R) == len(t)
        self.calls.append(("integrate_batch", list(kfs)))

    def reintegrate_batch(self, kset, intr, T_int, T_new, m, mode, stream=None):
        self.calls.append(("update", len(kset)))
        return [], T_new


def _held_session(monkeypatch, every, n_frames, updates_at, kappa=2):
    """Frames through a session whose fusion and packing are stubbed (the
    keyframe is its index), with pose-graph updates after the given numbers
    of keyframes; returns the recorded volume calls."""
    import torch
    counter = iter(range(1000))
    monkeypatch.setattr(online.scsurf, "kf_fuse", lambda *a, **k: next(counter))
    monkeypatch.setattr(online.scsurf, "keyframe_pack", lambda kf, stream=None: kf)
    monkeypatch.setattr(online.scsurf, "KeyframeSet", lambda kfs: list(kfs))
    vol = _CallLog()
    sess = online.OnlineSession(vol, None, kappa, 2, integrate_every=every)
    z, c = torch.zeros((4, 4)), torch.zeros((4, 4, 3), dtype=torch.uint8)
    for f in range(n_frames):
        k = sess.add_frame(z, c, np.eye(3), np.zeros(3))
        if k is not None and (k + 1) in updates_at:
            sess.pose_update(np.repeat(np.eye(3)[None], k + 1, 0), np.zeros((k + 1, 3)))
    sess.final_pass()
    return vol.calls


def test_held_integrations_flush_in_order(monkeypatch):
    # 11 keyframes of 2 frames (the last one completed by the final pass),
    # held 3 at a time, updates after keyframes 5 and 9
    calls = _held_session(monkeypatch, 3, 21, {5, 9})
    assert calls == [("integrate_batch", [0, 1, 2]), ("integrate_batch", [3, 4]), ("update", 5),
                     ("integrate_batch", [5, 6, 7]), ("integrate_batch", [8]), ("update", 9),
                     ("integrate_batch", [9, 10]), ("update", 11)]


def test_unheld_integrations_are_one_at_a_time(monkeypatch):
    calls = _held_session(monkeypatch, 1, 8, {2})
    assert calls == [("integrate", 0), ("integrate", 1), ("update", 2), ("integrate", 2), ("integrate", 3),
                     ("update", 4)]
