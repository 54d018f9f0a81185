"""Host-side pieces of the online session (no GPU): the synthetic drift and
pose-graph correction used by the online loop's tests and benchmark."""
import numpy as np

from paper_1709_03763_amd import online, synth


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
