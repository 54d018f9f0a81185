"""GPU parity of the online loop (Sec. 4.1 and the final pass of Sec. 4.3):
frames fused into keyframes of kappa frames, each keyframe integrated at its
drifting pose estimate, periodic pose-graph updates re-integrating the Eq. 3
window of m keyframes, and a final pass over the keyframes still integrated
at a stale pose.  The oracle runs the same sequence with its own fusion,
selection and volume; the final fields must agree (bit-exact block set,
weights and RGBA8 colour; D within 1e-5)."""
import numpy as np
import pytest
import torch

import oracle
from oracle import selection as osel
from paper_1709_03763_amd import online, scsurf, synth
from tests.helpers import compare_fields

pytestmark = pytest.mark.gpu

S, MU, KAPPA, M, EVERY = 0.01, 0.04, 5, 3, 4


def _say(msg):
    print(f"[gpu] {msg}", flush=True)


def _scenario():
    wl = synth.workload(3)
    groups = synth.keyframe_groups(wl)
    first = np.array([g[0] for g in groups])
    Rk, tk = wl.R[first], wl.t[first]
    drift = online.drifting_estimates(Rk, tk, seed=31)
    Re, te = online.corrected(Rk, tk, drift, 1.0)  # the tracked estimates
    frame_poses = []
    for k, g in enumerate(groups):
        # frames keep their true poses relative to the keyframe's first frame
        A = Re[k] @ Rk[k].T
        for f in g:
            frame_poses.append((A @ wl.R[f], A @ (wl.t[f] - tk[k]) + te[k]))
    updates = {}
    for n in range(EVERY, len(groups) + 1, EVERY):
        u = n // EVERY
        updates[n] = online.corrected(Rk[:n], tk[:n], drift[:n], 0.5 ** u)
    return wl, groups, frame_poses, updates


@pytest.mark.parametrize("integrate_every", [1, 3])
def test_online_session_matches_oracle(integrate_every):
    """integrate_every 3: keyframes integrated three at a time by the batched
    integration, and before each update (held groups of 1 to 3)."""
    assert torch.cuda.is_available(), "GPU tests need a device"
    wl, groups, frame_poses, updates = _scenario()
    z, rgb = synth.frames(wl, np.arange(wl.n_frames), device="cuda")
    _say(f"online session: {len(groups)} keyframes of {KAPPA} frames, update every {EVERY}, m = {M}, "
         f"integrations held {integrate_every}")
    vol = scsurf.Volume(S, MU, 1 << 17, 1 << 16)
    sess = online.OnlineSession(vol, wl.intr, KAPPA, M, integrate_every=integrate_every)
    got_orders = []
    for f in range(wl.n_frames):
        R, t = frame_poses[f]
        k = sess.add_frame(torch.from_numpy(z[f]).cuda(), torch.from_numpy(rgb[f]).cuda(), R, t)
        if k is not None and (k + 1) in updates:
            got_orders.append(sess.pose_update(*updates[k + 1]))
    got_orders.append(sess.final_pass())
    vol.check_error()
    got = vol.export_sorted()

    # the oracle runs the same sequence
    ref = oracle.Volume(S, MU)
    kfs = []
    R_int, t_int = np.zeros((0, 3, 3)), np.zeros((0, 3))
    R_new, t_new = R_int, t_int
    exp_orders = []
    for k, g in enumerate(groups):
        Rf = np.array([frame_poses[f][0] for f in g])
        tf = np.array([frame_poses[f][1] for f in g])
        kf = oracle.kf_fuse(z[g], rgb[g], wl.intr, Rf, tf)
        kfs.append(kf)
        assert ref.integrate(kf, wl.intr, Rf[0], tf[0]) == oracle.OK
        R_int, t_int = np.concatenate([R_int, Rf[:1]]), np.concatenate([t_int, tf[:1]])
        R_new, t_new = np.concatenate([R_new, Rf[:1]]), np.concatenate([t_new, tf[:1]])
        if (k + 1) in updates:
            R_new, t_new = updates[k + 1]
            sel = osel.select(osel.distances(R_int, t_int, R_new, t_new), M, osel.EQ3)
            exp_orders.append(sel)
            for j in sel:
                assert ref.deintegrate(kfs[j], wl.intr, R_int[j], t_int[j]) == oracle.OK
            for j in sel:
                assert ref.integrate(kfs[j], wl.intr, R_new[j], t_new[j]) == oracle.OK
            R_int, t_int = R_int.copy(), t_int.copy()
            R_int[sel], t_int[sel] = R_new[sel], t_new[sel]
    sel = osel.select(osel.distances(R_int, t_int, R_new, t_new), len(kfs), osel.ALL_ORDERED)
    exp_orders.append(sel)
    for j in sel:
        assert ref.deintegrate(kfs[j], wl.intr, R_int[j], t_int[j]) == oracle.OK
    for j in sel:
        assert ref.integrate(kfs[j], wl.intr, R_new[j], t_new[j]) == oracle.OK

    assert got_orders == exp_orders
    assert len(exp_orders[-1]) > 0, "the final pass has stale keyframes to correct"
    dmax = compare_fields(got, ref.export())
    _say(f"online session: orders {got_orders}, max |D - D_oracle| = {dmax:.2e}")
    vol.close()

