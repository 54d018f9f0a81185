"""The online loop at the benchmark's size (Sec. 4.1 and the final pass of
Sec. 4.3): the corridor, 1000 frames at 640x480 fused five per keyframe into
200 keyframes, each integrated at its drifting estimate, an Eq. 3 update of
m = 20 keyframes every 20 keyframes, then the final pass — the session the
benchmark times.  The oracle fuses its own keyframes from the same frames
and poses, takes every selection itself, and evaluates sampled voxels through
their whole operation sequence one by one: weights and RGBA8 colour exact,
D within 1e-5."""
import numpy as np
import pytest
import torch

import oracle
from oracle import selection as osel
from paper_1709_03763_amd import online, scsurf, synth

pytestmark = pytest.mark.gpu

N_FRAMES, EVERY, M = 1000, 20, 20


def _say(msg):
    print(f"[gpu] {msg}", flush=True)


def test_online_corridor_sampled_voxels_match_oracle():
    assert torch.cuda.is_available(), "GPU tests need a device"
    wl = synth.workload(5)
    groups = synth.keyframe_groups(wl)[: N_FRAMES // wl.kappa]
    first = np.array([g[0] for g in groups])
    Rk, tk = wl.R[first], wl.t[first]
    drift = online.drifting_estimates(Rk, tk, seed=55)
    Re, te = online.corrected(Rk, tk, drift, 1.0)
    poses = []
    for k, g in enumerate(groups):
        A = Re[k] @ Rk[k].T
        poses += [(A @ wl.R[f], A @ (wl.t[f] - tk[k]) + te[k]) for f in g]
    updates = {n: online.corrected(Rk[:n], tk[:n], drift[:n], 0.5 ** (n // EVERY))
               for n in range(EVERY, len(groups) + 1, EVERY)}
    idx = np.concatenate(groups)
    _say(f"rendering {len(idx)} frames at 640x480")
    z, rgb = synth.frames(wl, idx, device="cuda")

    _say("GPU session")
    vol = scsurf.Volume(wl.volume.voxel_size, wl.volume.trunc, 1 << 22, 1 << 21, scsurf.COLOR_RGBA8,
                        max_batch_ops=512)
    sess = online.OnlineSession(vol, wl.intr, wl.kappa, M)
    got_orders = []
    for f in range(len(idx)):
        k = sess.add_frame(torch.from_numpy(z[f]).cuda(), torch.from_numpy(rgb[f]).cuda(), *poses[f])
        if k is not None and (k + 1) in updates:
            got_orders.append(sess.pose_update(*updates[k + 1]))
    got_orders.append(sess.final_pass())
    n_blocks = vol.check_error()
    field = {key: v.cpu().numpy() for key, v in vol.export().items()}
    vol.close()

    _say("oracle: keyframe fusion, selections and the operation sequence")
    kfs, ops, exp_orders = [], [], []
    R_int, t_int = np.zeros((0, 3, 3)), np.zeros((0, 3))
    R_new, t_new = R_int, t_int
    for k, g in enumerate(groups):
        Rf = np.array([poses[f][0] for f in range(k * wl.kappa, (k + 1) * wl.kappa)])
        tf = np.array([poses[f][1] for f in range(k * wl.kappa, (k + 1) * wl.kappa)])
        sl = slice(k * wl.kappa, (k + 1) * wl.kappa)
        kfs.append(oracle.kf_fuse(z[sl], rgb[sl], wl.intr, Rf, tf))
        ops.append((k, +1, Rf[0], tf[0]))
        R_int, t_int = np.concatenate([R_int, Rf[:1]]), np.concatenate([t_int, tf[:1]])
        R_new, t_new = np.concatenate([R_new, Rf[:1]]), np.concatenate([t_new, tf[:1]])
        if (k + 1) in updates:
            R_new, t_new = updates[k + 1]
            sel = osel.select(osel.distances(R_int, t_int, R_new, t_new), M, osel.EQ3)
            exp_orders.append(sel)
            ops += [(j, -1, R_int[j], t_int[j]) for j in sel] + [(j, +1, R_new[j], t_new[j]) for j in sel]
            R_int, t_int = R_int.copy(), t_int.copy()
            R_int[sel], t_int[sel] = R_new[sel], t_new[sel]
    sel = osel.select(osel.distances(R_int, t_int, R_new, t_new), len(kfs), osel.ALL_ORDERED)
    exp_orders.append(sel)
    ops += [(j, -1, R_int[j], t_int[j]) for j in sel] + [(j, +1, R_new[j], t_new[j]) for j in sel]
    assert got_orders == exp_orders
    assert len(exp_orders[-1]) > 0, "the final pass has stale keyframes to correct"
    _say(f"{n_blocks} blocks, {len(ops)} operations, final pass over {len(exp_orders[-1])} keyframes")

    probe = oracle.Volume(wl.volume.voxel_size, wl.volume.trunc)
    rng = np.random.default_rng(21)
    W = field["W"]
    live = np.argwhere(W > 0)
    pick = live[rng.choice(len(live), 1200, replace=False)]
    nb = field["blocks"].shape[0]
    pick = np.concatenate([pick, np.stack([rng.integers(0, nb, 300), rng.integers(0, 512, 300)], 1)])
    dmax = 0.0
    for b, i in pick:
        nvox = 8 * field["blocks"][b].astype(np.int64) + np.array([i & 7, (i >> 3) & 7, i >> 6])
        D, Wv, C, rc = probe.voxel_sequence(kfs, wl.intr, ops, nvox)
        assert rc >= 0
        assert W[b, i] == Wv, (b, i)
        assert np.array_equal(field["C"][b, i, :3].astype(np.float64), C), (b, i)
        dmax = max(dmax, abs(float(field["D"][b, i]) - D))
    _say(f"online corridor sampled voxels: max |D - D_oracle| = {dmax:.2e}")
    assert dmax <= 1e-5
