"""GPU parity of the keyframe strategies of Sec. 4.2.

* `sc_overlap` counts (valid, visible) pixels of a frame against a reference
  view; the counts must equal the oracle's FP64 count exactly, on rendered
  frames at growing distance from the reference, on degenerate poses
  (identity, a half turn), on several depth windows and on ragged
  synthetic images holding zeros, NaN, infinities and out-of-range depths.
* A session on a dense 60-frame scan splits frames into keyframes with the
  distance strategy (5 cm / 5 deg) and with the overlap strategy (85 %),
  integrates each keyframe at its drifting pose estimate, applies pose-graph
  updates every third keyframe and ends with the final pass.  The oracle runs
  the same sequence, taking every split decision with its own arithmetic; the
  keyframe sizes, the re-integration orders and the final field must agree
  (bit-exact block set, weights and RGBA8 colour; D within 1e-5)."""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import selection as osel
from oracle import strategies as ostr
from paper_1709_03763_amd import online, scsurf, synth
from tests.helpers import compare_fields

pytestmark = pytest.mark.gpu

S, MU, M, EVERY, N_FRAMES = 0.01, 0.04, 3, 3, 60


def _say(msg):
    print(f"[gpu] {msg}", flush=True)


@pytest.fixture(scope="module")
def scan():
    assert torch.cuda.is_available(), "GPU tests need a device"
    wl = synth.scan(N_FRAMES)
    z, rgb = synth.frames(wl, np.arange(N_FRAMES), device="cuda")
    drift = online.drifting_estimates(wl.R, wl.t, seed=41, rho_step=0.0005, phi_step_deg=0.03)
    Re, te = online.corrected(wl.R, wl.t, drift, 1.0)  # per-frame tracked estimates
    return wl, z, rgb, drift, Re, te


def test_overlap_counts_match_oracle(scan):
    wl, z, rgb, drift, Re, te = scan
    half = synth.se3_exp(np.array([0, 0, 0, 0, math.pi, 0]))
    cases = [(f, 0) for f in (0, 1, 3, 6, 9, 14, 25, 59)] + [(30, 29), (59, 40)]
    for f, r in cases:
        _say(f"overlap: frame {f} against the view of frame {r}")
        got = scsurf.overlap(torch.from_numpy(z[f]).cuda(), wl.intr, Re[f], te[f], Re[r], te[r])
        assert got == ostr.overlap(z[f], wl.intr, Re[f], te[f], Re[r], te[r]), (f, r)
    d = torch.from_numpy(z[5]).cuda()
    # identity: every valid pixel projects onto itself
    v, vis = scsurf.overlap(d, wl.intr, Re[5], te[5], Re[5], te[5])
    assert vis == v == int(((z[5] >= 0.3) & (z[5] <= 4.0)).sum())
    # a half turn about the camera's own y axis: nothing is in front
    Rh, th = synth.compose(Re[5], te[5], *half)
    assert scsurf.overlap(d, wl.intr, Re[5], te[5], Rh, th) == (v, 0)
    assert ostr.overlap(z[5], wl.intr, Re[5], te[5], Rh, th) == (v, 0)
    # other depth windows
    for lo, hi in ((0.5, 1.5), (2.0, 2.0), (5.0, 9.0)):
        got = scsurf.overlap(d, wl.intr, Re[5], te[5], Re[0], te[0], lo, hi)
        assert got == ostr.overlap(z[5], wl.intr, Re[5], te[5], Re[0], te[0], lo, hi), (lo, hi)


def test_overlap_ragged_image_with_invalid_depths():
    assert torch.cuda.is_available(), "GPU tests need a device"
    rng = np.random.default_rng(77)
    for H, W in ((29, 37), (1, 300), (257, 3)):
        intr = synth.Intrinsics(W, H, 0.8 * max(W, H), 0.8 * max(W, H), (W - 1) / 2 + 0.25, (H - 1) / 2 - 0.25)
        z = rng.uniform(0.1, 5.0, (H, W)).astype(np.float32)
        bad = rng.random((H, W))
        z[bad < 0.05] = 0.0
        z[(bad >= 0.05) & (bad < 0.08)] = np.nan
        z[(bad >= 0.08) & (bad < 0.1)] = np.inf
        z[(bad >= 0.1) & (bad < 0.12)] = -1.0
        sig = 0.1 if min(H, W) > 3 else 0.001  # a thin image needs a nearby reference view
        seen = partial = 0
        for seed in range(4):
            R, t = synth.se3_exp(np.concatenate([rng.normal(0, 0.2, 3), rng.normal(0, 0.1, 3)]))
            dR, dt = synth.se3_exp(np.concatenate([rng.normal(0, 2 * sig, 3), rng.normal(0, sig, 3)]))
            Rr, tr = synth.compose(R, t, dR, dt)
            _say(f"overlap: ragged {H}x{W}, pose pair {seed}")
            got = scsurf.overlap(torch.from_numpy(z).cuda(), intr, R, t, Rr, tr)
            exp = ostr.overlap(z, intr, R, t, Rr, tr)
            assert got == exp, (H, W, seed)
            assert exp[1] <= exp[0]
            seen += exp[1]
            partial += exp[1] < exp[0]
        assert seen > 0 and partial > 0, "the cases mix visible and hidden pixels"


def test_overlap_rejects_bad_arguments():
    assert torch.cuda.is_available(), "GPU tests need a device"
    d = torch.zeros(4, 4, device="cuda")
    bad = synth.Intrinsics(4, 4, 0.0, 10.0, 1.5, 1.5)
    with pytest.raises(scsurf.ScError):
        scsurf.overlap(d, bad, np.eye(3), np.zeros(3), np.eye(3), np.zeros(3))


def _updates_for(first, wl, drift, n):
    """Pose-graph update after n keyframes: the drift of each keyframe's
    first frame shrinks by 2^-(n / EVERY)."""
    f = np.asarray(first[:n])
    return online.corrected(wl.R[f], wl.t[f], drift[f], 0.5 ** (n // EVERY))


def _oracle_run(wl, z, rgb, drift, Re, te, decide):
    """The oracle's own run of the strategy-driven session."""
    ref = oracle.Volume(S, MU)
    groups, cur = [], [0]
    for f in range(1, N_FRAMES):
        if len(cur) >= online.MAX_FRAMES or decide(cur[0], f):
            groups.append(cur)
            cur = [f]
        else:
            cur.append(f)
    groups.append(cur)
    kfs, orders = [], []
    R_int, t_int = np.zeros((0, 3, 3)), np.zeros((0, 3))
    R_new, t_new = R_int, t_int
    first = [g[0] for g in groups]
    for k, g in enumerate(groups):
        kf = oracle.kf_fuse(z[g], rgb[g], wl.intr, Re[g], te[g])
        kfs.append(kf)
        assert ref.integrate(kf, wl.intr, Re[g[0]], te[g[0]]) == oracle.OK
        R_int, t_int = np.concatenate([R_int, Re[g[:1]]]), np.concatenate([t_int, te[g[:1]]])
        R_new, t_new = np.concatenate([R_new, Re[g[:1]]]), np.concatenate([t_new, te[g[:1]]])
        # the last keyframe is completed by the final pass, after every update
        if k + 1 < len(groups) and (k + 1) % EVERY == 0:
            R_new, t_new = _updates_for(first, wl, drift, k + 1)
            sel = osel.select(osel.distances(R_int, t_int, R_new, t_new), M, osel.EQ3)
            orders.append(sel)
            for j in sel:
                assert ref.deintegrate(kfs[j], wl.intr, R_int[j], t_int[j]) == oracle.OK
            for j in sel:
                assert ref.integrate(kfs[j], wl.intr, R_new[j], t_new[j]) == oracle.OK
            R_int, t_int = R_int.copy(), t_int.copy()
            R_int[sel], t_int[sel] = R_new[sel], t_new[sel]
    sel = osel.select(osel.distances(R_int, t_int, R_new, t_new), len(kfs), osel.ALL_ORDERED)
    orders.append(sel)
    for j in sel:
        assert ref.deintegrate(kfs[j], wl.intr, R_int[j], t_int[j]) == oracle.OK
    for j in sel:
        assert ref.integrate(kfs[j], wl.intr, R_new[j], t_new[j]) == oracle.OK
    return [len(g) for g in groups], orders, ref.export()


@pytest.mark.parametrize("strategy", ["dist", "overlap"])
def test_strategy_session_matches_oracle(scan, strategy):
    wl, z, rgb, drift, Re, te = scan
    kw = dict(max_trans=0.05, max_rot=math.radians(5.0)) if strategy == "dist" else dict(min_overlap=0.85)
    _say(f"{strategy} session: {N_FRAMES} frames, update every {EVERY} keyframes, m = {M}")
    vol = scsurf.Volume(S, MU, 1 << 17, 1 << 16)
    sess = online.OnlineSession(vol, wl.intr, 5, M, strategy=strategy, **kw)
    got_orders, first = [], [0]
    for f in range(N_FRAMES):
        k = sess.add_frame(torch.from_numpy(z[f]).cuda(), torch.from_numpy(rgb[f]).cuda(), Re[f], te[f])
        if k is not None:
            first.append(f)  # this frame starts the next keyframe
            if (k + 1) % EVERY == 0:
                got_orders.append(sess.pose_update(*_updates_for(first, wl, drift, k + 1)))
    got_orders.append(sess.final_pass())
    vol.check_error()
    got = vol.export_sorted()

    if strategy == "dist":
        def decide(s, f):
            dt, dr = ostr.relative_motion(Re[s], te[s], Re[f], te[f])
            return dt > kw["max_trans"] or dr > kw["max_rot"]
    else:
        def decide(s, f):
            v, vis = ostr.overlap(z[f], wl.intr, Re[f], te[f], Re[s], te[s])
            return v > 0 and vis < kw["min_overlap"] * v
    sizes, exp_orders, exp = _oracle_run(wl, z, rgb, drift, Re, te, decide)
    assert sess.keyframe_sizes == sizes
    assert len(set(sizes)) > 2, "the strategy yields keyframes of several sizes"
    assert got_orders == exp_orders
    dmax = compare_fields(got, exp)
    _say(f"{strategy} session: keyframe sizes {sizes}, max |D - D_oracle| = {dmax:.2e}")
    vol.close()


def test_overlap_of_an_invalid_frame_is_empty():
    assert torch.cuda.is_available(), "GPU tests need a device"
    intr = synth.QVGA
    z = torch.zeros((intr.height, intr.width), device="cuda")
    assert scsurf.overlap(z, intr, np.eye(3), np.zeros(3), np.eye(3), np.zeros(3)) == (0, 0)
    z = torch.full((intr.height, intr.width), 5.0, device="cuda")  # beyond z_max
    assert scsurf.overlap(z, intr, np.eye(3), np.zeros(3), np.eye(3), np.zeros(3)) == (0, 0)
