"""Pins of the oracle's adjoint of integration: the closed form against FP64
central finite differences with frozen decisions (eps = 1e-4 m / 1e-4 rad),
and the frozen forward against the C oracle's running average."""
import numpy as np
import pytest

import oracle
from oracle import adjoint
from paper_1709_03763_amd import synth

S, MU = 0.01, 0.04
EPS = 1e-4


@pytest.fixture(scope="module")
def setup():
    wl = synth.workload(3)
    kfs, Rs, ts = [], [], []
    for k in range(3):
        idx = np.arange(5) + 5 * k * 3
        z, rgb = synth.frames(wl, idx)
        kf = oracle.kf_fuse(z, rgb, wl.intr, wl.R[idx], wl.t[idx])
        kfs.append({"depth": kf["depth"], "weight": kf["weight"],
                    "color": kf["color"][..., :3].astype(np.float32) / 255.0})
        Rs.append(wl.R[idx[0]])
        ts.append(wl.t[idx[0]])
    R, t = np.array(Rs), np.array(ts)
    fz = adjoint.FrozenIntegration(S, MU, kfs, wl.intr, R, t)
    target = np.clip(synth.scene_sdf(wl.scene, fz.xv), -MU, MU)
    cref = np.full((fz.V, 3), 0.5)
    return wl, kfs, R, t, fz, target, cref


def _loss(fz, kfs, R, t, target, cref, depths=None, colors=None):
    depths = depths if depths is not None else [k["depth"] for k in kfs]
    colors = colors if colors is not None else [k["color"] for k in kfs]
    D, C, W = fz.field(depths, colors, R, t)
    return adjoint.sdf_loss(D, C, target, cref, lam=0.1)


def test_frozen_forward_equals_running_average(setup):
    wl, kfs, R, t, fz, target, cref = setup
    v = oracle.Volume(S, MU, color_f32=True)
    for k in range(len(kfs)):
        assert v.integrate(kfs[k], wl.intr, R[k], t[k]) == oracle.OK
    f = v.export()
    k = np.arange(512)
    off = np.stack([k & 7, (k >> 3) & 7, k >> 6], 1)
    n = (8 * f["blocks"][:, None, :] + off[None]).reshape(-1, 3)
    live = f["W"].reshape(-1) > 0
    assert live.sum() == fz.V
    order = np.lexsort((n[live][:, 2], n[live][:, 1], n[live][:, 0]))
    D, C, W = fz.field([x["depth"] for x in kfs], [x["color"] for x in kfs], R, t)
    np.testing.assert_array_equal(n[live][order], fz.vox)
    np.testing.assert_array_equal(f["W"].reshape(-1)[live][order], W)
    assert np.abs(f["D"].reshape(-1)[live][order] - D).max() < 1e-13
    assert np.abs(f["C"].reshape(-1, 3)[live][order] - C).max() < 1e-13


def _pose_fd(fz, kfs, R, t, target, cref, eps):
    fd = np.zeros((len(kfs), 6))
    for k in range(len(kfs)):
        for j in range(6):
            e = np.zeros(6)
            e[j] = eps
            Rp, tp = R.copy(), t.copy()
            Rp[k], tp[k] = adjoint.right_perturb(R[k], t[k], e)
            Lp = _loss(fz, kfs, Rp, tp, target, cref)[0]
            Rp[k], tp[k] = adjoint.right_perturb(R[k], t[k], -e)
            Lm = _loss(fz, kfs, Rp, tp, target, cref)[0]
            fd[k, j] = (Lp - Lm) / (2 * eps)
    return fd


def test_pose_gradient_matches_central_differences(setup):
    """At eps = 1e-4 the central difference carries an O(eps^2) truncation error
    (rotation enters p_z non-linearly), which stays within the 1e-4 relative bar;
    Richardson extrapolation of eps and eps/2 cancels it to O(eps^4)."""
    wl, kfs, R, t, fz, target, cref = setup
    D, C, W = fz.field([x["depth"] for x in kfs], [x["color"] for x in kfs], R, t)
    L0, gD, gC = adjoint.sdf_loss(D, C, target, cref, lam=0.1)
    g = fz.grad(gD, gC, R, t, W)
    fd1 = _pose_fd(fz, kfs, R, t, target, cref, EPS)
    fd2 = _pose_fd(fz, kfs, R, t, target, cref, EPS / 2)
    assert np.linalg.norm(g["xi"] - fd1) / np.linalg.norm(fd1) < 1e-4
    rich = (4 * fd2 - fd1) / 3
    for k in range(len(kfs)):
        assert np.linalg.norm(g["xi"][k] - rich[k]) <= 1e-8 * np.linalg.norm(rich[k]) + 1e-9
    # the projective distance does not see camera-x/y translation or roll about z
    assert np.all(g["xi"][:, [0, 1, 5]] == 0)


def test_depth_and_colour_gradients_match_central_differences(setup):
    """The loss is exactly quadratic in depth and colour, so a central difference
    is exact up to rounding for any step; a 1e-2 step keeps the rounding of the
    ~1e5-term sums far below the tolerance, and the depth and colour terms are
    differenced separately so that one does not swamp the other."""
    h = 1e-2
    wl, kfs, R, t, fz, target, cref = setup
    D, C, W = fz.field([x["depth"] for x in kfs], [x["color"] for x in kfs], R, t)
    _, gD, _ = adjoint.sdf_loss(D, C, target)
    _, _, gC = adjoint.sdf_loss(D, C, D, cref, lam=0.1)
    gz = fz.grad(gD, np.zeros_like(gC), R, t, W)["depth"]
    gc = fz.grad(np.zeros_like(gD), gC, R, t, W)["color"]

    def depth_loss(depths):
        Dd, _, _ = fz.field(depths, [x["color"] for x in kfs], R, t)
        return adjoint.sdf_loss(Dd, C, target)[0]

    def colour_loss(colors):
        _, Cc, _ = fz.field([x["depth"] for x in kfs], colors, R, t)
        return 0.1 * float(np.sum((Cc - cref) ** 2))

    rng = np.random.default_rng(0)
    for k in range(len(kfs)):
        flat = gz[k].reshape(-1)
        for p in rng.choice(np.flatnonzero(flat != 0), 8, replace=False):
            dp = [x["depth"].astype(np.float64).copy() for x in kfs]
            dp[k].reshape(-1)[p] += h
            Lp = depth_loss(dp)
            dp[k].reshape(-1)[p] -= 2 * h
            Lm = depth_loss(dp)
            assert flat[p] == pytest.approx((Lp - Lm) / (2 * h), rel=1e-7, abs=1e-11)
        cflat = gc[k].reshape(-1, 3)
        for p in rng.choice(np.flatnonzero(np.abs(cflat).sum(1) > 0), 4, replace=False):
            for ch in range(3):
                cp = [x["color"].astype(np.float64).copy() for x in kfs]
                cp[k].reshape(-1, 3)[p, ch] += h
                Lp = colour_loss(cp)
                cp[k].reshape(-1, 3)[p, ch] -= 2 * h
                Lm = colour_loss(cp)
                assert cflat[p, ch] == pytest.approx((Lp - Lm) / (2 * h), rel=1e-7, abs=1e-11)


def test_single_keyframe_closed_form(setup):
    """One keyframe into an empty field: D = d, so dL/dZ(u) is the plain sum of
    g_D over the voxels that sample u, and dL/dxi = sum g_D (0,0,1,p_y,-p_x,0)."""
    wl, kfs, R, t, _, _, _ = setup
    fz = adjoint.FrozenIntegration(S, MU, kfs[:1], wl.intr, R[:1], t[:1])
    rng = np.random.default_rng(1)
    gD = rng.standard_normal(fz.V)
    gC = np.zeros((fz.V, 3))
    D, C, W = fz.field([kfs[0]["depth"]], [kfs[0]["color"]], R[:1], t[:1])
    g = fz.grad(gD, gC, R[:1], t[:1], W)
    H, Wd = kfs[0]["depth"].shape
    exp = np.zeros(H * Wd)
    np.add.at(exp, fz.pix[0], gD[fz.vid[0]])
    assert np.abs(g["depth"][0].reshape(-1) - exp).max() < 1e-12
    x = fz.xv[fz.vid[0]]
    p = (x - t[0]) @ R[0]
    gd = gD[fz.vid[0]]
    exp_xi = np.array([0, 0, gd.sum(), (gd * p[:, 1]).sum(), -(gd * p[:, 0]).sum(), 0])
    assert np.abs(g["xi"][0] - exp_xi).max() < 1e-9
