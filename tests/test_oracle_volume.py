"""Pins of the oracle's voxel-hashed TSDF: integration (Sec. 3, SDF volume)
and de-integration (Sec. 4.3, Eq. 2), against closed forms, brute force,
exact reversibility and order independence."""
import math

import numpy as np
import pytest

import oracle
from paper_1709_03763_amd import synth

S, MU = 0.01, 0.04
INTR = synth.QVGA


def _rot(roll, pitch, yaw):
    cr, sr, cp, sp, cy, sy = (math.cos(roll), math.sin(roll), math.cos(pitch), math.sin(pitch),
                              math.cos(yaw), math.sin(yaw))
    Rx = np.array([[1, 0, 0], [0, cr, -sr], [0, sr, cr]])
    Ry = np.array([[cp, 0, sp], [0, 1, 0], [-sp, 0, cp]])
    Rz = np.array([[cy, -sy, 0], [sy, cy, 0], [0, 0, 1]])
    return Rz @ Ry @ Rx


def _const_kf(z, w=1.0, rgb=(10, 20, 30), f32=False, shape=(INTR.height, INTR.width)):
    H, W = shape
    kf = {"depth": np.full((H, W), z, np.float32), "weight": np.full((H, W), w, np.float32)}
    if f32:
        kf["color"] = np.broadcast_to(np.array(rgb, np.float32) / 255.0, (H, W, 3)).copy()
    else:
        c = np.zeros((H, W, 4), np.uint8)
        c[..., :3] = rgb
        c[..., 3] = 255
        kf["color"] = c
    return kf


def _plane_depth(n, c, R, t, intr):
    """Exact z-depth of the world plane n.x = c seen from pose (R, t)."""
    u = np.arange(intr.width, dtype=np.float64)
    v = np.arange(intr.height, dtype=np.float64)
    rc = np.stack(np.broadcast_arrays((u[None, :] - intr.cx) / intr.fx, (v[:, None] - intr.cy) / intr.fy,
                                      np.ones((intr.height, intr.width))), -1)
    dw = rc @ R.T
    lam = (c - n @ t) / (dw @ n)
    return lam


def _voxels(field):
    b = field["blocks"]
    k = np.arange(512)
    off = np.stack([k & 7, (k >> 3) & 7, k >> 6], 1)
    return (8 * b[:, None, :] + off[None]).reshape(-1, 3)


def test_fronto_parallel_wall_closed_form():
    """Camera at the origin looking along +z at a constant-depth keyframe: every
    touched voxel holds D = Z0 - z_v (positive in front of the surface), W = w and
    the keyframe colour; the touched set is the band |Z0 - z_v| <= mu inside the
    image."""
    Z0 = np.float32(1.5)
    vol = oracle.Volume(S, MU)
    kf = _const_kf(Z0, w=0.5)
    assert vol.integrate(kf, INTR, np.eye(3), np.zeros(3)) == oracle.OK
    f = vol.export()
    n = _voxels(f)
    W = f["W"].reshape(-1)
    D = f["D"].reshape(-1)
    C = f["C"].reshape(-1, 3)
    hit = W > 0
    zv = S * n[:, 2]
    np.testing.assert_array_equal(D[hit], np.float64(Z0) - np.float32(S).astype(np.float64) * n[hit, 2])
    assert np.all(W[hit] == 0.5)
    assert np.all(C[hit] == [10, 20, 30])
    assert np.all(np.abs(D[hit]) <= MU + 1e-6)
    # completeness: voxels well inside the band and the image are all touched
    x = np.float32(S).astype(np.float64) * n
    u = INTR.fx * x[:, 0] / x[:, 2] + INTR.cx
    v = INTR.fy * x[:, 1] / x[:, 2] + INTR.cy
    inside = (np.abs(Z0 - zv) < MU - 1e-4) & (u > 0.5) & (u < INTR.width - 1.5) & (v > 0.5) & (v < INTR.height - 1.5)
    assert inside.sum() > 1000
    assert np.all(hit[inside])
    # soundness: nothing outside the band; the in-front side has D > 0
    assert np.all(np.abs(Z0 - zv[hit]) <= MU + 1e-6)
    assert np.all(D[hit & (zv < Z0 - 1e-6)] > 0) and np.all(D[hit & (zv > Z0 + 1e-6)] < 0)


@pytest.mark.parametrize("pose_id", [0, 1, 2])
def test_slanted_plane_rotated_camera(pose_id):
    """A world plane seen from a rotated, translated camera with noise-free depth.
    Each touched voxel's D equals the projective distance with depth sampled at
    the voxel's own ray up to the nearest-pixel offset (<= 0.71 px times the
    depth gradient), and the voxel lies within the band of the plane in world
    coordinates; a transposed rotation or a sign error in t breaks both."""
    rng = np.random.default_rng(pose_id)
    R = _rot(rng.uniform(-0.2, 0.2), rng.uniform(-0.5, 0.2), rng.uniform(-3, 3))
    t = np.array([1.0, 2.0, 1.4]) + rng.uniform(-0.3, 0.3, 3)
    fwd = R[:, 2]
    nrm = -fwd + 0.4 * rng.standard_normal(3)
    nrm /= np.linalg.norm(nrm)
    c = float(nrm @ (t + 1.8 * fwd))
    Z = _plane_depth(nrm, c, R, t, INTR)
    ok = (Z > 0.3) & (Z < 4.0)
    kf = {"depth": np.where(ok, Z, 0).astype(np.float32), "weight": ok.astype(np.float32),
          "color": np.zeros((INTR.height, INTR.width, 4), np.uint8)}
    vol = oracle.Volume(S, MU)
    assert vol.integrate(kf, INTR, R, t) == oracle.OK
    f = vol.export()
    n = _voxels(f)
    W = f["W"].reshape(-1)
    D = f["D"].reshape(-1)
    hit = W > 0
    assert hit.sum() > 5000
    x = np.float32(S).astype(np.float64) * n[hit]
    p = (x - t) @ R  # camera coordinates
    uu = INTR.fx * p[:, 0] / p[:, 2] + INTR.cx
    vv = INTR.fy * p[:, 1] / p[:, 2] + INTR.cy
    ray = np.stack([(uu - INTR.cx) / INTR.fx, (vv - INTR.cy) / INTR.fy, np.ones_like(uu)], 1)
    z_ray = (c - nrm @ t) / ((ray @ R.T) @ nrm)
    d_ray = z_ray - p[:, 2]
    # depth gradient of the plane in pixels at the voxel's projection
    eps = 1e-3
    ray_u = ray + np.array([eps / INTR.fx, 0, 0])
    ray_v = ray + np.array([0, eps / INTR.fy, 0])
    gz = np.abs((c - nrm @ t) / ((ray_u @ R.T) @ nrm) - z_ray) / eps + np.abs(
        (c - nrm @ t) / ((ray_v @ R.T) @ nrm) - z_ray) / eps
    bound = 0.71 * gz + 1e-5
    assert np.all(np.abs(D[hit] - d_ray) <= bound)
    # world-space band: the Euclidean distance to the plane is at most the
    # distance along the viewing ray, |d_proj| * |(x/z, y/z, 1)|
    d_euc = c - x @ nrm
    assert np.all(np.abs(d_euc) <= np.linalg.norm(ray, axis=1) * (MU + bound) + 1e-6)


def _c1_keyframe():
    wl = synth.workload(1)
    z, rgb = synth.frames(wl, range(5))
    kf = oracle.kf_fuse(z, rgb, wl.intr, wl.R, wl.t)
    return wl, kf


@pytest.fixture(scope="module")
def c1():
    return _c1_keyframe()


def test_sparse_enumeration_equals_brute_force(c1):
    wl, kf = c1
    Rp, tp = synth.perturb_fixed(wl.R[:1], wl.t[:1], 0.01, 0.5, 11)
    for R, t in [(wl.R[0], wl.t[0]), (Rp[0], tp[0])]:
        a = oracle.Volume(S, MU)
        assert a.integrate(kf, wl.intr, R, t) == oracle.OK
        fa = a.export()
        lo, hi = fa["blocks"].min(0) - 3, fa["blocks"].max(0) + 3
        b = oracle.Volume(S, MU)
        assert b.integrate(kf, wl.intr, R, t, box=(lo, hi)) == oracle.OK
        fb = b.export()
        np.testing.assert_array_equal(fa["blocks"], fb["blocks"])
        np.testing.assert_array_equal(fa["W"], fb["W"])
        np.testing.assert_array_equal(fa["D"], fb["D"])
        np.testing.assert_array_equal(fa["C"], fb["C"])


def _kfs_f32(n_kf=4, seed=0):
    wl = synth.workload(3)
    out = []
    for k in range(n_kf):
        idx = np.arange(5) + 5 * k * 4
        z, rgb = synth.frames(wl, idx)
        kf = oracle.kf_fuse(z, rgb, wl.intr, wl.R[idx], wl.t[idx])
        kf = {"depth": kf["depth"], "weight": kf["weight"], "color": kf["color"][..., :3].astype(np.float32) / 255.0}
        out.append((kf, wl.R[idx[0]], wl.t[idx[0]]))
    return wl, out


@pytest.fixture(scope="module")
def kfs4():
    return _kfs_f32()


def _run(seq, wl, color_f32=True):
    v = oracle.Volume(S, MU, color_f32=color_f32)
    for sign, (kf, R, t) in seq:
        rc = v.integrate(kf, wl.intr, R, t) if sign > 0 else v.deintegrate(kf, wl.intr, R, t)
        assert rc == oracle.OK
    return v.export()


def _align(fa, fb):
    """Compare two fields on the union of their blocks (never-touched = zero)."""
    keys = np.unique(np.concatenate([fa["blocks"], fb["blocks"]]), axis=0)

    def pad(f):
        idx = {tuple(b): i for i, b in enumerate(f["blocks"])}
        D = np.zeros((len(keys), 512))
        W = np.zeros((len(keys), 512))
        C = np.zeros((len(keys), 512, 3))
        for j, k in enumerate(map(tuple, keys)):
            if k in idx:
                D[j], W[j], C[j] = f["D"][idx[k]], f["W"][idx[k]], f["C"][idx[k]]
        return D, W, C

    return pad(fa), pad(fb)


def test_reversibility(kfs4):
    """Integrate A, B, C then de-integrate B equals integrating A, C (Eq. 2
    reverses the running average): W bit-exact, D and C to 1e-12."""
    wl, ks = kfs4
    A, B, Cc = ks[0], ks[1], ks[2]
    f1 = _run([(1, A), (1, B), (1, Cc), (-1, B)], wl)
    f2 = _run([(1, A), (1, Cc)], wl)
    (D1, W1, C1), (D2, W2, C2) = _align(f1, f2)
    np.testing.assert_array_equal(W1, W2)
    assert np.abs(D1 - D2).max() <= 1e-12
    assert np.abs(C1 - C2).max() <= 1e-12
    # everything out again -> empty field (blocks stay allocated)
    f3 = _run([(1, A), (1, B), (-1, A), (-1, B)], wl)
    assert np.all(f3["W"] == 0) and np.all(f3["D"] == 0) and np.all(f3["C"] == 0)


def test_order_independence(kfs4):
    wl, ks = kfs4
    rng = np.random.default_rng(3)
    ref = _run([(1, k) for k in ks], wl)
    for _ in range(3):
        perm = rng.permutation(len(ks))
        f = _run([(1, ks[i]) for i in perm], wl)
        np.testing.assert_array_equal(f["blocks"], ref["blocks"])
        np.testing.assert_array_equal(f["W"], ref["W"])
        assert np.abs(f["D"] - ref["D"]).max() <= 1e-12
        assert np.abs(f["C"] - ref["C"]).max() <= 1e-12


def test_running_average_two_keyframes_closed_form():
    """Two constant-depth keyframes at the identity pose: D = (w1 d1 + w2 d2)/(w1 + w2)."""
    Z1, Z2, w1, w2 = np.float32(1.50), np.float32(1.52), 0.75, 0.25
    v = oracle.Volume(S, MU, color_f32=True)
    v.integrate(_const_kf(Z1, w1, (255, 0, 0), f32=True), INTR, np.eye(3), np.zeros(3))
    v.integrate(_const_kf(Z2, w2, (0, 255, 0), f32=True), INTR, np.eye(3), np.zeros(3))
    f = v.export()
    n = _voxels(f)
    W, D, C = f["W"].reshape(-1), f["D"].reshape(-1), f["C"].reshape(-1, 3)
    zv = np.float32(S).astype(np.float64) * n[:, 2]
    both = W == w1 + w2
    assert both.sum() > 1000
    exp = (w1 * (np.float64(Z1) - zv[both]) + w2 * (np.float64(Z2) - zv[both])) / (w1 + w2)
    assert np.abs(D[both] - exp).max() <= 1e-15
    np.testing.assert_allclose(C[both], [[w1, w2, 0]] * both.sum(), atol=1e-15)


def test_rgba8_colour_rounding_ties_to_even():
    v = oracle.Volume(S, MU)
    v.integrate(_const_kf(np.float32(1.5), 0.5, (10, 11, 200)), INTR, np.eye(3), np.zeros(3))
    v.integrate(_const_kf(np.float32(1.5), 0.5, (11, 12, 201)), INTR, np.eye(3), np.zeros(3))
    f = v.export()
    C = f["C"].reshape(-1, 3)[f["W"].reshape(-1) > 0]
    # 10.5 -> 10, 11.5 -> 12, 200.5 -> 200
    assert np.all(C == [10, 12, 200])
    # de-integrating one of them from uint8 storage: (10*1 - 11*0.5)/0.5 = 9
    v.deintegrate(_const_kf(np.float32(1.5), 0.5, (11, 12, 201)), INTR, np.eye(3), np.zeros(3))
    f = v.export()
    C = f["C"].reshape(-1, 3)[f["W"].reshape(-1) > 0]
    assert np.all(C == [9, 12, 199])


def test_error_paths(c1):
    wl, kf = c1
    v = oracle.Volume(S, MU)
    assert v.deintegrate(kf, wl.intr, wl.R[0], wl.t[0]) == oracle.ENOTALLOC
    assert v.integrate(kf, wl.intr, wl.R[0], wl.t[0]) == oracle.OK
    assert v.deintegrate(kf, wl.intr, wl.R[0], wl.t[0]) == oracle.OK
    assert v.deintegrate(kf, wl.intr, wl.R[0], wl.t[0]) == oracle.EWEIGHT
    heavy = _const_kf(np.float32(1.5), 8192.0)
    v2 = oracle.Volume(S, MU)
    assert v2.integrate(heavy, INTR, np.eye(3), np.zeros(3)) == oracle.OK
    assert v2.integrate(heavy, INTR, np.eye(3), np.zeros(3)) == oracle.EWEIGHT


def test_weight_quantisation_drops_tiny_weights():
    v = oracle.Volume(S, MU)
    assert v.integrate(_const_kf(np.float32(1.5), 0.0004), INTR, np.eye(3), np.zeros(3)) == oracle.OK
    assert v.n_blocks == 0
    v.integrate(_const_kf(np.float32(1.5), 0.0006), INTR, np.eye(3), np.zeros(3))
    f = v.export()
    assert np.all(f["W"][f["W"] > 0] == 2.0**-10)


def test_voxel_sequence_equals_volume_path(c1):
    """The per-voxel sequence (used to check large volumes on samples) equals
    the volume path on every voxel of a small case."""
    wl, kf = c1
    Rp, tp = synth.perturb_fixed(wl.R[:1], wl.t[:1], 0.01, 0.5, 11)
    v = oracle.Volume(S, MU)
    v.integrate(kf, wl.intr, wl.R[0], wl.t[0])
    v.deintegrate(kf, wl.intr, wl.R[0], wl.t[0])
    v.integrate(kf, wl.intr, Rp[0], tp[0])
    f = v.export()
    ops = [(0, 1, wl.R[0], wl.t[0]), (0, -1, wl.R[0], wl.t[0]), (0, 1, Rp[0], tp[0])]
    rng = np.random.default_rng(0)
    for b in rng.choice(len(f["blocks"]), 20, replace=False):
        for i in rng.choice(512, 8, replace=False):
            n = 8 * f["blocks"][b] + np.array([i & 7, (i >> 3) & 7, i >> 6])
            D, W, C, rc = v.voxel_sequence([kf], wl.intr, ops, n)
            assert rc >= 0 and W == f["W"][b, i] and D == f["D"][b, i] and np.array_equal(C, f["C"][b, i])
