"""The oracle's FP32 decision convention against the plain FP64 definitions.

The oracle takes its discrete decisions (which pixel a voxel or a warped
point falls on, band membership, the discontinuity test, the quantised depth
weight) in FP32 in a written order, the same convention the HIP path
follows.  The paper fixes no precision, so these tests write the plain
definitions of Sec. 3 out in FP64, independently of the oracle, and check
that the convention agrees with them everywhere except where the FP64 value
lies within the convention's own rounding bound of a decision boundary:

* camera point of voxel n: p = R^T (s n - t)                 (Sec. 3, SDF volume)
* nearest pixel: floor(fx X / Z + cx + 1/2), likewise v     (Sec. 3, pinhole)
* touched: p_z > 0, pixel inside the image, q(W*) > 0 and
  |Z*(pixel) - p_z| <= mu                                    (Sec. 3; Sec. 4.3 names d)
* depth weight: w_z = q(cos(theta) / Z^2) with the central-difference normal,
  rejected next to a discontinuity or an invalid neighbour     (Sec. 3, Keyframe Fusion)
* forward warp of Eq. 1: p* = T*^-1 T_i pi^-1(x, Z_i(x)), target pixel the
  nearest pixel of pi(p*), weighted mean of the warped depths  (Sec. 3, Eq. 1)

Each bound is derived from the FP32 operations of the convention (unit
roundoff u = 2^-24 per operation, first order, then doubled); a disagreement
farther from its boundary than that bound fails the test, and the counts are
printed.  The inputs are fused keyframes of the tiny room, the
differentiation room and the large batched room (640x480, 1 cm voxels).
"""

import numpy as np
import pytest

import oracle
from paper_1709_03763_amd import synth

U32 = 2.0 ** -24


def _f32(x):
    return float(np.float32(x))


# --------------------------------------------------------------------------
# FP64 definitions
# --------------------------------------------------------------------------


def _cam_points(n, s, R, t):
    """p = R^T (s n - t) in FP64, and the FP32 convention's error bound on it."""
    x = s * n.astype(np.float64)
    e = x - t[None, :]
    p = e @ R  # column r of R is row r of R^T
    # The convention rounds the FP64 block-origin point once, rounds the three
    # per-axis steps fl32(s R), and adds k * step along x, y, z in FP32: at
    # most eight roundings, each of a value no larger than |p|_inf + 21 s
    # (the partial sums of the in-block offset, 7 voxels per axis).
    eps = 8.0 * U32 * (np.abs(p).max(1) + 21.0 * s)
    return p, 2.0 * eps


def _pixel(p, fx, cx):
    """u = fx X / Z + cx and its nearest pixel floor(u + 1/2)."""
    u = fx * p[:, 0] / p[:, 2] + cx
    return u, np.floor(u + 0.5)


def _pixel_eps(p, eps_p, fx, cx, u):
    """Bound on |u_fp32 - u_fp64| for the convention fl(fl(fl(fx X) / Z) + cx),
    then fl(u + 1/2), given |p_fp32 - p| <= eps_p per component."""
    Z = p[:, 2]
    X = p[:, 0]
    prop = (fx / Z) * (1.0 + np.abs(X) / Z) * eps_p
    rnd = U32 * (2.0 * np.abs(fx * X / Z) + 2.0 * np.abs(u) + 1.0)
    return 2.0 * (prop + rnd)


def _half_margin(u):
    """Distance of u to the nearest half-integer, where floor(u + 1/2) steps."""
    return np.abs(u - (np.floor(u) + 0.5))


def _tile_domain(kf, intr, R, t, s, mu, tile=16):
    """Every lattice point that can be touched under the FP64 definition: a
    touched voxel lies in its pixel's frustum cell between Z* - mu and Z* + mu,
    so inside the world AABB of the frustum piece of that pixel's image tile
    between the tile's smallest depth - mu and largest depth + mu (a convex
    set spanned by its 8 corners), padded by one voxel."""
    Z = kf["depth"].astype(np.float64)
    Wq = np.rint(kf["weight"].astype(np.float64) * 1024.0)
    ok = (Wq > 0) & (Z > 0)
    H, W = Z.shape
    keys = []
    for v0 in range(0, H, tile):
        for u0 in range(0, W, tile):
            m = ok[v0:v0 + tile, u0:u0 + tile]
            if not m.any():
                continue
            zz = Z[v0:v0 + tile, u0:u0 + tile][m]
            zl, zh = max(zz.min() - mu, 1e-3), zz.max() + mu
            u1, v1 = min(u0 + tile, W) - 1, min(v0 + tile, H) - 1
            cs = []
            for uu in (u0 - 0.5, u1 + 0.5):
                for vv in (v0 - 0.5, v1 + 0.5):
                    for z in (zl, zh):
                        cs.append(((uu - intr.cx) * z / intr.fx, (vv - intr.cy) * z / intr.fy, z))
            w = np.array(cs) @ R.T + t[None, :]
            lo = np.floor(w.min(0) / s).astype(np.int64) - 1
            hi = np.ceil(w.max(0) / s).astype(np.int64) + 1
            g = np.stack(np.meshgrid(*[np.arange(lo[a], hi[a] + 1) for a in range(3)], indexing="ij"), -1)
            keys.append(_pack(g.reshape(-1, 3)))
    k = np.unique(np.concatenate(keys))
    return _unpack(k)


def _pack(n):
    n = n.astype(np.int64) + (1 << 20)
    return (n[:, 0] << 42) | (n[:, 1] << 21) | n[:, 2]


def _unpack(k):
    m = (1 << 21) - 1
    return np.stack([(k >> 42) & m, (k >> 21) & m, k & m], 1).astype(np.int64) - (1 << 20)


def _touched_fp64(kf, intr, R, t, s, mu):
    n = _tile_domain(kf, intr, R, t, s, mu)
    p, eps_p = _cam_points(n, s, R, t)
    H, W = kf["depth"].shape
    front = p[:, 2] > 0
    n, p, eps_p = n[front], p[front], eps_p[front]
    u, iu = _pixel(p, intr.fx, intr.cx)
    v, iv = _pixel(p[:, [1, 0, 2]], intr.fy, intr.cy)
    inb = (iu >= 0) & (iu <= W - 1) & (iv >= 0) & (iv <= H - 1)
    pix = np.where(inb, iv * W + iu, 0).astype(np.int64)
    Zs = kf["depth"].reshape(-1).astype(np.float64)
    wq = np.rint(kf["weight"].reshape(-1).astype(np.float64) * 1024.0)
    d = Zs[pix] - p[:, 2]
    hit = inb & (wq[pix] > 0) & (np.abs(d) <= mu)
    eps_u = _pixel_eps(p, eps_p, intr.fx, intr.cx, u)
    eps_v = _pixel_eps(p[:, [1, 0, 2]], eps_p, intr.fy, intr.cy, v)
    near_px = (_half_margin(u) <= eps_u) | (_half_margin(v) <= eps_v)
    eps_d = 2.0 * (eps_p + U32 * mu)
    near_band = np.abs(np.abs(d) - mu) <= eps_d
    return {"n": n, "hit": hit, "pix": pix, "d": d, "near_px": near_px, "near_band": near_band,
            "px_ratio": np.minimum(_half_margin(u) / eps_u, _half_margin(v) / eps_v),
            "band_ratio": np.abs(np.abs(d) - mu) / eps_d}


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------


_CASES = {
    "tiny": (1, range(0, 5)),
    "diff": (3, range(20, 25)),
    "batched_vga": (4, range(0, 5)),
}


@pytest.fixture(scope="module", params=sorted(_CASES))
def case(request):
    cfg, grp = _CASES[request.param]
    wl = synth.workload(cfg)
    g = np.asarray(list(grp))
    z, rgb = synth.frames(wl, g)
    kf = oracle.kf_fuse(z, rgb, wl.intr, wl.R[g], wl.t[g])
    return request.param, wl, g, z, kf


def _poses(wl, g):
    R0, t0 = wl.R[g[0]], wl.t[g[0]]
    Rn, tn = synth.perturb_fixed(wl.R[g[:1]], wl.t[g[:1]], 0.03, 1.5, 7)
    return [(R0, t0), (Rn[0], tn[0])]


# --------------------------------------------------------------------------
# the touched set (and so every allocated block set)
# --------------------------------------------------------------------------


def test_touched_set_matches_fp64_definition(case):
    name, wl, g, _, kf = case
    s, mu = _f32(wl.volume.voxel_size), _f32(wl.volume.trunc)
    for pi, (R, t) in enumerate(_poses(wl, g)):
        ref = _touched_fp64(kf, wl.intr, R, t, s, mu)
        vol = oracle.Volume(wl.volume.voxel_size, wl.volume.trunc)
        rec = vol.record(kf, wl.intr, R, t)
        k64 = _pack(ref["n"])
        k32 = _pack(rec["n"].astype(np.int64))
        # the FP64 domain holds every voxel the convention touches
        assert np.isin(k32, k64).all(), "a touched voxel lies outside the FP64 frustum domain"
        hit64 = np.isin(k64, k32)
        disagree = hit64 != ref["hit"]
        explained = ref["near_px"] | ref["near_band"]
        n_dis = int(disagree.sum())
        assert np.all(explained[disagree]), (
            f"{name}: {int((disagree & ~explained).sum())} touched-set disagreements away from any "
            f"decision boundary")
        # on agreement the pixel is the FP64 pixel unless the pixel decision is
        # within its bound, and d is the FP64 projective distance
        both = hit64 & ref["hit"]
        order = np.argsort(k32)
        j = order[np.searchsorted(k32, k64[both], sorter=order)]
        same_px = rec["pix"][j] == ref["pix"][both]
        assert np.all(same_px | ref["near_px"][both])
        sp = same_px
        np.testing.assert_allclose(rec["d"][j][sp], ref["d"][both][sp], rtol=0, atol=1e-12)
        blocks64 = np.unique(_pack(np.floor_divide(ref["n"][ref["hit"]], 8)))
        blocks32 = np.unique(_pack(np.floor_divide(rec["n"].astype(np.int64), 8)))
        n_bdis = len(np.setxor1d(blocks64, blocks32))
        print(f"[fp64-definition] {name} pose {pi}: {int(ref['hit'].sum())} voxels touched in FP64, "
              f"{len(k32)} by the convention, {n_dis} differ (all within the rounding bound of a pixel "
              f"or band boundary; closest ratio to the bound "
              f"{float(np.minimum(ref['px_ratio'], ref['band_ratio'])[disagree].max()) if n_dis else 0:.3f}); "
              f"{len(blocks64)} blocks in FP64, {n_bdis} differ; "
              f"{int((~same_px).sum())} agreeing voxels at a different pixel", flush=True)
        assert ref["hit"].sum() > 1000


# --------------------------------------------------------------------------
# the depth weight w_z
# --------------------------------------------------------------------------


def _depth_weight_fp64(Z32, intr, zmin, zmax, disc):
    """w_z = q(cos(theta) / Z^2) in FP64, with the bound of the FP32 convention
    on 1024 w and the margins of its discrete decisions."""
    Z = Z32.astype(np.float64)
    H, W = Z.shape
    out = np.zeros((H, W))
    valid = (Z32 >= np.float32(zmin)) & (Z32 <= np.float32(zmax))
    c = (slice(1, H - 1), slice(1, W - 1))
    z = Z[c]
    nb = {"l": Z[1:H - 1, 0:W - 2], "r": Z[1:H - 1, 2:W], "u": Z[0:H - 2, 1:W - 1], "d": Z[2:H, 1:W - 1]}
    vb = {"l": valid[1:H - 1, 0:W - 2], "r": valid[1:H - 1, 2:W], "u": valid[0:H - 2, 1:W - 1],
          "d": valid[2:H, 1:W - 1]}
    ok = valid[c] & vb["l"] & vb["r"] & vb["u"] & vb["d"]
    th = disc * z  # exact in FP64 (24-bit by 24-bit product)
    disc_margin = np.full(z.shape, np.inf)
    for k in nb:
        diff = np.abs(nb[k] - z)
        ok &= ~(diff > th)
        disc_margin = np.minimum(disc_margin, np.abs(diff - th))
    vv, uu = np.mgrid[1:H - 1, 1:W - 1].astype(np.float64)

    def bp(u, v, zz):
        return np.stack([(u - intr.cx) * zz / intr.fx, (v - intr.cy) * zz / intr.fy, zz], -1)

    Pl, Pr = bp(uu - 1, vv, nb["l"]), bp(uu + 1, vv, nb["r"])
    Pu, Pd = bp(uu, vv - 1, nb["u"]), bp(uu, vv + 1, nb["d"])
    a, b = Pr - Pl, Pd - Pu
    n = np.cross(a, b)
    nn = (n * n).sum(-1)
    cos = np.abs(n[..., 2]) / np.sqrt(np.where(nn > 0, nn, 1.0))
    w = np.where(ok, cos / np.where(ok, z * z, 1.0), 0.0)
    # FP32 error bound of the convention, first order: back-projected
    # coordinates carry two roundings, differences and cross products one or
    # two more per term, then the norm, the square root and the divisions.
    da = 2 * U32 * (np.abs(Pr) + np.abs(Pl)) + U32 * np.abs(a)
    db = 2 * U32 * (np.abs(Pd) + np.abs(Pu)) + U32 * np.abs(b)
    aa, ab = np.abs(a), np.abs(b)
    dn = np.stack([
        da[..., 1] * ab[..., 2] + aa[..., 1] * db[..., 2] + da[..., 2] * ab[..., 1] + aa[..., 2] * db[..., 1]
        + 3 * U32 * (aa[..., 1] * ab[..., 2] + aa[..., 2] * ab[..., 1]),
        da[..., 2] * ab[..., 0] + aa[..., 2] * db[..., 0] + da[..., 0] * ab[..., 2] + aa[..., 0] * db[..., 2]
        + 3 * U32 * (aa[..., 2] * ab[..., 0] + aa[..., 0] * ab[..., 2]),
        da[..., 0] * ab[..., 1] + aa[..., 0] * db[..., 1] + da[..., 1] * ab[..., 0] + aa[..., 1] * db[..., 0]
        + 3 * U32 * (aa[..., 0] * ab[..., 1] + aa[..., 1] * ab[..., 0])], -1)
    nabs = np.abs(n)
    rel_nn = (2 * (nabs * dn).sum(-1) + 3 * U32 * nn) / np.where(nn > 0, nn, 1.0)
    rel_cos = dn[..., 2] / np.maximum(nabs[..., 2], 1e-300) + 0.5 * rel_nn + 2 * U32
    rel_w = rel_cos + 3 * U32
    q = np.rint(w * 1024.0) / 1024.0
    inner = np.where(ok & (nn > 0), q, 0.0)
    out[c] = inner
    eps_q = np.zeros((H, W))
    eps_q[c] = 2.0 * 1024.0 * w * rel_w
    w1024 = np.zeros((H, W))
    w1024[c] = w * 1024.0
    dm = np.full((H, W), np.inf)
    dm[c] = disc_margin
    eps_disc = np.zeros((H, W))
    eps_disc[c] = 2.0 * U32 * th
    return out, w1024, eps_q, dm, eps_disc


def test_depth_weight_matches_fp64_definition(case):
    name, wl, g, z, _ = case
    zmin, zmax, disc = _f32(synth.Z_MIN), _f32(synth.Z_MAX), _f32(0.05)
    tot_dis = tot = 0
    for i in range(len(g)):
        w32 = oracle.depth_weight(z[i], wl.intr).astype(np.float64)
        w64, w1024, eps_q, dm, eps_disc = _depth_weight_fp64(z[i], wl.intr, zmin, zmax, disc)
        dis = w32 != w64
        near_q = np.abs(w1024 - (np.floor(w1024) + 0.5)) <= eps_q
        near_disc = dm <= eps_disc
        expl = near_q | near_disc
        assert np.all(expl[dis]), f"{name} frame {i}: {int((dis & ~expl).sum())} w_z differ away from a boundary"
        # a disagreement is one quantum of 2^-10, or a rejection decided at its boundary
        one_q = np.abs(w32 - w64) <= 1.0 / 1024 + 1e-12
        assert np.all((one_q | near_disc)[dis])
        tot_dis += int(dis.sum())
        tot += int((w64 > 0).sum())
    print(f"[fp64-definition] {name}: w_z of {tot} pixels, {tot_dis} differ by one 2^-10 quantum, each "
          f"within the FP32 bound of a rounding boundary", flush=True)
    assert tot > 1000


# --------------------------------------------------------------------------
# the forward warp of Eq. 1
# --------------------------------------------------------------------------


def _fuse_depth_fp64(Z, wz, intr, R, t, ref=0):
    """Eq. 1 in FP64: target pixels from the exact relative pose, K_W and
    K_Z accumulated exactly, with each contribution's pixel margin and the
    convention's bound on it."""
    n, H, W = Z.shape
    KW = np.zeros(H * W, np.int64)
    KZ = np.zeros(H * W, np.int64)
    near = np.zeros(H * W, bool)
    eps_z = 0.0
    Rs, ts = R[ref], t[ref]
    vv, uu = np.mgrid[0:H, 0:W].astype(np.float64)
    for i in range(n):
        Rr = Rs.T @ R[i]
        tr = Rs.T @ (t[i] - ts)
        w = wz[i].astype(np.float64)
        m = w > 0
        z = Z[i].astype(np.float64)[m]
        P = np.stack([(uu[m] - intr.cx) * z / intr.fx, (vv[m] - intr.cy) * z / intr.fy, z], 1)
        q = P @ Rr.T + tr[None, :]
        # FP32 convention: P with two roundings per coordinate, R_rel and t_rel
        # rounded to FP32, then three products and three sums per row
        S = np.abs(P) @ np.abs(Rr).T + np.abs(tr)[None, :]
        eps_p = 2.0 * 9.0 * U32 * S
        front = q[:, 2] > 0
        u = intr.fx * q[:, 0] / q[:, 2] + intr.cx
        v = intr.fy * q[:, 1] / q[:, 2] + intr.cy
        iu, iv = np.floor(u + 0.5), np.floor(v + 0.5)
        inb = front & (iu >= 0) & (iu <= W - 1) & (iv >= 0) & (iv <= H - 1)
        ep = eps_p.max(1)
        eu = _pixel_eps(q, ep, intr.fx, intr.cx, u)
        ev = _pixel_eps(q[:, [1, 0, 2]], ep, intr.fy, intr.cy, v)
        nu = _half_margin(u) <= eu
        nv = _half_margin(v) <= ev
        wk = np.rint(w[m] * 1024.0).astype(np.int64)
        zk = np.rint(q[:, 2] * 1048576.0).astype(np.int64)
        tgt = (iv * W + iu).astype(np.int64)
        np.add.at(KW, tgt[inb], wk[inb])
        np.add.at(KZ, tgt[inb], wk[inb] * zk[inb])
        eps_z = max(eps_z, float(eps_p[inb, 2].max()) if inb.any() else 0.0)
        # a contribution whose pixel decision lies within its bound may land on
        # the FP64 target or on the neighbour across the near boundary
        for flag, du, dv in ((nu, 1, 0), (nv, 0, 1)):
            sel = flag & front
            if not sel.any():
                continue
            side_u = np.where(u[sel] - iu[sel] > 0, 1, -1) if du else 0
            side_v = np.where(v[sel] - iv[sel] > 0, 1, -1) if dv else 0
            for cu, cv in ((iu[sel], iv[sel]), (iu[sel] + du * side_u, iv[sel] + dv * side_v)):
                okp = (cu >= 0) & (cu <= W - 1) & (cv >= 0) & (cv <= H - 1)
                near[(cv[okp] * W + cu[okp]).astype(np.int64)] = True
        both = nu & nv & front
        if both.any():
            su = np.where(u[both] - iu[both] > 0, 1, -1)
            sv = np.where(v[both] - iv[both] > 0, 1, -1)
            cu, cv = iu[both] + su, iv[both] + sv
            okp = (cu >= 0) & (cu <= W - 1) & (cv >= 0) & (cv <= H - 1)
            near[(cv[okp] * W + cu[okp]).astype(np.int64)] = True
    Ws = KW / 1024.0
    Zs = np.where(KW > 0, (KZ / np.maximum(KW, 1)) * 2.0 ** -20, 0.0).astype(np.float32)
    return Zs.reshape(H, W), Ws.reshape(H, W).astype(np.float32), near.reshape(H, W), eps_z


def test_forward_warp_matches_fp64_definition(case):
    name, wl, g, z, _ = case
    wz = np.stack([oracle.depth_weight(z[i], wl.intr) for i in range(len(g))])
    Z32, W32 = oracle.fuse_depth(z, wz, wl.intr, wl.R[g], wl.t[g])
    Z64, W64, near, eps_z = _fuse_depth_fp64(z, wz, wl.intr, wl.R[g], wl.t[g])
    dis = W32 != W64
    assert np.all(near[dis]), f"{name}: {int((dis & ~near).sum())} fused weights differ away from a boundary"
    same = ~dis & (W64 > 0)
    # each contribution's 2^-20 m depth quantum can move by the FP32 error of
    # its warped depth (plus one quantum for the rounding), and Z* is rounded
    # to FP32 once
    dz = np.abs(Z32.astype(np.float64) - Z64.astype(np.float64))[same]
    bound = eps_z + 2.0 ** -20 + U32 * 2 * synth.Z_MAX
    assert dz.max() <= bound, (dz.max(), bound)
    print(f"[fp64-definition] {name}: {int((W64 > 0).sum())} fused pixels, {int(dis.sum())} with a different "
          f"weight sum (all next to a warp target within the FP32 bound of a pixel boundary); "
          f"max |Z*_fp32 - Z*_fp64| = {dz.max():.2e} m on the rest (bound {bound:.2e})", flush=True)
    assert (W64 > 0).sum() > 1000
