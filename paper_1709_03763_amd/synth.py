"""Seeded synthetic RGB-D inputs shaped like handheld indoor scans.

This module is input generation only and is shared by the FP64 oracle tests
and the HIP path.  It holds none of the surface-correction method's
arithmetic: it builds analytic scenes (room interiors, spheres, axis-aligned
boxes), ray-casts exact z-depth in float64, adds the sensor noise model,
paints a procedural 3-D checker texture, draws smooth camera trajectories and
the pose-graph corrections that drive re-integration.

Conventions (the paper's problem statement, Sec. 3 "Preliminaries"): a pose
T = (R, t) maps camera coordinates to world coordinates, g(T, p) = R p + t.
Cameras are OpenCV-style (x right, y down, z forward); the world is z-up.
Depth is z-depth in camera coordinates.  A pixel (u, v) has its centre at
integer coordinates, so the ray through it is ((u-cx)/fx, (v-cy)/fy, 1) in
camera coordinates and the ray parameter equals the z-depth.

Every random draw uses numpy's PCG64 seeded explicitly, so a configuration is
reproducible bit for bit on any machine; only ray casting may run on a GPU
through torch (float64), and its inputs are the seeded arrays made here.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import torch

# ----------------------------------------------------------------------------
# cameras
# ----------------------------------------------------------------------------


@dataclass(frozen=True)
class Intrinsics:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float

    def as_array(self) -> np.ndarray:
        return np.array([self.fx, self.fy, self.cx, self.cy], dtype=np.float32)


QVGA = Intrinsics(320, 240, 262.5, 262.5, 159.5, 119.5)
VGA = Intrinsics(640, 480, 525.0, 525.0, 319.5, 239.5)

Z_MIN, Z_MAX = 0.3, 4.0


def noise_sigma(z: np.ndarray | torch.Tensor):
    """Axial depth noise of a structured-light sensor, metres."""
    return 0.0012 + 0.0019 * (z - 0.4) ** 2


# ----------------------------------------------------------------------------
# SE(3) helpers used to *generate* poses (never by the method itself)
# ----------------------------------------------------------------------------


def _skew(w):
    return np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]])


def se3_exp(xi: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Exponential map of xi = (rho, phi) -> (R, t)."""
    rho, phi = np.asarray(xi[:3], float), np.asarray(xi[3:], float)
    th = float(np.linalg.norm(phi))
    K = _skew(phi)
    if th < 1e-12:
        R = np.eye(3) + K
        V = np.eye(3) + 0.5 * K
    else:
        a = math.sin(th) / th
        b = (1 - math.cos(th)) / th**2
        c = (th - math.sin(th)) / th**3
        R = np.eye(3) + a * K + b * (K @ K)
        V = np.eye(3) + b * K + c * (K @ K)
    return R, V @ rho


def compose(Ra, ta, Rb, tb):
    """(Ra, ta) o (Rb, tb)."""
    return Ra @ Rb, Ra @ tb + ta


def look_pose(pos, yaw, pitch):
    """Camera-to-world pose at `pos` looking along (yaw, pitch), no roll."""
    f = np.array([math.cos(yaw) * math.cos(pitch), math.sin(yaw) * math.cos(pitch), math.sin(pitch)])
    r = np.array([math.sin(yaw), -math.cos(yaw), 0.0])
    d = np.cross(f, r)
    R = np.stack([r, d, f], axis=1)
    return R, np.asarray(pos, float).copy()


# ----------------------------------------------------------------------------
# scenes
# ----------------------------------------------------------------------------


@dataclass
class Scene:
    room_lo: np.ndarray
    room_hi: np.ndarray
    spheres: np.ndarray  # (S, 4): centre, radius
    boxes: np.ndarray  # (B, 6): lo xyz, hi xyz
    colors: np.ndarray  # (6 + S + B, 2, 3) uint8, two checker colours per surface
    checker: float = 0.10

    @property
    def n_prims(self) -> int:
        return 6 + len(self.spheres) + len(self.boxes)


def _point_aabb_dist(p, lo, hi):
    q = np.maximum(np.maximum(lo - p, p - hi), 0.0)
    return np.linalg.norm(q, axis=-1)


def _place_primitives(rng, lo, hi, path, n_sph, n_box, walls_extra=(), clearance=0.5,
                      r_range=(0.3, 0.6), side_range=(0.3, 1.2), tries=20000):
    spheres, boxes = [], []
    kinds = ["s"] * n_sph + ["b"] * n_box
    order = rng.permutation(len(kinds))
    for idx in order:
        kind = kinds[idx]
        for _ in range(tries):
            if kind == "s":
                r = rng.uniform(*r_range)
                c = rng.uniform(lo + r + 0.3, hi - r - 0.3)
                if np.min(np.linalg.norm(path - c, axis=1)) - r < clearance:
                    continue
                ok = all(np.linalg.norm(c - s[:3]) > r + s[3] + 0.05 for s in spheres)
                ok = ok and all(_point_aabb_dist(c, b[:3], b[3:]) > r + 0.05 for b in boxes)
                ok = ok and all(_point_aabb_dist(c, w[:3], w[3:]) > r + 0.05 for w in walls_extra)
                if ok:
                    spheres.append(np.array([*c, r]))
                    break
            else:
                sz = rng.uniform(*side_range, size=3)
                sz[2] = min(sz[2], 1.2)
                blo = np.array([rng.uniform(lo[0] + 0.3, hi[0] - 0.3 - sz[0]),
                                rng.uniform(lo[1] + 0.3, hi[1] - 0.3 - sz[1]), lo[2]])
                bhi = blo + sz
                if np.min(_point_aabb_dist(path, blo, bhi)) < clearance:
                    continue
                def overlaps(b):
                    return bool(np.all(blo < b[3:] + 0.05) and np.all(b[:3] < bhi + 0.05))

                ok = all(_point_aabb_dist(s[:3], blo, bhi) > s[3] + 0.05 for s in spheres)
                ok = ok and not any(overlaps(b) for b in boxes)
                ok = ok and not any(overlaps(np.asarray(w, float)) for w in walls_extra)
                if ok:
                    boxes.append(np.concatenate([blo, bhi]))
                    break
        else:
            raise RuntimeError("could not place primitive with the requested clearance")
    sph = np.array(spheres, float).reshape(-1, 4)
    box = np.array(boxes, float).reshape(-1, 6)
    return sph, box


def _colors(rng, n):
    c = rng.integers(30, 226, size=(n, 2, 3))
    return c.astype(np.uint8)


# ----------------------------------------------------------------------------
# trajectories
# ----------------------------------------------------------------------------


def _arclength_resample(curve, step, n):
    seg = np.linalg.norm(np.diff(curve, axis=0), axis=1)
    s = np.concatenate([[0.0], np.cumsum(seg)])
    targets = np.arange(n) * step
    if targets[-1] > s[-1]:
        raise ValueError("trajectory too short for the requested frame count")
    idx = np.searchsorted(s, targets, side="right") - 1
    idx = np.clip(idx, 0, len(curve) - 2)
    a = (targets - s[idx]) / np.maximum(seg[idx], 1e-15)
    return curve[idx] + a[:, None] * (curve[idx + 1] - curve[idx]), idx


def room_path(rng, lo, hi, n_frames, step=0.01, margin=1.0):
    """Smooth seeded Lissajous path at constant speed `step` m/frame."""
    c = 0.5 * (lo + hi)
    A = np.maximum(0.5 * (hi - lo) - margin, 0.2)
    fa, fb = 1.0, float(rng.choice([2.0, 3.0]))
    ph = rng.uniform(0, 2 * math.pi, size=4)
    need = n_frames * step * 1.2 + 1.0
    T = max(4.0 * math.pi, need)
    s = np.linspace(0.0, T * 8.0, 400000)
    curve = np.stack([c[0] + A[0] * np.sin(fa * s / 4 + ph[0]),
                      c[1] + A[1] * np.sin(fb * s / 4 + ph[1]),
                      1.5 + 0.3 * np.sin(0.7 * s / 4 + ph[2])], axis=1)
    pts, _ = _arclength_resample(curve, step, n_frames)
    return pts


def corridor_path(rng, n_frames, x0=1.0, x1=39.0):
    xs = np.linspace(x0, x1, 400000)
    ph = rng.uniform(0, 2 * math.pi)
    curve = np.stack([xs, 4.0 + 1.8 * np.sin(math.pi * xs / 10.0),
                      1.5 + 0.25 * np.sin(0.9 * xs + ph)], axis=1)
    seg = np.linalg.norm(np.diff(curve, axis=0), axis=1).sum()
    step = seg / (n_frames + 1)
    pts, _ = _arclength_resample(curve, step, n_frames)
    return pts


def _smooth(x, sigma):
    """Gaussian smoothing with edge padding (sigma in samples)."""
    r = int(3 * sigma)
    k = np.exp(-0.5 * (np.arange(-r, r + 1) / sigma) ** 2)
    k /= k.sum()
    return np.convolve(np.pad(x, r, mode="edge"), k, mode="valid")


def orient_path(rng, pts, sweep=1.0, pitch_amp=math.radians(12.0), heading_sigma=30.0):
    """Yaw follows the heading (smoothed over about a second, so a hand-held
    pan stays below a few degrees per frame through tight turns) plus a slow
    sweep; pitch stays within +-15 deg."""
    d = np.gradient(pts, axis=0)
    heading = _smooth(np.unwrap(np.arctan2(d[:, 1], d[:, 0])), heading_sigma)
    n = len(pts)
    k = np.arange(n)
    ph = rng.uniform(0, 2 * math.pi, size=2)
    yaw = heading + sweep * np.sin(2 * math.pi * k / 400.0 + ph[0])
    pitch = -math.radians(3.0) + pitch_amp * np.sin(2 * math.pi * k / 300.0 + ph[1])
    Rs, ts = [], []
    for i in range(n):
        R, t = look_pose(pts[i], yaw[i], pitch[i])
        Rs.append(R)
        ts.append(t)
    return np.array(Rs), np.array(ts)


# ----------------------------------------------------------------------------
# ray casting (torch float64; CPU or GPU)
# ----------------------------------------------------------------------------


def render(scene: Scene, R: np.ndarray, t: np.ndarray, intr: Intrinsics, device="cpu"):
    """Ray-cast exact z-depth and surface ids for a batch of poses.

    R: (F,3,3), t: (F,3).  Returns depth (F,H,W) float64 (0 = no hit),
    surface id (F,H,W) int64 and world hit points (F,H,W,3) float64.
    """
    dev = torch.device(device)
    f64 = torch.float64
    Rt = torch.as_tensor(np.asarray(R), dtype=f64, device=dev)
    tt = torch.as_tensor(np.asarray(t), dtype=f64, device=dev)
    H, W = intr.height, intr.width
    u = torch.arange(W, dtype=f64, device=dev)
    v = torch.arange(H, dtype=f64, device=dev)
    rc = torch.stack([((u[None, :] - intr.cx) / intr.fx).expand(H, W),
                      ((v[:, None] - intr.cy) / intr.fy).expand(H, W),
                      torch.ones(H, W, dtype=f64, device=dev)], dim=-1)  # (H,W,3)
    d = torch.einsum("fij,hwj->fhwi", Rt, rc)  # (F,H,W,3)
    o = tt[:, None, None, :]
    inf = torch.tensor(float("inf"), dtype=f64, device=dev)
    lo = torch.as_tensor(scene.room_lo, dtype=f64, device=dev)
    hi = torch.as_tensor(scene.room_hi, dtype=f64, device=dev)
    # room interior: the ray leaves the box through the nearest exit plane
    best = torch.full(d.shape[:-1], float("inf"), dtype=f64, device=dev)
    bid = torch.full(d.shape[:-1], -1, dtype=torch.int64, device=dev)
    for ax in range(3):
        da = d[..., ax]
        te = torch.where(da > 0, (hi[ax] - o[..., ax]) / da,
                         torch.where(da < 0, (lo[ax] - o[..., ax]) / da, inf))
        sid = torch.where(da > 0, 2 * ax + 1, 2 * ax)
        take = (te > 0) & (te < best)
        best = torch.where(take, te, best)
        bid = torch.where(take, sid, bid)
    base = 6
    for k, s in enumerate(scene.spheres):
        c = torch.as_tensor(s[:3], dtype=f64, device=dev)
        r = float(s[3])
        oc = o - c
        a = (d * d).sum(-1)
        b = (d * oc).sum(-1)
        cc = (oc * oc).sum(-1) - r * r
        disc = b * b - a * cc
        sq = torch.sqrt(torch.clamp(disc, min=0.0))
        te = (-b - sq) / a
        ok = (disc >= 0) & (te > 1e-9)
        take = ok & (te < best)
        best = torch.where(take, te, best)
        bid = torch.where(take, torch.full_like(bid, base + k), bid)
    base += len(scene.spheres)
    for k, bx in enumerate(scene.boxes):
        blo = torch.as_tensor(bx[:3], dtype=f64, device=dev)
        bhi = torch.as_tensor(bx[3:], dtype=f64, device=dev)
        with torch.no_grad():
            t1 = (blo - o) / d
            t2 = (bhi - o) / d
        tmin = torch.minimum(t1, t2).nan_to_num(nan=-inf).amax(-1)
        tmax = torch.maximum(t1, t2).nan_to_num(nan=inf).amin(-1)
        ok = (tmax >= tmin) & (tmin > 1e-9)
        take = ok & (tmin < best)
        best = torch.where(take, tmin, best)
        bid = torch.where(take, torch.full_like(bid, base + k), bid)
    hit = torch.isfinite(best)
    depth = torch.where(hit, best, torch.zeros_like(best))
    pts = o + depth[..., None] * d
    return depth, bid, pts


def shade(scene: Scene, sid: torch.Tensor, pts: torch.Tensor) -> torch.Tensor:
    """Procedural 3-D checker (cell size scene.checker) -> uint8 RGB."""
    cells = torch.floor(pts / scene.checker).to(torch.int64).sum(-1)
    parity = torch.remainder(cells, 2)
    cols = torch.as_tensor(scene.colors, device=sid.device).to(torch.int64)  # (P,2,3)
    idx = sid.clamp(min=0)
    rgb = cols[idx, parity]
    rgb = torch.where((sid >= 0)[..., None], rgb, torch.zeros_like(rgb))
    return rgb.to(torch.uint8)


def _gauss_blur_rgb(img: np.ndarray, sigma: float) -> np.ndarray:
    r = max(1, int(math.ceil(3 * sigma)))
    x = np.arange(-r, r + 1)
    k = np.exp(-0.5 * (x / sigma) ** 2)
    k /= k.sum()
    f = img.astype(np.float64)
    pad = np.pad(f, ((r, r), (0, 0), (0, 0)), mode="edge")
    f = sum(k[i] * pad[i:i + img.shape[0]] for i in range(2 * r + 1))
    pad = np.pad(f, ((0, 0), (r, r), (0, 0)), mode="edge")
    f = sum(k[i] * pad[:, i:i + img.shape[1]] for i in range(2 * r + 1))
    return np.clip(np.rint(f), 0, 255).astype(np.uint8)


def gaussian_blur(img: np.ndarray, sigma: float) -> np.ndarray:
    """Separable Gaussian blur of an (H,W,3) uint8 image (input degradation)."""
    return _gauss_blur_rgb(img, sigma)


# ----------------------------------------------------------------------------
# configurations
# ----------------------------------------------------------------------------


@dataclass
class VolumeSpec:
    voxel_size: float
    trunc: float
    n_buckets_log2: int
    color_mode: str  # "rgba8" | "f32"


@dataclass
class Workload:
    name: str
    intr: Intrinsics
    scene: Scene
    R: np.ndarray  # (N,3,3) frame poses, camera->world
    t: np.ndarray  # (N,3)
    kappa: int
    volume: VolumeSpec
    seed: int
    invalid_frac: float = 0.0
    blur_frac: float = 0.0
    extra: dict = field(default_factory=dict)

    @property
    def n_frames(self) -> int:
        return len(self.R)

    @property
    def n_keyframes(self) -> int:
        return self.n_frames // self.kappa


def _room_scene(rng, lo, hi, path, n_sph, n_box, clearance=0.5, walls_extra=()):
    sph, box = _place_primitives(rng, lo, hi, path, n_sph, n_box, walls_extra=walls_extra,
                                 clearance=clearance)
    allbox = np.concatenate([np.array(walls_extra, float).reshape(-1, 6), box], axis=0)
    colors = _colors(rng, 6 + len(sph) + len(allbox))
    return Scene(np.asarray(lo, float), np.asarray(hi, float), sph, allbox, colors)


def workload(cfg: int) -> Workload:
    """The five workloads: 1 tiny plain, 2 full plain, 3 differentiation,
    4 batched (large room), 5 corridor."""
    if cfg in (1, 3):
        rng = np.random.default_rng(1)
        lo, hi = np.zeros(3), np.array([4.0, 4.0, 3.0])
        n = 5 if cfg == 1 else 80
        path = room_path(rng, lo, hi, 600, step=0.01, margin=1.2)
        scene = _room_scene(rng, lo, hi, path, 3, 0)
        R, t = orient_path(rng, path)
        if cfg == 1:
            R, t = R[:n], t[:n]
            return Workload("tiny", QVGA, scene, R, t, 5, VolumeSpec(0.01, 0.04, 16, "rgba8"),
                            seed=1, invalid_frac=0.05)
        # 16 keyframes spread along the scan so that they overlap partially
        sel = np.arange(0, 600, 600 // 80)[:80]
        return Workload("diff", QVGA, scene, R[sel], t[sel], 5, VolumeSpec(0.01, 0.04, 16, "f32"),
                        seed=3, invalid_frac=0.05)
    if cfg == 2:
        rng = np.random.default_rng(2)
        lo, hi = np.zeros(3), np.array([4.0, 4.0, 3.0])
        path = room_path(rng, lo, hi, 600, step=0.01, margin=1.2)
        scene = _room_scene(rng, lo, hi, path, 3, 0)
        R, t = orient_path(rng, path)
        return Workload("full", VGA, scene, R, t, 60, VolumeSpec(0.005, 0.025, 20, "rgba8"),
                        seed=2, blur_frac=0.1)
    if cfg == 4:
        rng = np.random.default_rng(4)
        lo, hi = np.zeros(3), np.array([10.0, 10.0, 3.0])
        path = room_path(rng, lo, hi, 1000, step=0.01, margin=1.5)
        scene = _room_scene(rng, lo, hi, path, 20, 20)
        R, t = orient_path(rng, path)
        return Workload("batched", VGA, scene, R, t, 5, VolumeSpec(0.01, 0.04, 21, "rgba8"),
                        seed=4, blur_frac=0.1)
    if cfg == 5:
        rng = np.random.default_rng(5)
        lo, hi = np.zeros(3), np.array([40.0, 8.0, 3.0])
        walls = []
        for x in (10.0, 20.0, 30.0):
            walls.append([x - 0.05, 0.0, 0.0, x + 0.05, 3.4, 3.0])
            walls.append([x - 0.05, 4.6, 0.0, x + 0.05, 8.0, 3.0])
        path = corridor_path(rng, 3000)
        scene = _room_scene(rng, lo, hi, path, 75, 75, walls_extra=walls)
        R, t = orient_path(rng, path, sweep=0.8)
        return Workload("corridor", VGA, scene, R, t, 5, VolumeSpec(0.01, 0.04, 22, "rgba8"),
                        seed=5, blur_frac=0.1)
    raise ValueError(f"unknown workload {cfg}")


def scan(n_frames: int) -> Workload:
    """The first n_frames (at most 600) of the tiny workload's room scan, one
    frame per centimetre of path: the dense sequence keyframe strategies
    split into keyframes."""
    if not 1 <= n_frames <= 600:
        raise ValueError("scan length must be in [1, 600]")
    wl = workload(1)
    rng = np.random.default_rng(1)
    lo, hi = np.zeros(3), np.array([4.0, 4.0, 3.0])
    path = room_path(rng, lo, hi, 600, step=0.01, margin=1.2)
    _room_scene(rng, lo, hi, path, 3, 0)
    R, t = orient_path(rng, path)
    return Workload("scan", QVGA, wl.scene, R[:n_frames], t[:n_frames], 5, wl.volume, seed=1, invalid_frac=0.05)


def frames(wl: Workload, idx, device="cpu", chunk=64):
    """Render frames `idx` of a workload -> (depth float32 (F,H,W), rgb uint8 (F,H,W,3)).

    Noise, invalid pixels and blur are drawn from a generator seeded by
    (workload seed, frame index), so any subset renders identically.
    """
    idx = np.atleast_1d(np.asarray(idx))
    H, W = wl.intr.height, wl.intr.width
    depth_out = np.empty((len(idx), H, W), np.float32)
    rgb_out = np.empty((len(idx), H, W, 3), np.uint8)
    for s in range(0, len(idx), chunk):
        sub = idx[s:s + chunk]
        z, sid, pts = render(wl.scene, wl.R[sub], wl.t[sub], wl.intr, device)
        rgb = shade(wl.scene, sid, pts).cpu().numpy()
        z = z.cpu().numpy()
        for j, fi in enumerate(sub):
            rng = np.random.default_rng([wl.seed, int(fi)])
            zz = z[j]
            noisy = zz + noise_sigma(zz) * rng.standard_normal(zz.shape)
            bad = (zz <= 0) | (noisy < Z_MIN) | (noisy > Z_MAX)
            if wl.invalid_frac > 0:
                bad |= rng.random(zz.shape) < wl.invalid_frac
            depth_out[s + j] = np.where(bad, 0.0, noisy).astype(np.float32)
            im = rgb[j]
            if wl.blur_frac > 0 and rng.random() < wl.blur_frac:
                im = gaussian_blur(im, rng.uniform(0.5, 2.0))
            rgb_out[s + j] = im
    return depth_out, rgb_out


def keyframe_groups(wl: Workload):
    """KF_CONST grouping: consecutive runs of kappa frames (Sec. 4.2)."""
    k = wl.kappa
    return [np.arange(i * k, (i + 1) * k) for i in range(wl.n_keyframes)]


def column_strip_mask(valid: np.ndarray, frac: float, rng) -> np.ndarray:
    """Boolean (H,W) mask that zeroes a contiguous cyclic column strip so that
    about `frac` of the currently valid pixels remain (to within one column).
    A spatially coherent mask is used because i.i.d. dropout barely changes
    the set of voxel blocks a keyframe touches."""
    H, W = valid.shape
    per_col = valid.sum(0).astype(np.int64)
    total = int(per_col.sum())
    keep = np.ones((H, W), bool)
    if total == 0 or frac >= 1.0:
        return keep
    drop_target = total * (1.0 - frac)
    start = int(rng.integers(0, W))
    acc, width = 0, 0
    while width < W and acc + per_col[(start + width) % W] <= drop_target:
        acc += per_col[(start + width) % W]
        width += 1
    cols = (start + np.arange(width)) % W
    keep[:, cols] = False
    return keep


def strip_masks(ref_depth, seed, lo=0.4, hi=1.0):
    """Uneven keyframe sizes: valid-pixel fractions f_k ~ U(lo, hi) and, per
    keyframe, the column-strip mask that keeps about f_k of its range-valid
    pixels (those of its reference frame with a depth).  Depends on the
    rendered frames only, so both the GPU path and the oracle apply the same
    masks to the keyframes they fuse themselves."""
    rng = np.random.default_rng(seed)
    fracs = rng.uniform(lo, hi, len(ref_depth))
    return fracs, [column_strip_mask(np.asarray(ref_depth[k]) > 0, fracs[k], rng) for k in range(len(ref_depth))]


def perturb_all(R, t, sigma_rho, sigma_phi_deg, seed):
    """T' = Exp(delta) T with delta ~ N(0, sigma) per axis (world frame)."""
    rng = np.random.default_rng(seed)
    Rn, tn = np.empty_like(R), np.empty_like(t)
    for i in range(len(R)):
        xi = np.concatenate([rng.normal(0, sigma_rho, 3), rng.normal(0, math.radians(sigma_phi_deg), 3)])
        dR, dt = se3_exp(xi)
        Rn[i], tn[i] = compose(dR, dt, R[i], t[i])
    return Rn, tn


def perturb_fixed(R, t, rho, phi_deg, seed):
    """T' = Exp(delta) T with |rho| = rho and |phi| = phi_deg in seeded random directions."""
    rng = np.random.default_rng(seed)
    Rn, tn = np.empty_like(R), np.empty_like(t)
    for i in range(len(R)):
        a = rng.standard_normal(3)
        b = rng.standard_normal(3)
        xi = np.concatenate([rho * a / np.linalg.norm(a), math.radians(phi_deg) * b / np.linalg.norm(b)])
        dR, dt = se3_exp(xi)
        Rn[i], tn[i] = compose(dR, dt, R[i], t[i])
    return Rn, tn


def loop_closure_updates(R, t, n_updates, seed, n_range=(50, 300), rho_max=0.10, phi_max_deg=3.0):
    """Successive corrections that ramp linearly along the newest n_u keyframes
    from zero to (rho_max_u, phi_max_u) at the newest, like a loop closure
    spreading its error.  Returns a list of (R', t') pose arrays, each applied
    to the poses produced by the previous update."""
    rng = np.random.default_rng(seed)
    K = len(R)
    out = []
    Rc, tc = R.copy(), t.copy()
    for _ in range(n_updates):
        n_u = int(rng.integers(n_range[0], n_range[1] + 1))
        n_u = min(n_u, K)
        rmax = rng.uniform(0, rho_max)
        pmax = math.radians(rng.uniform(0, phi_max_deg))
        a = rng.standard_normal(3)
        b = rng.standard_normal(3)
        a /= np.linalg.norm(a)
        b /= np.linalg.norm(b)
        Rn, tn = Rc.copy(), tc.copy()
        for j in range(n_u):
            i = K - n_u + j
            s = (j + 1) / n_u
            dR, dt = se3_exp(np.concatenate([s * rmax * a, s * pmax * b]))
            Rn[i], tn[i] = compose(dR, dt, Rc[i], tc[i])
        out.append((Rn, tn))
        Rc, tc = Rn, tn
    return out


# ----------------------------------------------------------------------------
# analytic signed distance of a scene (loss target for the adjoint workload)
# ----------------------------------------------------------------------------


def _box_face_samples(rng, lo, hi, n):
    """n points uniform on the surface of the box [lo, hi] (area-weighted faces)."""
    ext = hi - lo
    areas = np.array([ext[1] * ext[2], ext[0] * ext[2], ext[0] * ext[1]] * 2)
    face = rng.choice(6, n, p=areas / areas.sum())
    u = rng.random((n, 3))
    pts = lo + u * ext
    axis = face % 3
    pts[np.arange(n), axis] = np.where(face < 3, lo[axis], hi[axis])
    return pts


def surface_points(scene: Scene, n: int, seed: int) -> np.ndarray:
    """About n points uniform over the scene's visible geometry (the room's
    inner walls and the primitives' surfaces, area-weighted), keeping those
    on the boundary of free space: a stand-in for a reference cloud sampled
    from the ground-truth mesh."""
    rng = np.random.default_rng(seed)
    lo, hi = scene.room_lo, scene.room_hi
    ext = hi - lo
    parts = [("room", 2 * (ext[0] * ext[1] + ext[0] * ext[2] + ext[1] * ext[2]), None)]
    parts += [("sph", 4 * np.pi * sp[3] ** 2, sp) for sp in scene.spheres]
    parts += [("box", 2 * ((b[3] - b[0]) * (b[4] - b[1]) + (b[3] - b[0]) * (b[5] - b[2]) + (b[4] - b[1]) * (b[5] - b[2])),
               b) for b in scene.boxes]
    area = np.array([p[1] for p in parts])
    counts = rng.multinomial(n, area / area.sum())
    out = []
    for (kind, _, prm), k in zip(parts, counts):
        if k == 0:
            continue
        if kind == "room":
            out.append(_box_face_samples(rng, lo, hi, k))
        elif kind == "sph":
            v = rng.normal(size=(k, 3))
            out.append(prm[:3] + prm[3] * v / np.linalg.norm(v, axis=1, keepdims=True))
        else:
            out.append(_box_face_samples(rng, prm[:3], prm[3:], k))
    pts = np.concatenate(out)
    keep = np.abs(scene_sdf(scene, pts)) < 1e-6
    return pts[keep].astype(np.float32)


def scene_sdf(scene: Scene, x: np.ndarray) -> np.ndarray:
    """Signed Euclidean distance, positive in free space, for points (N,3)."""
    x = np.asarray(x, float)
    d = np.minimum(x - scene.room_lo, scene.room_hi - x).min(-1)
    for s in scene.spheres:
        d = np.minimum(d, np.linalg.norm(x - s[:3], axis=-1) - s[3])
    for b in scene.boxes:
        lo, hi = b[:3], b[3:]
        c, h = 0.5 * (lo + hi), 0.5 * (hi - lo)
        q = np.abs(x - c) - h
        out = np.linalg.norm(np.maximum(q, 0.0), axis=-1)
        inside = np.minimum(q.max(-1), 0.0)
        d = np.minimum(d, out + inside)
    return d
