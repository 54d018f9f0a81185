#!/usr/bin/env python3
"""Benchmark of the batched surface correction on one MI355X.

Workload (the batched re-integration configuration): a 10 x 10 x 3 m room
with 40 seeded boxes and spheres, 1000 synthetic 640x480 RGB-D frames fused
5 per keyframe into 200 keyframes (kf_fuse), each keyframe cut to a seeded
valid-pixel fraction in [0.4, 1.0] by a contiguous column strip, integrated
into a voxel-hashed TSDF (1 cm voxels, 4 cm truncation, 2^21 buckets, FP64
TSDF + RGBA8 colour + FP32 weight).  A pose-graph update moves all 200 poses
by N(0, 3 cm / 1.5 deg); one step re-integrates every changed keyframe in
order of pose change (de-integrate at the integration pose, re-integrate at
the new pose) with reintegrate_batch.  Steps alternate between the two pose
sets, so every step has the same amount of work.

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "keyframes re-integrated/sec (de+re) and voxel updates/sec; % of HBM peak"
HBM_PEAK_GBS = 8000.0
VOXEL_BYTES = 12  # the method's voxel: FP32 D + FP32 W + RGBA8 colour (algorithmic bytes)
STORAGE_VOXEL_BYTES = 16  # the voxel as stored here: FP64 D + FP32 W + RGBA8 colour
KF_PIXEL_BYTES = 12  # keyframe depth + weight + RGBA8 colour
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "voxel_pass_traffic_batched_reintegration.json")
KERNEL_SOURCES = ["paper_1709_03763_amd/csrc/batch.hip", "paper_1709_03763_amd/csrc/kernels.hpp",
                  "paper_1709_03763_amd/csrc/common.hpp"]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_model():
    """The host CPU's model name (as lscpu reports it), from /proc/cpuinfo."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def source_digest():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def render_groups(torch, synth, wl, groups, tag):
    """Frames of keyframe groups rendered on the device, in chunks of 20
    groups: list of (depth (kappa,H,W) f32, rgb (kappa,H,W,3) u8, frame
    indices) on the host."""
    out = []
    t0 = time.time()
    k = wl.kappa
    for g0 in range(0, len(groups), 20):
        gs = groups[g0:g0 + 20]
        z, rgb = synth.frames(wl, np.concatenate(gs), device="cuda")
        for j, g in enumerate(gs):
            out.append((z[j * k:(j + 1) * k], rgb[j * k:(j + 1) * k], g))
        log(f"  {tag}: rendered {min(g0 + 20, len(groups))}/{len(groups)} keyframe groups ({time.time() - t0:.0f} s)")
    return out


def gpu_keyframes(torch, scsurf, wl, frames, masks=None):
    """Keyframes fused on the GPU (kf_fuse), each cut by its valid-pixel mask
    when given; returns (keyframes, seconds spent in kf_fuse)."""
    dev = torch.device("cuda")
    dz = [torch.from_numpy(f[0]).to(dev) for f in frames]
    dc = [torch.from_numpy(f[1]).to(dev) for f in frames]
    # one untimed pass first (code loading, the library's scratch, the GPU's
    # clocks leaving idle): the first pass of a fresh process ran about 4x
    # slower than the next ones
    for k, f in enumerate(frames):
        scsurf.kf_fuse(dz[k], dc[k], wl.R[f[2]], wl.t[f[2]], wl.intr)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    kfs = [scsurf.kf_fuse(dz[k], dc[k], wl.R[f[2]], wl.t[f[2]], wl.intr) for k, f in enumerate(frames)]
    torch.cuda.synchronize()
    fuse_s = time.perf_counter() - t0
    if masks is not None:
        for kf, m in zip(kfs, masks):
            keep = torch.from_numpy(m).to(dev)
            kf.depth.mul_(keep)
            kf.weight.mul_(keep)
            kf.color.mul_(keep[..., None].to(torch.uint8))
    return kfs, fuse_s


def oracle_keyframes(oracle, wl, frames, idx, masks=None):
    """The oracle's own fusion of the frame groups `idx` (a thread pool over
    keyframes), cut by the same masks: the CPU-baseline legs' keyframes."""
    from concurrent.futures import ThreadPoolExecutor

    def one(k):
        z, rgb, g = frames[k]
        kf = oracle.kf_fuse(z, rgb, wl.intr, wl.R[g], wl.t[g])
        out = {"depth": kf["depth"], "weight": kf["weight"], "color": kf["color"]}
        if masks is not None:
            m = masks[k]
            out = {"depth": np.where(m, out["depth"], 0).astype(np.float32),
                   "weight": np.where(m, out["weight"], 0).astype(np.float32),
                   "color": np.where(m[..., None], out["color"], 0).astype(np.uint8)}
        return out

    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        return dict(zip(idx, ex.map(one, idx)))


def build_workload(torch, scsurf, synth, n_kf, seed, pack=True):
    wl = synth.workload(4)
    groups = synth.keyframe_groups(wl)[:n_kf]
    log(f"rendering {n_kf * wl.kappa} frames at {wl.intr.width}x{wl.intr.height}")
    frames = render_groups(torch, synth, wl, groups, "batched workload")
    # uneven valid-pixel fractions: column strips fixed by each group's reference frame
    fracs, masks = synth.strip_masks([f[0][0] for f in frames], seed)
    kfs, fuse_s = gpu_keyframes(torch, scsurf, wl, frames, masks)
    R = np.array([wl.R[g[0]] for g in groups])
    t = np.array([wl.t[g[0]] for g in groups])
    pack_s = None
    if pack:
        # the interleaved copy the voxel passes gather from, made once per keyframe
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        kfs = [scsurf.keyframe_pack(k) for k in kfs]
        torch.cuda.synchronize()
        pack_s = time.perf_counter() - t0
    return wl, kfs, R, t, fuse_s, fracs, pack_s, frames, masks


def cpu_baseline(oracle, kfs_np, intr, A, B, sample):
    """The oracle re-integrating a sample of keyframes (FP64, host cores)."""
    vol = oracle.Volume(0.01, 0.04)
    for k in sample:
        vol.integrate(kfs_np[k], intr, A[0][k], A[1][k])
    t0 = time.perf_counter()
    for k in sample:
        assert vol.deintegrate(kfs_np[k], intr, A[0][k], A[1][k]) == oracle.OK
    for k in sample:
        assert vol.integrate(kfs_np[k], intr, B[0][k], B[1][k]) == oracle.OK
    dt = time.perf_counter() - t0
    return len(sample) / dt, dt


def adjoint_stage(torch, scsurf, synth):
    """Forward + backward of integration on the differentiation workload
    (16 keyframes at 320x240, F32 colour), timed."""
    from paper_1709_03763_amd import autograd as sca

    wl = synth.workload(3)
    groups = synth.keyframe_groups(wl)
    z, rgb = synth.frames(wl, np.arange(wl.n_frames), device="cuda")
    dev = torch.device("cuda")
    kfs = [scsurf.kf_fuse(torch.from_numpy(z[g]).to(dev), torch.from_numpy(rgb[g]).to(dev), wl.R[g], wl.t[g], wl.intr)
           for g in groups]
    depth = torch.stack([k.depth for k in kfs]).requires_grad_(True)
    color = torch.stack([k.color[..., :3].float() / 255.0 for k in kfs]).requires_grad_(True)
    weight = torch.stack([k.weight for k in kfs])
    xi = torch.zeros((len(kfs), 6), device=dev, requires_grad=True)
    R = np.array([wl.R[g[0]] for g in groups])
    t = np.array([wl.t[g[0]] for g in groups])
    vol = scsurf.Volume(0.01, 0.04, 1 << 17, 1 << 16, color_mode=scsurf.COLOR_F32)
    times = []
    for rep in range(4):
        for p in (depth, color, xi):
            p.grad = None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        D, C, W = sca.integrate(depth, color, weight, xi, vol, wl.intr, R, t)
        loss = ((D * (W > 0)) ** 2).sum() + 0.1 * ((C - 0.5) ** 2).sum()
        loss.backward()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    vol.close()
    return float(np.median(times[1:]) * 1e3)


def backward_full_stage(torch, vol, kset, wl, A, reps=4):
    """Backward of integration at the benchmark's size: all 200 keyframes at
    640x480 as integrated at their first poses in the benchmark volume, with
    a seeded upstream dL/dD, gradients for depth and the se(3) poses (RGBA8
    colour carries none).  Median wall-clock of the call, synchronised."""
    n_blocks, _ = vol.query()
    H, Wd = wl.intr.height, wl.intr.width
    g = torch.Generator(device="cuda").manual_seed(7)
    grad_D = torch.randn((n_blocks, 512), device="cuda", generator=g)
    grad_depth = torch.zeros((len(kset), H, Wd), device="cuda")
    grad_xi = torch.zeros((len(kset), 6), device="cuda")
    times = []
    for _ in range(reps):
        grad_depth.zero_()
        grad_xi.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        vol.integrate_backward(kset, wl.intr, A[0], A[1], grad_D, None, grad_depth, None, grad_xi)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    return float(np.median(times[1:]) * 1e3)


def kernel_variant(sched):
    """Name of the voxel-pass kernel a schedule (vpl, waves_per_wg, wgs_per_cu,
    compact) launches."""
    vpl, _, _, compact = sched
    if compact == 4:
        return "batch_ring_kernel<RGBA8,packed>"
    if compact == 3:
        return "batch_pipe_kernel<RGBA8>"
    if compact:
        return f"batch_compact_kernel<RGBA8,{8 if compact == 1 else 4}>"
    return "batch_main_wave_kernel<RGBA8>" if vpl == 8 else f"batch_main_group_kernel<RGBA8,{vpl}>"


def online_stage(torch, scsurf, synth, n_frames=1000, every=20, m=20, stream_radius=None, pool_blocks=None,
                 integrate_every=1):
    """The online loop on the corridor workload: frames fused into keyframes of
    five, each keyframe integrated at its drifting estimate, a pose-graph
    update every `every` keyframes re-integrating the Eq. 3 window of m,
    then the final pass.  Frames are rendered to the device first; the loop
    is timed.  With a stream radius the volume streams (a pool of
    `pool_blocks`, batches of 4 operations) and the bytes moved between the
    GPU and the host are reported, in all and per pose-graph update.  With
    integrate_every > 1 finished keyframes are integrated that many at a
    time by the batched integration (and before each update)."""
    from paper_1709_03763_amd import online

    wl = synth.workload(5)
    kappa = wl.kappa
    groups = synth.keyframe_groups(wl)[: n_frames // kappa]
    first = np.array([g[0] for g in groups])
    Rk, tk = wl.R[first], wl.t[first]
    drift = online.drifting_estimates(Rk, tk, seed=55)
    Re, te = online.corrected(Rk, tk, drift, 1.0)
    idx = np.concatenate(groups)
    zs, cs = [], []
    for s0 in range(0, len(idx), 100):
        z, rgb = synth.frames(wl, idx[s0:s0 + 100], device="cuda")
        zs.append(torch.from_numpy(z).cuda())
        cs.append(torch.from_numpy(rgb).cuda())
    Z, C = torch.cat(zs), torch.cat(cs)
    poses = []
    for k, g in enumerate(groups):
        A = Re[k] @ Rk[k].T
        poses += [(A @ wl.R[f], A @ (wl.t[f] - tk[k]) + te[k]) for f in g]
    updates = {n: online.corrected(Rk[:n], tk[:n], drift[:n], 0.5 ** (n // every))
               for n in range(every, len(groups) + 1, every)}
    streamed = stream_radius is not None
    pool = pool_blocks if streamed else 1 << 21
    vol = scsurf.Volume(wl.volume.voxel_size, wl.volume.trunc, 1 << 22, pool, scsurf.COLOR_RGBA8,
                        max_batch_ops=4 if streamed else 512)
    sess = online.OnlineSession(vol, wl.intr, wl.kappa, m, stream_radius=stream_radius,
                                integrate_every=integrate_every)
    per_update = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for f in range(len(idx)):
        k = sess.add_frame(Z[f], C[f], *poses[f])
        if k is not None and (k + 1) in updates:
            before = vol.stream_stats() if streamed else None
            sess.pose_update(*updates[k + 1])
            if streamed:
                after = vol.stream_stats()
                per_update.append(after[4] - before[4] + after[5] - before[5])
    final = sess.final_pass()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    n_blocks = vol.check_error()
    out = {"frames": len(idx), "keyframes": len(groups), "updates": len(updates), "m": m,
           "final_pass_keyframes": len(final), "reintegrated_keyframes": sess.reintegrated, "blocks": n_blocks,
           "seconds": round(dt, 4), "frames_per_s": round(len(idx) / dt, 1), "integrate_every": integrate_every}
    if streamed:
        st = vol.stream_stats()
        out.update({"pool_blocks": pool, "stream_radius_m": stream_radius, "device_blocks": st[0],
                    "host_blocks": st[1], "streamed_out_bytes": st[4], "streamed_in_bytes": st[5],
                    "streamed_bytes_per_update_mean": int(np.mean(per_update)) if per_update else 0})
    vol.close()
    return out


def mesh_stage(torch, scsurf, surface, synth, vol, wl):
    """Marching Cubes of the benchmark volume, its distinct vertices, and CORR
    against a dense reference cloud of the scene (wall-clock of each call,
    which synchronises)."""
    n_blocks, _ = vol.query()

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return r, time.perf_counter() - t0

    vol.mesh()  # warm-up (table upload)
    (xyz, keys), mesh_s = timed(vol.mesh)
    verts, vert_s = timed(lambda: surface.mesh_vertices(xyz, keys))
    ref = torch.from_numpy(synth.surface_points(wl.scene, 4_000_000, 7)).cuda()
    corr, corr_s = timed(lambda: surface.corr(verts, ref, 0.05))
    n_tri = int(xyz.shape[0])
    # one 9^3 halo of D (8 B) and W (4 B) read per block, triangles written (36 B positions + 48 B keys);
    # the call meshes twice (count, then fill)
    mesh_bytes = n_blocks * 729 * 12 * 2 + n_tri * (36 + 48)
    return {"blocks": int(n_blocks), "triangles": n_tri, "vertices": int(verts.shape[0]),
            "mesh_ms": round(mesh_s * 1e3, 3), "triangles_per_s": round(n_tri / mesh_s, 1),
            "mesh_hbm_frac": round(mesh_bytes / mesh_s / 1e9 / HBM_PEAK_GBS, 5),
            "vertices_ms": round(vert_s * 1e3, 3), "reference_points": int(ref.shape[0]),
            "corr_ms": round(corr_s * 1e3, 3), "corr_mm": round(corr * 1e3, 4)}


def surface_stage(torch, scsurf, surface, online, synth, log):
    """Synthetic analogue of the keyframe-strategy study of Sec. 5 (Fig. 5):
    the 4 x 4 x 3 m room scanned in 600 frames at 640x480 with ground-truth
    poses, fused into keyframes by each strategy and integrated (5 mm voxels,
    2.5 cm truncation); CORR of the mesh against a dense cloud on the scene's
    surfaces, COMPL of the per-frame reconstruction's vertices (kappa = 1)
    against the mesh, both capped at 5 cm."""
    wl = synth.workload(2)
    n = wl.n_frames
    log(f"surface study: rendering {n} frames")
    z, rgb = synth.frames(wl, np.arange(n), device="cuda")
    zt = [torch.from_numpy(z[f]).cuda() for f in range(n)]
    ct = [torch.from_numpy(rgb[f]).cuda() for f in range(n)]
    ref = torch.from_numpy(synth.surface_points(wl.scene, 8_000_000, 5)).cuda()
    runs = [("const", {"kappa": k}) for k in (1, 2, 5, 10, 20, 60)]
    runs += [("dist", {"max_trans": a, "max_rot": np.radians(b)}) for a, b in ((0.05, 5.0), (0.15, 10.0), (0.4, 30.0))]
    runs += [("overlap", {"min_overlap": o}) for o in (0.9, 0.75, 0.5)]
    out, ref_vertices = [], None
    for strategy, kw in runs:
        vol = scsurf.Volume(wl.volume.voxel_size, wl.volume.trunc, 1 << 21, 1 << 20)
        kappa = kw.pop("kappa", 5)
        sess = online.OnlineSession(vol, wl.intr, kappa, 1, strategy=strategy, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for f in range(n):
            sess.add_frame(zt[f], ct[f], wl.R[f], wl.t[f])
        sess.flush()
        torch.cuda.synchronize()
        fuse_s = time.perf_counter() - t0
        vol.check_error()
        xyz, keys = vol.mesh()
        v = surface.mesh_vertices(xyz, keys)
        if ref_vertices is None:
            ref_vertices = v.clone()  # the first run is kappa = 1: the reference of COMPL
        rec = {"strategy": strategy, **{k: (round(float(x), 4) if isinstance(x, float) else x) for k, x in kw.items()},
               "kappa": kappa if strategy == "const" else None, "keyframes": sess.n_keyframes,
               "mean_kappa": round(n / sess.n_keyframes, 2), "fuse_integrate_s": round(fuse_s, 3),
               "triangles": int(xyz.shape[0]), "corr_mm": round(surface.corr(v, ref, 0.05) * 1e3, 3),
               "compl_mm": round(surface.compl(ref_vertices, v, 0.05) * 1e3, 3)}
        log(f"surface study: {rec}")
        out.append(rec)
        vol.close()
    return out


def _rgba(rgb):
    col = np.zeros(rgb.shape[:2] + (4,), np.uint8)
    col[..., :3] = rgb
    return col


def _update_rates(torch, scsurf, vol, kset, intr, A, B, m, mode, fn, steps):
    """(keyframes re-integrated/s, updates/s, voxel updates per update as the
    volume's counters report them) of `steps` alternating updates
    A -> B -> A ... (two untimed updates first; the volume ends at A)."""
    state = [A, B]

    def step():
        order, _ = fn(kset, intr, state[0], state[1], m, mode)
        state[0], state[1] = state[1], state[0]
        return order

    steps += steps & 1  # an even count leaves the keyframes integrated at A again
    step()
    step()
    torch.cuda.synchronize()
    s0 = vol.stats()
    t0 = time.perf_counter()
    n = 0
    for _ in range(steps):
        n += len(step())
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    upd = vol.stats()[2] - s0[2]
    vol.check_error()
    return n / dt, steps / dt, upd / steps


def _oracle_rate(oracle, kfs, intr, A, B, sample, threads, s, mu):
    """Oracle keyframes re-integrated/s (de at A, re at B) over `sample`."""
    oracle.set_threads(threads)
    vol = oracle.Volume(s, mu)
    for k in sample:
        vol.integrate(kfs[k], intr, A[0][k], A[1][k])
    t0 = time.perf_counter()
    for k in sample:
        assert vol.deintegrate(kfs[k], intr, A[0][k], A[1][k]) == oracle.OK
    for k in sample:
        assert vol.integrate(kfs[k], intr, B[0][k], B[1][k]) == oracle.OK
    return len(sample) / (time.perf_counter() - t0)


def _pass_rates(vol, steps_ms_fn):
    """Runs `steps_ms_fn()` with the voxel-pass events and counters on and
    returns (its return value, total voxel-pass ms, counter deltas)."""
    s0 = vol.stats()
    vol.batch_timing(4096)
    r = steps_ms_fn()
    ms = vol.batch_timing_read()
    vol.batch_timing(0)
    s1 = vol.stats()
    return r, float(np.sum(ms)), [b - a for a, b in zip(s0, s1)]


def configs_stage(torch, scsurf, synth, oracle, log):
    """Rates on the other workloads, with keyframes fused at each one's kappa:
    plain tiny (5 frames at 320x240 -> 1 keyframe, a 1 cm / 0.5 deg
    perturbation), plain full resolution (600 frames at 640x480 -> 10
    keyframes of 60, 5 mm voxels, N(0, 2 cm / 1 deg)), and the corridor (3000
    frames -> 600 keyframes of 5, 20 loop-closure updates of the Eq. 3 window
    of 100).  GPU keyframes come from kf_fuse, the oracle's from its own
    fusion of the same frames.  GPU: plain per-keyframe and batched paths,
    with the batched voxel pass's algorithmic fraction of HBM peak; oracle:
    FP64 on 1 and on all host threads."""
    n_all = oracle.threads()
    out = {}
    for cfg in (1, 2):
        wl = synth.workload(cfg)
        groups = synth.keyframe_groups(wl)
        frames = render_groups(torch, synth, wl, groups, f"config {cfg}")
        kfs, _ = gpu_keyframes(torch, scsurf, wl, frames)
        first = np.array([g[0] for g in groups])
        A = (wl.R[first], wl.t[first])
        B = synth.perturb_all(A[0], A[1], 0.01, 0.5, 1) if cfg == 1 else synth.perturb_all(A[0], A[1], 0.02, 1.0, 2)
        s, mu = wl.volume.voxel_size, wl.volume.trunc
        nb = 1 << (16 if cfg == 1 else 20)
        vol = scsurf.Volume(s, mu, nb, nb // 2, scsurf.COLOR_RGBA8, max_batch_ops=64)
        kfs = [scsurf.keyframe_pack(k) for k in kfs]
        for k in range(len(kfs)):
            vol.integrate(kfs[k], wl.intr, A[0][k], A[1][k])
        kset = scsurf.KeyframeSet(kfs)
        n = len(kfs)
        steps = 200 if cfg == 1 else 20
        plain = _update_rates(torch, scsurf, vol, kfs, wl.intr, A, B, n, scsurf.SEL_ALL_ORDERED,
                              vol.reintegrate_plain, steps)
        (batch, pass_ms, d) = _pass_rates(vol, lambda: _update_rates(torch, scsurf, vol, kset, wl.intr, A, B, n,
                                                                      scsurf.SEL_ALL_ORDERED, vol.reintegrate_batch,
                                                                      steps))
        H, Wd = wl.intr.height, wl.intr.width
        n_pass = steps + (steps & 1) + 2  # the timed updates and the two untimed ones before them
        alg = d[3] * 512 * 2 * VOXEL_BYTES + n_pass * 2 * n * H * Wd * KF_PIXEL_BYTES
        vol.close()
        sample = list(range(n))
        okfs = oracle_keyframes(oracle, wl, frames, sample)
        o1 = _oracle_rate(oracle, okfs, wl.intr, A, B, sample[:3], 1, s, mu)
        on = _oracle_rate(oracle, okfs, wl.intr, A, B, sample, n_all, s, mu)
        per_update = batch[2]  # the batched pass counts its voxel updates; the plain path does the same work
        out[f"config{cfg}"] = {"keyframes": n, "kappa": wl.kappa, "voxel_updates_per_update": int(per_update),
                               "plain_kf_per_s": round(plain[0], 1),
                               "plain_voxel_updates_per_s": round(plain[1] * per_update, 1),
                               "batched_kf_per_s": round(batch[0], 1),
                               "batched_voxel_updates_per_s": round(batch[1] * per_update, 1),
                               "batched_pass_hbm_frac": round(alg / (pass_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                               "oracle_1core_kf_per_s": round(o1, 3), f"oracle_{n_all}core_kf_per_s": round(on, 3)}
        log(f"config {cfg}: {out[f'config{cfg}']}")
    # corridor
    wl = synth.workload(5)
    groups = synth.keyframe_groups(wl)[:600]
    log("corridor: rendering 3000 frames")
    frames = render_groups(torch, synth, wl, groups, "corridor")
    kfs, _ = gpu_keyframes(torch, scsurf, wl, frames)
    kfs = [scsurf.keyframe_pack(k) for k in kfs]
    first = np.array([g[0] for g in groups])
    R, t = wl.R[first], wl.t[first]
    updates = list(synth.loop_closure_updates(R, t, 20, 5))
    H, Wd = wl.intr.height, wl.intr.width
    res = {}
    for path in ("plain", "batched"):
        vol = scsurf.Volume(wl.volume.voxel_size, wl.volume.trunc, 1 << 22, 1 << 21, scsurf.COLOR_RGBA8,
                            max_batch_ops=256)
        for k in range(len(kfs)):
            vol.integrate(kfs[k], wl.intr, R[k], t[k])
        kset = scsurf.KeyframeSet(kfs)
        fn = vol.reintegrate_plain if path == "plain" else vol.reintegrate_batch
        Ti = (R.copy(), t.copy())
        fn(kset, wl.intr, Ti, updates[0], 100, scsurf.SEL_EQ3)  # warm-up, then back
        fn(kset, wl.intr, updates[0], Ti, 100, scsurf.SEL_EQ3)

        def run():
            Tc = Ti
            n = 0
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for Tn in updates:
                order, Tc = fn(kset, wl.intr, Tc, Tn, 100, scsurf.SEL_EQ3)
                n += len(order)
            torch.cuda.synchronize()
            return n, time.perf_counter() - t0

        (n, dt), pass_ms, d = _pass_rates(vol, run)
        nb = vol.check_error()
        vol.close()
        res[path] = {"kf_per_s": n / dt, "reintegrated": n, "blocks": nb, "updates_per_s": d[2] / dt}
        if path == "batched":
            alg = d[3] * 512 * 2 * VOXEL_BYTES + 2 * n * H * Wd * KF_PIXEL_BYTES
            res[path]["hbm_frac"] = alg / (pass_ms / 1e3) / 1e9 / HBM_PEAK_GBS
        log(f"corridor {path}: {res[path]}")
    sample = list(range(0, 600, 60))
    okfs = oracle_keyframes(oracle, wl, frames, sample)
    A = (R, t)
    B = synth.perturb_all(R, t, 0.05, 1.5, 6)
    o1 = _oracle_rate(oracle, okfs, wl.intr, A, B, sample[:3], 1, wl.volume.voxel_size, wl.volume.trunc)
    on = _oracle_rate(oracle, okfs, wl.intr, A, B, sample, n_all, wl.volume.voxel_size, wl.volume.trunc)
    out["config5"] = {"keyframes": 600, "kappa": wl.kappa, "updates": len(updates),
                      "reintegrated": res["batched"]["reintegrated"], "blocks": int(res["batched"]["blocks"]),
                      "plain_kf_per_s": round(res["plain"]["kf_per_s"], 1),
                      "batched_kf_per_s": round(res["batched"]["kf_per_s"], 1),
                      "batched_speedup": round(res["batched"]["kf_per_s"] / res["plain"]["kf_per_s"], 2),
                      "batched_voxel_updates_per_s": round(res["batched"]["updates_per_s"], 1),
                      "batched_pass_hbm_frac": round(res["batched"]["hbm_frac"], 4),
                      "oracle_1core_kf_per_s": round(o1, 3), f"oracle_{n_all}core_kf_per_s": round(on, 3)}
    log(f"config 5: {out['config5']}")
    oracle.set_threads(n_all)
    return out


def traffic_from_profile(digest, variant):
    """HBM bytes per launch of the voxel pass from the committed rocprofv3
    counter summary, if it was taken from the current kernel sources and the
    same kernel variant."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("source_digest") != digest or rec.get("kernel") != variant:
        return None
    return rec.get("bytes_per_launch")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--keyframes", type=int, default=200)
    ap.add_argument("--plain-steps", type=int, default=2)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--sweep", action="store_true",
                    help="also time every voxel-pass schedule (stderr) before the timed steps")
    ap.add_argument("--schedule", type=str, default="",
                    help="fixed voxel-pass schedule vpl,waves_per_wg,wgs_per_cu,compact (skips the autotuner)")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-online", action="store_true")
    ap.add_argument("--no-pack", action="store_true",
                    help="keyframes without the interleaved copy (three gathers per voxel test)")
    ap.add_argument("--cpu-sample", type=int, default=200,
                    help="keyframes the oracle re-integrates for the CPU baseline (all 200 by default)")
    ap.add_argument("--no-mesh", action="store_true")
    ap.add_argument("--configs", action="store_true",
                    help="also time the plain tiny, plain full-resolution and corridor workloads (GPU and oracle)")
    ap.add_argument("--surface", action="store_true",
                    help="also run the keyframe-strategy surface study (CORR / COMPL per strategy)")
    ap.add_argument("--calib-copy-gib", type=float, default=0.0,
                    help="also run a device copy of this size (for counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the surface-correction path runs on a single MI355X "
              "(sharding across GPUs is designed, not built); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import oracle
    from paper_1709_03763_amd import online, scsurf, surface, synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    torch.cuda.set_device(0)
    scsurf.lib()
    n_kf = args.keyframes
    wl, kfs, R, t, fuse_s, fracs, pack_s, frames, masks = build_workload(torch, scsurf, synth, n_kf, seed=4,
                                                                        pack=not args.no_pack)
    H, Wd = wl.intr.height, wl.intr.width
    log(f"fused {n_kf} keyframes in {fuse_s * 1e3:.1f} ms")
    A = (R, t)
    B = synth.perturb_all(R, t, 0.03, 1.5, 4)
    vol = scsurf.Volume(0.01, 0.04, 1 << 21, 1 << 21, scsurf.COLOR_RGBA8, max_batch_ops=512)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(n_kf):
        vol.integrate(kfs[k], wl.intr, R[k], t[k])
    torch.cuda.synchronize()
    integrate_s = time.perf_counter() - t0
    n_blocks = vol.check_error()
    log(f"integrated {n_kf} keyframes in {integrate_s * 1e3:.1f} ms; {n_blocks} blocks")
    # the same 200 integrations in one batched call, into a fresh volume (a
    # first call untimed), checked equal to the sequential volume's blocks
    vb = scsurf.Volume(0.01, 0.04, 1 << 21, 1 << 21, scsurf.COLOR_RGBA8, max_batch_ops=512)
    vb.integrate_batch(kfs, wl.intr, R, t)
    vb.reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    vb.integrate_batch(kfs, wl.intr, R, t)
    torch.cuda.synchronize()
    integrate_batch_s = time.perf_counter() - t0
    if vb.check_error() != n_blocks:
        raise RuntimeError("batched integration allocated a different block count")
    vb.close()
    log(f"integrated {n_kf} keyframes in one batched call in {integrate_batch_s * 1e3:.2f} ms")
    mode = scsurf.SEL_ALL_ORDERED
    kset = scsurf.KeyframeSet(kfs)  # marshalled once, reused by every update
    state = [A, B]  # state[0] = current integration poses, state[1] = the other set

    def step(fn):
        order, _ = fn(kset, wl.intr, state[0], state[1], n_kf, mode)
        state[0], state[1] = state[1], state[0]
        return order

    tune_ms = None
    if args.schedule:
        vol.set_schedule(*[int(x) for x in args.schedule.split(",")])
    sched = vol.get_schedule()
    if not args.no_autotune and not args.schedule:
        sched, tune_ms = vol.autotune(kset, wl.intr, state[0], state[1], n_kf, mode)
        log(f"autotuned schedule {sched} ({tune_ms:.2f} ms)")
    if args.sweep:
        sweep = [(8, 4, 2, 0), (8, 4, 4, 0), (8, 4, 8, 0), (4, 2, 8, 0), (4, 2, 16, 0), (2, 4, 4, 0), (2, 4, 8, 0),
                 (1, 8, 2, 0), (1, 8, 4, 0), (8, 4, 2, 1), (8, 4, 4, 1), (8, 2, 4, 1), (8, 2, 8, 1), (8, 1, 16, 1), (8, 4, 4, 2), (8, 2, 8, 2), (8, 1, 16, 2), (8, 4, 4, 3), (8, 2, 8, 3), (8, 1, 16, 3),
                 (8, 4, 4, 4), (8, 2, 8, 4), (8, 1, 16, 4)]
        keep = vol.get_schedule()
        for sc in sweep:
            vol.set_schedule(*sc)
            step(vol.reintegrate_batch)
            vol.batch_timing(4)
            for _ in range(4):
                step(vol.reintegrate_batch)
            ms = vol.batch_timing_read()
            vol.batch_timing(0)
            log(f"sweep schedule {sc}: voxel pass {min(ms):.3f} ms (median {sorted(ms)[len(ms) // 2]:.3f})")
        vol.set_schedule(*keep)
    order = []
    for _ in range(args.warmup):
        order = step(vol.reintegrate_batch)
    torch.cuda.synchronize()
    vol.check_error()
    n_sel = len(order) if order else n_kf
    n_ops = 2 * n_sel
    # timed region
    vol.batch_timing(args.steps)
    s0 = vol.stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    host_s = 0.0
    for _ in range(args.steps):
        th = time.perf_counter()
        order = step(vol.reintegrate_batch)
        host_s += time.perf_counter() - th
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    main_ms = vol.batch_timing_read()
    s1 = vol.stats()
    vol.batch_timing(0)
    n_blocks_after = vol.check_error()
    if len(main_ms) != args.steps:
        raise RuntimeError(f"voxel-pass timing events recorded {len(main_ms)} of {args.steps} launches")
    n_sel = len(order)
    n_ops = 2 * n_sel
    cand, pairs, upd, written = [(b - a) / args.steps for a, b in zip(s0, s1)]
    log(f"voxel pass per launch: min {min(main_ms):.3f} median {float(np.median(main_ms)):.3f} "
        f"max {max(main_ms):.3f} ms; host time in the update calls {host_s * 1e3 / args.steps:.3f} ms/step")
    log(f"batched: {ms_per_step:.3f} ms/step, voxel pass {np.mean(main_ms):.3f} ms, "
        f"{cand:.0f} candidate blocks, {written:.0f} written, {upd / 1e6:.1f} M voxel updates, "
        f"{n_blocks_after} blocks allocated")
    value = n_sel / (ms_per_step / 1e3)
    pass_ms = float(np.mean(main_ms))
    # algorithmic bytes of one pass: every written block read and written once at the method's 12 B per
    # voxel, every operation's keyframe read once; the storage figure counts the FP64 D kept here
    kf_bytes = n_ops * H * Wd * KF_PIXEL_BYTES
    alg_bytes = written * 512 * 2 * VOXEL_BYTES + kf_bytes
    storage_bytes = written * 512 * 2 * STORAGE_VOXEL_BYTES + kf_bytes
    achieved = alg_bytes / (pass_ms / 1e3) / 1e9
    # the keyframes end integrated at the poses they were first integrated at, whatever the step count,
    # so the plain-path steps and the mesh below start from that state
    if state[0] is not A:
        step(vol.reintegrate_batch)
        torch.cuda.synchronize()
    digest = source_digest()
    variant = kernel_variant(sched)
    traffic = traffic_from_profile(digest, variant)

    plain = None
    if not args.no_plain and args.plain_steps > 0:
        plain_steps = args.plain_steps + (args.plain_steps & 1)  # even: the volume returns to the first poses
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(plain_steps):
            step(vol.reintegrate_plain)
        torch.cuda.synchronize()
        pms = (time.perf_counter() - t0) * 1e3 / plain_steps
        vol.check_error()
        plain = {"ms_per_step": round(pms, 3), "keyframes_per_s": round(n_sel / (pms / 1e3), 1),
                 "batched_speedup": round(pms / ms_per_step, 2)}
        log(f"plain: {pms:.3f} ms/step ({plain['batched_speedup']}x slower than batched)")

    mesh_res = None
    if not args.no_mesh:
        mesh_res = mesh_stage(torch, scsurf, surface, synth, vol, wl)
        log(f"mesh: {mesh_res}")

    bwd_full_ms = None
    if not args.no_adjoint:
        bwd_full_ms = backward_full_stage(torch, vol, kset, wl, A)
        log(f"backward of integrating the 200 keyframes (depth and pose gradients): {bwd_full_ms:.2f} ms")

    online_res = None
    if not args.no_online:
        online_res = online_stage(torch, scsurf, synth)
        log(f"online loop (corridor, {online_res['frames']} frames): {online_res['frames_per_s']} frames/s, "
            f"{online_res['reintegrated_keyframes']} keyframe re-integrations incl. a final pass of "
            f"{online_res['final_pass_keyframes']}")
        online_res["held_integrations"] = online_stage(torch, scsurf, synth, integrate_every=20)
        log(f"online loop, keyframes integrated 20 at a time: {online_res['held_integrations']['frames_per_s']} "
            f"frames/s")
        online_res["streaming"] = online_stage(torch, scsurf, synth, stream_radius=3.0,
                                               pool_blocks=online_res["blocks"] // 4)
        log(f"online loop with streaming (pool of a quarter of the field, 3 m sphere): {online_res['streaming']}")

    adj_ms = None
    if not args.no_adjoint:
        adj_ms = adjoint_stage(torch, scsurf, synth)
        log(f"adjoint forward+backward (16 keyframes, 320x240): {adj_ms:.2f} ms")

    configs_res = None
    if args.configs:
        configs_res = configs_stage(torch, scsurf, synth, oracle, log)

    surface_res = None
    if args.surface:
        surface_res = surface_stage(torch, scsurf, surface, online, synth, log)

    cpu = None
    if not args.no_cpu:
        sample = sorted(np.random.default_rng(0).choice(n_kf, min(args.cpu_sample, n_kf), replace=False).tolist())
        log(f"oracle: fusing the {len(sample)} sampled keyframes")
        kfs_np = oracle_keyframes(oracle, wl, frames, sample, masks)
        rate, dt = cpu_baseline(oracle, kfs_np, wl.intr, A, B, sample)
        cpu = {"value": round(rate, 4), "unit": "keyframes/s", "cores": oracle.threads(), "kind": "oracle",
               "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
               "sample": f"{len(sample)} of the {n_kf} keyframes, each de-integrated at its integration pose and "
                         f"re-integrated at its new pose on a volume holding those {len(sample)} ({dt:.1f} s)"}
        log(f"oracle: {rate:.3f} keyframes/s on {oracle.threads()} threads")
        if args.configs:
            n_all = oracle.threads()
            oracle.set_threads(1)
            rate1, _ = cpu_baseline(oracle, kfs_np, wl.intr, A, B, sample[:3])
            oracle.set_threads(n_all)
            cpu["one_core_value"] = round(rate1, 4)
            log(f"oracle on one thread: {rate1:.3f} keyframes/s")

    if args.calib_copy_gib > 0:
        n = int(args.calib_copy_gib * (1 << 30)) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"calibration copy of {args.calib_copy_gib} GiB done")

    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "keyframes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32/f64",
        "data": "synthetic",
        "config": {
            "workload": "batched re-integration: 10x10x3 m room with 40 boxes/spheres, 1000 frames at 640x480 "
                        "fused 5 per keyframe into 200 keyframes with valid-pixel fractions U(0.4,1.0), "
                        "voxel 1 cm, truncation 4 cm, 2^21 buckets, FP64 TSDF + RGBA8 colour + FP32 weight; "
                        "one pose-graph update moving all 200 poses by N(0, 3 cm / 1.5 deg), keyframes "
                        "ordered by pose change, de-integrated and re-integrated in one persistent launch",
            "keyframes": n_kf, "operations": n_ops, "resolution": [Wd, H], "blocks": n_blocks_after,
            "schedule": list(sched), "parallelism": "single GPU",
        },
        "voxel_updates_per_s": round(upd / (ms_per_step / 1e3), 1),
        "voxel_updates_per_step": int(upd),
        "hbm_frac": round(achieved / HBM_PEAK_GBS, 4),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": variant,
                     "kernel_ms": round(pass_ms, 4), "algorithmic_bytes": int(alg_bytes),
                     "algorithmic_bytes_rule": "blocks written x 512 voxels x 2 x 12 B (FP32 D, FP32 W, RGBA8 C) "
                                               "+ operations x H x W x 12 B (keyframe depth, weight, RGBA8)",
                     "storage_bytes": int(storage_bytes),
                     "storage_frac": round(storage_bytes / (pass_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                     "blocks_written": int(written), "candidate_blocks": int(cand), "block_op_pairs": int(pairs),
                     "source_digest": digest},
        "cpu_baseline": cpu,
        "plain": plain,
        "stages": {"kf_fuse_frames_per_s": round(n_kf * wl.kappa / fuse_s, 1),
                   # algorithmic bytes of fusing one keyframe: kappa frames of depth (4 B) and RGB (3 B)
                   # read, one keyframe of depth, weight and RGBA8 (12 B) written, per pixel
                   "kf_fuse_hbm_frac": round(n_kf * H * Wd * (wl.kappa * 7 + 12) / fuse_s / 1e9 / HBM_PEAK_GBS, 5),
                   "integrate_keyframes_per_s": round(n_kf / integrate_s, 1),
                   "integrate_batch_keyframes_per_s": round(n_kf / integrate_batch_s, 1),
                   # plain integration of the 200 keyframes into the empty volume: blocks written once
                   # (read and write at the method's 12 B per voxel) plus each keyframe read once
                   "integrate_hbm_frac": round((n_blocks * 512 * 2 * VOXEL_BYTES + n_kf * H * Wd * KF_PIXEL_BYTES)
                                               / integrate_s / 1e9 / HBM_PEAK_GBS, 5),
                   "keyframe_pack_ms_per_keyframe": None if pack_s is None else round(pack_s * 1e3 / n_kf, 4),
                   "autotune_best_ms": tune_ms, "adjoint_fwd_bwd_ms": adj_ms,
                   "backward_200_keyframes_ms": bwd_full_ms, "online_loop": online_res,
                   "mesh": mesh_res, "mesh_poses": "the keyframes integrated at their first poses"},
    }
    if surface_res is not None:
        out["surface_study"] = surface_res
    if configs_res is not None:
        out["configs"] = configs_res
    print(json.dumps(out), flush=True)
    vol.close()


if __name__ == "__main__":
    main()
