"""Batched re-integration at the benchmark's full size (200 keyframes at
640x480, 1 cm voxels, 2^21 buckets, autotuned schedule) checked on samples
the oracle computes one by one: sampled voxels through the whole operation
sequence, sampled blocks, and the touched blocks of sampled operations.

Keyframes come from the input generator alone (one rendered frame per
keyframe, seeded weights on the 2^-10 grid, the same valid-fraction column
strips as the benchmark), so no oracle input comes from the HIP path."""
import numpy as np
import pytest
import torch

import oracle
from oracle import selection as osel
from paper_1709_03763_amd import scsurf, synth

from tests.helpers import compare_fields

pytestmark = pytest.mark.gpu

S, MU, N_KF = 0.01, 0.04, 200


def _say(msg):
    print(f"[gpu] {msg}", flush=True)


@pytest.fixture(scope="module")
def full():
    assert torch.cuda.is_available(), "GPU tests need a device"
    wl = synth.workload(4)
    first = np.array([g[0] for g in synth.keyframe_groups(wl)[:N_KF]])
    _say("rendering 200 keyframes at 640x480")
    z, rgb = synth.frames(wl, first, device="cuda")
    rng = np.random.default_rng(44)
    kfs = []
    for k in range(N_KF):
        valid = z[k] > 0
        keep = synth.column_strip_mask(valid, rng.uniform(0.4, 1.0), rng)
        w = rng.integers(64, 4096, z[k].shape).astype(np.float32) / 1024.0
        w = np.where(valid & keep, w, 0).astype(np.float32)
        col = np.zeros(z[k].shape + (4,), np.uint8)
        col[..., :3] = rgb[k]
        kfs.append({"depth": np.where(w > 0, z[k], 0).astype(np.float32), "weight": w, "color": col})
    R, t = wl.R[first], wl.t[first]
    Rn, tn = synth.perturb_all(R, t, 0.03, 1.5, 4)
    _say("integrate 200 keyframes, autotune, batched update")
    vol = scsurf.Volume(S, MU, 1 << 21, 1 << 21, scsurf.COLOR_RGBA8, max_batch_ops=512)
    dks = [scsurf.Keyframe(torch.from_numpy(k["depth"]).cuda(), torch.from_numpy(k["weight"]).cuda(),
                           torch.from_numpy(k["color"]).cuda()) for k in kfs]
    for k in range(N_KF):
        vol.integrate(dks[k], wl.intr, R[k], t[k])
    vol.check_error()
    vol.autotune(dks, wl.intr, (R, t), (Rn, tn), N_KF, scsurf.SEL_ALL_ORDERED)
    order, _ = vol.reintegrate_batch(dks, wl.intr, (R, t), (Rn, tn), N_KF, scsurf.SEL_ALL_ORDERED)
    assert order == osel.select(osel.distances(R, t, Rn, tn), N_KF, osel.ALL_ORDERED)
    n = vol.check_error()
    f = vol.export()
    field = {k: v.cpu().numpy() for k, v in f.items()}
    ops = [(k, +1, R[k], t[k]) for k in range(N_KF)]
    ops += [(k, -1, R[k], t[k]) for k in order] + [(k, +1, Rn[k], tn[k]) for k in order]
    _say(f"{n} blocks, schedule {vol.get_schedule()}")
    yield wl, kfs, field, ops, vol
    vol.close()


def test_sampled_voxels_match_oracle(full):
    wl, kfs, field, ops, vol = full
    probe = oracle.Volume(S, MU)
    rng = np.random.default_rng(0)
    nb = field["blocks"].shape[0]
    W = field["W"]
    live = np.argwhere(W > 0)
    pick = live[rng.choice(len(live), 2000, replace=False)]
    pick = np.concatenate([pick, np.stack([rng.integers(0, nb, 500), rng.integers(0, 512, 500)], 1)])
    dmax = 0.0
    for b, i in pick:
        nvox = 8 * field["blocks"][b].astype(np.int64) + np.array([i & 7, (i >> 3) & 7, i >> 6])
        D, Wv, C, rc = probe.voxel_sequence(kfs, wl.intr, ops, nvox)
        assert rc >= 0
        assert W[b, i] == Wv, (b, i)
        assert np.array_equal(field["C"][b, i, :3].astype(np.float64), C), (b, i)
        dmax = max(dmax, abs(float(field["D"][b, i]) - D))
    print(f"sampled voxels: max |D - D_oracle| = {dmax:.2e}", flush=True)
    assert dmax <= 1e-5


def test_sampled_blocks_are_touched(full):
    """Every sampled allocated block holds a voxel that some operation touches."""
    wl, kfs, field, ops, vol = full
    probe = oracle.Volume(S, MU)
    rng = np.random.default_rng(1)
    nb = field["blocks"].shape[0]
    for b in rng.choice(nb, 40, replace=False):
        base = 8 * field["blocks"][b].astype(np.int64)
        hit = False
        for i in rng.permutation(512):
            nvox = base + np.array([i & 7, (i >> 3) & 7, i >> 6])
            if probe.voxel_sequence(kfs, wl.intr, ops, nvox)[3] > 0:
                hit = True
                break
        assert hit, f"block {field['blocks'][b]} allocated but never touched"


def test_touched_blocks_of_sampled_operations_are_allocated(full):
    wl, kfs, field, ops, vol = full
    probe = oracle.Volume(S, MU)
    have = set(map(tuple, field["blocks"].tolist()))
    rng = np.random.default_rng(2)
    for j in rng.choice(len(ops), 4, replace=False):
        k, sign, R, t = ops[j]
        rec = probe.record(kfs[k], wl.intr, R, t)
        blocks = set(map(tuple, np.floor_divide(rec["n"], 8).tolist()))
        assert blocks <= have, f"operation {j}: {len(blocks - have)} touched blocks missing"


@pytest.fixture(scope="module")
def oracle_field(full):
    """The oracle's own field after the same 600 operations."""
    wl, kfs, field, ops, vol = full
    _say("oracle: 200 integrations and the 400-operation update")
    ref = oracle.Volume(S, MU)
    for k, sign, R, t in ops:
        rc = ref.integrate(kfs[k], wl.intr, R, t) if sign > 0 else ref.deintegrate(kfs[k], wl.intr, R, t)
        assert rc == oracle.OK
    return ref.export()


def test_whole_field_matches_oracle(full, oracle_field):
    """The whole field after the 600 operations: the allocated-block set
    bit-exact as a set, W and RGBA8 colour exact, D within 1e-5 m."""
    wl, kfs, field, ops, vol = full
    compare_fields(vol.export_sorted(), oracle_field)


def _anchor_blocks(keys):
    """Block of the cube each triangle comes from: the centre vertex's voxel
    when the triangle has one, else the componentwise minimum of its edge
    keys (three edge vertices of one cube never all lie on its far faces)."""
    k = keys.astype(np.int64)
    centre = k[:, :, 3] >= 3
    anchor = k[:, :, :3].min(axis=1)
    has_c = centre.any(axis=1)
    ci = np.argmax(centre, axis=1)
    anchor[has_c] = k[has_c, ci[has_c], :3]
    return np.floor_divide(anchor, 8)


def _pack(b):
    b = np.asarray(b, np.int64) + (1 << 20)
    return (b[:, 0] << 42) | (b[:, 1] << 21) | b[:, 2]


def test_mesh_on_sampled_blocks_matches_oracle(full, oracle_field):
    """Marching Cubes at the benchmark's full size: the cubes anchored in 3000
    sampled blocks give the same triangles (keys and orientation) on the
    GPU and in the oracle, with vertices within 1e-6 m."""
    from oracle import mesh as M
    wl, kfs, field, ops, vol = full
    rng = np.random.default_rng(3)
    ob = oracle_field["blocks"]
    pick = ob[rng.choice(len(ob), 3000, replace=False)]
    tri_o, key_o = M.marching_cubes(oracle_field, S, pick)
    assert np.isin(_pack(_anchor_blocks(key_o)), _pack(pick)).all(), "the anchor rule holds on the oracle's mesh"
    xyz, keys = vol.mesh()
    _say(f"full-size mesh: {xyz.shape[0]} triangles on the GPU")
    kg = keys.cpu().numpy().astype(np.int64)
    mine = np.isin(_pack(_anchor_blocks(kg)), _pack(pick))
    kg, xg = kg[mine], xyz.cpu().numpy().astype(np.float64)[mine]
    assert len(kg) == len(key_o) > 10000
    allk = np.concatenate([kg.reshape(-1, 4), key_o.reshape(-1, 4)])
    _, inv = np.unique(allk, axis=0, return_inverse=True)
    inv = inv.reshape(-1)
    ig, io = inv[:kg.size // 4].reshape(-1, 3), inv[kg.size // 4:].reshape(-1, 3)

    def canon(t):
        r = np.argmin(t, axis=1)
        rows = np.arange(len(t))
        c = np.stack([t[rows, r], t[rows, (r + 1) % 3], t[rows, (r + 2) % 3]], 1)
        return c[np.lexsort((c[:, 2], c[:, 1], c[:, 0]))]

    np.testing.assert_array_equal(canon(ig), canon(io))
    pg = np.zeros((inv.max() + 1, 3))
    po = np.zeros_like(pg)
    pg[ig.reshape(-1)] = xg.reshape(-1, 3)
    po[io.reshape(-1)] = tri_o.reshape(-1, 3)
    err = np.abs(pg - po).max()
    _say(f"full-size mesh: {len(kg)} triangles in the sampled blocks, max vertex difference {err:.2e} m")
    assert err <= 1e-6


def test_nn_distance_full_size_sampled():
    """Capped distances at the benchmark's sizes (3 M queries against 4 M
    reference points on the large room's surfaces), checked on 200 k
    sampled queries against the oracle."""
    from oracle import mesh as M
    from paper_1709_03763_amd import surface
    wl = synth.workload(4)
    ref = synth.surface_points(wl.scene, 4_000_000, 7)
    rng = np.random.default_rng(8)
    q = synth.surface_points(wl.scene, 3_000_000, 9)
    q = (q + rng.normal(0, 0.01, q.shape)).astype(np.float32)
    d, total = surface.nn_distance(torch.from_numpy(ref).cuda(), torch.from_numpy(q).cuda(), 0.05)
    d = d.cpu().numpy()
    pick = rng.choice(len(q), 200_000, replace=False)
    exp = M.nn_distance(ref.astype(np.float64), q[pick].astype(np.float64), float(np.float32(0.05)))
    np.testing.assert_allclose(d[pick], exp, rtol=1e-6, atol=1e-9)
    assert total == pytest.approx(float(d.astype(np.float64).sum()), rel=1e-9)
