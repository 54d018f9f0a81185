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
