"""Failure handling of the volume: a pose-graph update that overflows the
block pool (or the hash table) in the middle of a batched update leaves a
sticky error; reset clears it, and re-integrating the stored keyframes at
their integration poses rebuilds the field the oracle holds (Sec. 4.3: the
keyframes are kept so that the volume can be rebuilt from them).  Also the
treatment of non-finite keyframe values: a pixel whose depth is not finite,
or whose weight is NaN, touches no voxel; an infinite weight is a weight
error."""
import numpy as np
import pytest
import torch

import oracle
from paper_1709_03763_amd import scsurf, synth
from tests.helpers import compare_fields, oracle_keyframes

pytestmark = pytest.mark.gpu

S, MU = 0.01, 0.04


def _say(msg):
    print(f"[gpu] {msg}", flush=True)


def _dev_kf(kf):
    return scsurf.Keyframe(torch.from_numpy(np.ascontiguousarray(kf["depth"])).cuda(),
                           torch.from_numpy(np.ascontiguousarray(kf["weight"])).cuda(),
                           torch.from_numpy(np.ascontiguousarray(kf["color"])).cuda())


@pytest.fixture(scope="module")
def scene():
    assert torch.cuda.is_available(), "GPU tests need a device"
    wl = synth.workload(3)
    groups = [np.arange(5) + 5 * k for k in range(0, 16, 2)]
    kfs = oracle_keyframes(wl, groups)
    R = np.array([wl.R[g[0]] for g in groups])
    t = np.array([wl.t[g[0]] for g in groups])
    # a large correction, so that re-integration allocates many new blocks
    Rn, tn = synth.perturb_fixed(R, t, 0.06, 4.0, 77)
    ref_old = oracle.Volume(S, MU)
    for k in range(len(kfs)):
        assert ref_old.integrate(kfs[k], wl.intr, R[k], t[k]) == oracle.OK
    ref_new = oracle.Volume(S, MU)
    for k in range(len(kfs)):
        assert ref_new.integrate(kfs[k], wl.intr, R[k], t[k]) == oracle.OK
    order = list(range(len(kfs)))
    for k in order:
        assert ref_new.deintegrate(kfs[k], wl.intr, R[k], t[k]) == oracle.OK
    for k in order:
        assert ref_new.integrate(kfs[k], wl.intr, Rn[k], tn[k]) == oracle.OK
    return wl, kfs, R, t, Rn, tn, ref_old.export(), ref_new.export()


def test_pool_overflow_mid_batch_then_reset_and_rebuild(scene):
    wl, kfs, R, t, Rn, tn, f_old, f_new = scene
    n_old, n_new = len(f_old["blocks"]), len(f_new["blocks"])
    assert n_new > n_old + 200, (n_old, n_new)
    cap = n_old + (n_new - n_old) // 2
    _say(f"pool of {cap} blocks: {n_old} before the update, {n_new} after it")
    vol = scsurf.Volume(S, MU, 1 << 17, cap)
    dks = [_dev_kf(k) for k in kfs]
    for k in range(len(kfs)):
        vol.integrate(dks[k], wl.intr, R[k], t[k])
    assert vol.check_error() == n_old
    vol.reintegrate_batch(dks, wl.intr, (R, t), (Rn, tn), len(kfs), scsurf.SEL_ALL_ORDERED)
    n, err = vol.query()
    assert err == scsurf.SC_EPOOLFULL
    # reset clears the error and the field
    vol.reset()
    assert vol.query() == (0, scsurf.SC_OK)
    # rebuild: the stored keyframes at their integration poses (the failed
    # update is not applied)
    for k in range(len(kfs)):
        vol.integrate(dks[k], wl.intr, R[k], t[k])
    vol.check_error()
    compare_fields(vol.export_sorted(), f_old)
    # a volume sized for the update applies it and matches the oracle
    big = scsurf.Volume(S, MU, 1 << 17, n_new + 1024)
    for k in range(len(kfs)):
        big.integrate(dks[k], wl.intr, R[k], t[k])
    big.reintegrate_batch(dks, wl.intr, (R, t), (Rn, tn), len(kfs), scsurf.SEL_ALL_ORDERED)
    big.check_error()
    compare_fields(big.export_sorted(), f_new)
    vol.close()
    big.close()


def test_hash_overflow_then_reset_and_rebuild(scene):
    wl, kfs, R, t, Rn, tn, f_old, f_new = scene
    n_old = len(f_old["blocks"])
    buckets = 1 << int(np.floor(np.log2(n_old)))  # fewer buckets than blocks
    _say(f"{buckets} buckets for {n_old} blocks")
    vol = scsurf.Volume(S, MU, buckets, 1 << 16)
    dks = [_dev_kf(k) for k in kfs]
    for k in range(len(kfs)):
        vol.integrate(dks[k], wl.intr, R[k], t[k])
    assert vol.query()[1] == scsurf.SC_EHASHFULL
    vol.close()
    # the rebuild in a table of adequate size equals the oracle
    vol = scsurf.Volume(S, MU, 1 << 17, 1 << 16)
    for k in range(len(kfs)):
        vol.integrate(dks[k], wl.intr, R[k], t[k])
    vol.check_error()
    compare_fields(vol.export_sorted(), f_old)
    vol.close()


def test_non_finite_keyframe_values(scene):
    """Depth NaN or +-inf and weight NaN at seeded pixels: those pixels touch
    nothing, on the GPU as in the oracle, so both equal the field of the
    keyframe with those pixels zeroed; an infinite weight at a pixel whose
    depth lies in the band is a weight error."""
    wl, kfs, R, t, Rn, tn = scene[:6]
    kf = kfs[0]
    rng = np.random.default_rng(5)
    H, W = kf["depth"].shape
    valid = np.flatnonzero(kf["weight"].reshape(-1) > 0)
    pick = rng.choice(valid, 4000, replace=False)
    bad = {"depth": kf["depth"].copy(), "weight": kf["weight"].copy(), "color": kf["color"]}
    d, w = bad["depth"].reshape(-1), bad["weight"].reshape(-1)
    d[pick[:1000]] = np.nan
    d[pick[1000:2000]] = np.inf
    d[pick[2000:3000]] = -np.inf
    w[pick[3000:]] = np.nan
    zeroed = {"depth": kf["depth"].copy(), "weight": kf["weight"].copy(), "color": kf["color"]}
    zeroed["depth"].reshape(-1)[pick] = 0.0
    zeroed["weight"].reshape(-1)[pick] = 0.0
    _say("non-finite depth and weight")
    ref_bad, ref_zero = oracle.Volume(S, MU), oracle.Volume(S, MU)
    assert ref_bad.integrate(bad, wl.intr, R[0], t[0]) == oracle.OK
    assert ref_zero.integrate(zeroed, wl.intr, R[0], t[0]) == oracle.OK
    fz = ref_zero.export()
    fb = ref_bad.export()
    assert np.array_equal(fb["blocks"], fz["blocks"]) and np.array_equal(fb["W"], fz["W"])
    vol = scsurf.Volume(S, MU, 1 << 17, 1 << 16)
    bad_d = _dev_kf(bad)
    vol.integrate(bad_d, wl.intr, R[0], t[0])
    vol.check_error()
    compare_fields(vol.export_sorted(), fz)
    # the batched path treats them alike: an update of that keyframe equals
    # the oracle's update of the zeroed one
    order, _ = vol.reintegrate_batch([bad_d], wl.intr, (R[:1], t[:1]), (Rn[:1], tn[:1]), 1, scsurf.SEL_EQ3)
    assert order == [0]
    vol.check_error()
    assert ref_zero.deintegrate(zeroed, wl.intr, R[0], t[0]) == oracle.OK
    assert ref_zero.integrate(zeroed, wl.intr, Rn[0], tn[0]) == oracle.OK
    compare_fields(vol.export_sorted(), ref_zero.export())
    # an infinite weight on a patch of surface pixels: weight error, as in
    # the oracle
    inf_w = {"depth": kf["depth"], "weight": kf["weight"].copy(), "color": kf["color"]}
    v0, u0 = np.argwhere(kf["weight"] > 0)[len(valid) // 2]
    patch = (slice(max(v0 - 3, 0), v0 + 4), slice(max(u0 - 3, 0), u0 + 4))
    inf_w["weight"][patch] = np.where(kf["weight"][patch] > 0, np.inf, 0.0).astype(np.float32)
    assert oracle.Volume(S, MU).integrate(inf_w, wl.intr, R[0], t[0]) == oracle.EWEIGHT
    vol2 = scsurf.Volume(S, MU, 1 << 17, 1 << 16)
    vol2.integrate(_dev_kf(inf_w), wl.intr, R[0], t[0])
    assert vol2.query()[1] == scsurf.SC_EWEIGHT
    vol.close()
    vol2.close()
