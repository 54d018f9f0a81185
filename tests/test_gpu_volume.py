"""GPU parity of the voxel-hashed TSDF against the FP64 oracle: block
allocation, integration (Sec. 3 running average), de-integration (Eq. 2) and
the plain re-integration path (Sec. 4.3).  Block sets and weights must match
bit-exactly, RGBA8 colour exactly, D (and FP32 colour) within 1e-5."""
import numpy as np
import pytest
import torch

import oracle
from oracle import selection as osel
from paper_1709_03763_amd import scsurf, synth
from tests.helpers import as_f32_color, compare_fields, oracle_keyframes

pytestmark = pytest.mark.gpu

S, MU = 0.01, 0.04


def _say(msg):
    print(f"[gpu] {msg}", flush=True)


def _dev_kf(kf, f32=False):
    c = kf["color"]
    if f32:
        col = torch.from_numpy(np.ascontiguousarray(c, np.float32)).cuda()
    else:
        col = torch.from_numpy(np.ascontiguousarray(c, np.uint8)).cuda()
    return scsurf.Keyframe(torch.from_numpy(np.ascontiguousarray(kf["depth"])).cuda(),
                           torch.from_numpy(np.ascontiguousarray(kf["weight"])).cuda(), col)


@pytest.fixture(scope="module")
def c1():
    assert torch.cuda.is_available(), "GPU tests need a device"
    wl = synth.workload(1)
    kf = oracle_keyframes(wl, [np.arange(5)])[0]
    Rp, tp = synth.perturb_fixed(wl.R[:1], wl.t[:1], 0.01, 0.5, 101)
    return wl, kf, (wl.R[0], wl.t[0]), (Rp[0], tp[0])


def test_integrate_deintegrate_reintegrate_c1(c1):
    wl, kf, T0, T1 = c1
    _say("c1 integrate")
    vol = scsurf.Volume(S, MU, 1 << 16, 1 << 15)
    dk = _dev_kf(kf)
    ref = oracle.Volume(S, MU)
    vol.integrate(dk, wl.intr, *T0)
    assert ref.integrate(kf, wl.intr, *T0) == oracle.OK
    assert vol.check_error() == ref.n_blocks
    compare_fields(vol.export_sorted(), ref.export())
    _say("c1 deintegrate")
    vol.deintegrate(dk, wl.intr, *T0)
    assert ref.deintegrate(kf, wl.intr, *T0) == oracle.OK
    vol.check_error()
    g = vol.export_sorted()
    assert np.all(g["W"] == 0) and np.all(g["D"] == 0) and np.all(g["C"] == 0)
    compare_fields(g, ref.export())
    _say("c1 reintegrate at the corrected pose")
    vol.integrate(dk, wl.intr, *T1)
    assert ref.integrate(kf, wl.intr, *T1) == oracle.OK
    vol.check_error()
    compare_fields(vol.export_sorted(), ref.export())
    vol.close()


@pytest.fixture(scope="module")
def c3kfs():
    assert torch.cuda.is_available()
    wl = synth.workload(3)
    groups = [np.arange(5) + 5 * k for k in range(0, 16, 3)]
    return wl, oracle_keyframes(wl, groups), groups


@pytest.mark.parametrize("f32", [False, True])
def test_plain_reintegration_matches_oracle(c3kfs, f32):
    """Integrate six overlapping keyframes, then apply one pose-graph update with
    the plain per-keyframe path in each selection mode (Sec. 4.3)."""
    wl, kfs, groups = c3kfs
    R = np.array([wl.R[g[0]] for g in groups])
    t = np.array([wl.t[g[0]] for g in groups])
    Rn, tn = synth.perturb_all(R, t, 0.02, 1.0, 7)
    mode_c = scsurf.COLOR_F32 if f32 else scsurf.COLOR_RGBA8
    okf = [as_f32_color(k) for k in kfs] if f32 else kfs
    for mode in (scsurf.SEL_EQ3, scsurf.SEL_TOPM, scsurf.SEL_ALL_ORDERED):
        _say(f"plain reintegration f32={f32} mode={mode}")
        vol = scsurf.Volume(S, MU, 1 << 17, 1 << 16, color_mode=mode_c)
        ref = oracle.Volume(S, MU, color_f32=f32)
        dks = [_dev_kf(k, f32) for k in okf]
        for k in range(len(kfs)):
            vol.integrate(dks[k], wl.intr, R[k], t[k])
            assert ref.integrate(okf[k], wl.intr, R[k], t[k]) == oracle.OK
        order, (Ru, tu) = vol.reintegrate_plain(dks, wl.intr, (R, t), (Rn, tn), 3, mode)
        exp = osel.select(osel.distances(R, t, Rn, tn), 3, mode)
        assert order == exp
        for k in exp:
            assert ref.deintegrate(okf[k], wl.intr, R[k], t[k]) == oracle.OK
        for k in exp:
            assert ref.integrate(okf[k], wl.intr, Rn[k], tn[k]) == oracle.OK
        for k in range(len(kfs)):
            want = (Rn[k], tn[k]) if k in exp else (R[k], t[k])
            assert np.array_equal(Ru[k], want[0]) and np.array_equal(tu[k], want[1])
        vol.check_error()
        compare_fields(vol.export_sorted(), ref.export(), exact_color=not f32)
        vol.close()


def test_hash_alloc_dedup_and_idempotence():
    assert torch.cuda.is_available()
    _say("hash_alloc")
    rng = np.random.default_rng(0)
    base = rng.integers(-300, 300, (5000, 3)).astype(np.int32)
    xyz = np.concatenate([base, base[rng.integers(0, 5000, 20000)], base[:64].repeat(64, 0)])
    rng.shuffle(xyz)
    vol = scsurf.Volume(S, MU, 1 << 14, 1 << 14)
    d = torch.from_numpy(xyz).cuda()
    slots = vol.hash_alloc(d).cpu().numpy()
    uniq = np.unique(base, axis=0)
    n = vol.check_error()
    assert n == len(uniq)
    f = vol.export_sorted()
    np.testing.assert_array_equal(f["blocks"], uniq)
    # one slot per distinct key, equal keys share it
    key = [tuple(x) for x in xyz]
    first = {}
    for k, s in zip(key, slots):
        assert first.setdefault(k, s) == s
    assert len(set(first.values())) == len(uniq) and min(first.values()) >= 0
    slots2 = vol.hash_alloc(d).cpu().numpy()
    assert vol.check_error() == n
    np.testing.assert_array_equal(slots, slots2)
    vol.close()


def test_forced_collisions_keep_the_same_set():
    """A table of 2^13 buckets for 5000 keys forces long probe chains."""
    _say("hash collisions")
    rng = np.random.default_rng(1)
    xyz = rng.integers(-2000, 2000, (5000, 3)).astype(np.int32)
    vol = scsurf.Volume(S, MU, 1 << 13, 1 << 13)
    slots = vol.hash_alloc(torch.from_numpy(xyz).cuda()).cpu().numpy()
    vol.check_error()
    np.testing.assert_array_equal(vol.export_sorted()["blocks"], np.unique(xyz, axis=0))
    assert len(np.unique(slots)) == len(np.unique(xyz, axis=0))
    vol.close()


def test_error_paths(c1):
    wl, kf, T0, T1 = c1
    dk = _dev_kf(kf)
    _say("error: de-integrate an unallocated keyframe")
    vol = scsurf.Volume(S, MU, 1 << 16, 1 << 15)
    vol.deintegrate(dk, wl.intr, *T0)
    assert vol.query()[1] == scsurf.SC_ENOTALLOC
    _say("error: weight below zero")
    vol.reset()
    vol.integrate(dk, wl.intr, *T0)
    vol.deintegrate(dk, wl.intr, *T0)
    assert vol.query()[1] == scsurf.SC_OK
    vol.deintegrate(dk, wl.intr, *T0)
    assert vol.query()[1] == scsurf.SC_EWEIGHT
    vol.close()
    _say("error: pool full")
    small = scsurf.Volume(S, MU, 1 << 16, 64)
    small.integrate(dk, wl.intr, *T0)
    n, e = small.query()
    assert e == scsurf.SC_EPOOLFULL and n == 64
    small.close()
    _say("error: hash table full")
    tiny = scsurf.Volume(S, MU, 1 << 6, 1 << 15)
    tiny.integrate(dk, wl.intr, *T0)
    assert tiny.query()[1] == scsurf.SC_EHASHFULL
    tiny.close()


def test_argument_errors_enqueue_nothing():
    _say("argument errors")
    with pytest.raises(scsurf.ScError):
        scsurf.Volume(S, MU, 1000, 1 << 10)  # not a power of two
    vol = scsurf.Volume(S, MU, 1 << 10, 1 << 10)
    # zero-size images agree with zero-size intrinsics, so the binding passes
    # them on and the library's own check rejects them
    intr = synth.Intrinsics(0, 0, 1.0, 1.0, 0.0, 0.0)
    z = torch.zeros((0, 0), device="cuda")
    with pytest.raises(scsurf.ScError):
        vol.integrate(scsurf.Keyframe(z, z, torch.zeros((0, 0, 4), dtype=torch.uint8, device="cuda")), intr,
                      np.eye(3), np.zeros(3))
    assert vol.query() == (0, 0)
    vol.close()


def test_binding_rejects_mismatched_arguments(c1):
    wl, kf, T0, T1 = c1
    _say("binding checks: image size, colour type, pose counts, import layout")
    dk, dkf = _dev_kf(kf), _dev_kf(as_f32_color(kf), f32=True)
    vol = scsurf.Volume(S, MU, 1 << 16, 1 << 15)
    small = synth.Intrinsics(wl.intr.width - 1, wl.intr.height, wl.intr.fx, wl.intr.fy, wl.intr.cx, wl.intr.cy)
    with pytest.raises(ValueError, match="intrinsics"):
        vol.integrate(dk, small, *T0)
    with pytest.raises(ValueError, match="colour"):
        vol.integrate(dkf, wl.intr, *T0)
    R2, t2 = np.repeat(T0[0][None], 2, 0), np.repeat(np.asarray(T0[1])[None], 2, 0)
    with pytest.raises(ValueError, match="poses"):
        vol.reintegrate_batch([dk], wl.intr, (R2, t2), (R2[:1], t2[:1]), 1)
    f = {"blocks": torch.zeros((2, 3), dtype=torch.int32, device="cuda"),
         "D": torch.zeros((2, 512), device="cuda"), "W": torch.zeros((2, 512), device="cuda"),
         "C": torch.zeros((2, 512, 3), dtype=torch.uint8, device="cuda")}
    with pytest.raises(ValueError, match="C"):
        vol.import_field(f)
    # nothing reached the device
    assert vol.query() == (0, 0)
    vol.close()


def test_empty_keyframe_touches_nothing(c1):
    """A keyframe without a valid pixel allocates and changes nothing, alone
    and as one of the operations of a batched update."""
    wl, kf, T0, T1 = c1
    _say("empty keyframe")
    empty = {"depth": np.zeros_like(kf["depth"]), "weight": np.zeros_like(kf["weight"]),
             "color": np.zeros_like(kf["color"])}
    dk, de = _dev_kf(kf), _dev_kf(empty)
    vol = scsurf.Volume(S, MU, 1 << 16, 1 << 15)
    vol.integrate(de, wl.intr, *T0)
    assert vol.query() == (0, 0)
    vol.integrate(dk, wl.intr, *T0)
    vol.integrate(de, wl.intr, *T1)
    R = np.stack([T0[0], T1[0]])
    t = np.stack([np.asarray(T0[1]), np.asarray(T1[1])])
    Rn = np.stack([T1[0], T0[0]])
    tn = np.stack([np.asarray(T1[1]), np.asarray(T0[1])])
    order, _ = vol.reintegrate_batch([dk, de], wl.intr, (R, t), (Rn, tn), 2, scsurf.SEL_ALL_ORDERED)
    assert sorted(order) == [0, 1]
    vol.check_error()
    ref = oracle.Volume(S, MU)
    assert ref.integrate(kf, wl.intr, *T1) == oracle.OK
    g = vol.export_sorted()
    live = g["W"].reshape(len(g["blocks"]), -1).max(axis=1) > 0
    r = ref.export()
    np.testing.assert_array_equal(g["blocks"][live], r["blocks"])
    compare_fields({k: v[live] for k, v in g.items()}, r)
    vol.close()
