"""The binding checks shapes, dtypes and pose counts against the intrinsics
before a pointer reaches the library (whose kernels trust the sizes they are
given).  These checks raise before any device call, so they run on the CPU."""
import numpy as np
import pytest
import torch

from paper_1709_03763_amd import scsurf, synth

INTR = synth.Intrinsics(16, 12, 10.0, 10.0, 7.5, 5.5)


def test_depth_weight_checks_the_image_size():
    with pytest.raises(ValueError, match="depth"):
        scsurf.depth_weight(torch.zeros((2, 12, 15)), INTR)


def test_kf_fuse_checks_sizes_and_pose_count():
    z = torch.zeros((3, 12, 16))
    rgb = torch.zeros((3, 12, 16, 3), dtype=torch.uint8)
    R, t = np.repeat(np.eye(3)[None], 3, 0), np.zeros((3, 3))
    with pytest.raises(ValueError, match="depth"):
        scsurf.kf_fuse(torch.zeros((3, 11, 16)), rgb, R, t, INTR)
    with pytest.raises(ValueError, match="rgb"):
        scsurf.kf_fuse(z, torch.zeros((3, 12, 16, 4), dtype=torch.uint8), R, t, INTR)
    with pytest.raises(ValueError, match="poses"):
        scsurf.kf_fuse(z, rgb, R[:2], t[:2], INTR)


def test_color_prep_needs_three_channels():
    with pytest.raises(ValueError, match="rgb"):
        scsurf.color_prep(torch.zeros((1, 12, 16, 4), dtype=torch.uint8))


def test_overlap_checks_the_pixel_count():
    with pytest.raises(ValueError, match="pixels"):
        scsurf.overlap(torch.zeros((12, 15)), INTR, np.eye(3), np.zeros(3), np.eye(3), np.zeros(3))


def test_keyframe_tensors_must_agree():
    kf = scsurf.Keyframe(torch.zeros((12, 16)), torch.zeros((12, 16)), torch.zeros((12, 16, 3), dtype=torch.uint8))
    with pytest.raises(ValueError, match="RGBA8"):
        kf.image_size()
    kf = scsurf.Keyframe(torch.zeros((12, 16)), torch.zeros((12, 15)), torch.zeros((12, 16, 4), dtype=torch.uint8))
    with pytest.raises(ValueError, match="weight"):
        kf.image_size()
    kf = scsurf.Keyframe(torch.zeros((12, 16)), torch.zeros((12, 16)), torch.zeros((12, 16, 3), dtype=torch.float64))
    with pytest.raises(ValueError, match="colour"):
        kf.image_size()
    ok = scsurf.Keyframe(torch.zeros((12, 16)), torch.zeros((12, 16)), torch.zeros((12, 16, 4), dtype=torch.uint8))
    assert ok.image_size() == (12, 16)


def test_keyframe_set_must_share_size_and_colour_type():
    a = scsurf.Keyframe(torch.zeros((12, 16)), torch.zeros((12, 16)), torch.zeros((12, 16, 4), dtype=torch.uint8))
    b = scsurf.Keyframe(torch.zeros((12, 8)), torch.zeros((12, 8)), torch.zeros((12, 8, 4), dtype=torch.uint8))
    c = scsurf.Keyframe(torch.zeros((12, 16)), torch.zeros((12, 16)), torch.zeros((12, 16, 3)))
    for kfs in ([a, b], [a, c]):
        with pytest.raises(ValueError, match="share"):
            scsurf.KeyframeSet(kfs)
