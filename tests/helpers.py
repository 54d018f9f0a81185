"""Shared test helpers: workloads, keyframes and field comparison."""
import numpy as np

import oracle
from paper_1709_03763_amd import synth


def oracle_keyframes(wl, groups):
    """Oracle-fused keyframes for frame groups of a workload (numpy)."""
    out = []
    for g in groups:
        z, rgb = synth.frames(wl, g)
        out.append(oracle.kf_fuse(z, rgb, wl.intr, wl.R[g], wl.t[g]))
    return out


def as_f32_color(kf):
    return {"depth": kf["depth"], "weight": kf["weight"],
            "color": kf["color"][..., :3].astype(np.float32) / np.float32(255.0)}


def compare_fields(gpu, ref, d_tol=1e-5, c_tol=1e-5, exact_color=True):
    """Bit-exact block set and weights, D within d_tol, colour exact (RGBA8)
    or within c_tol (FP32)."""
    gb, rb = gpu["blocks"], ref["blocks"]
    assert gb.shape == rb.shape, f"block count {gb.shape[0]} vs oracle {rb.shape[0]}"
    assert np.array_equal(gb, rb), "block sets differ"
    np.testing.assert_array_equal(gpu["W"].astype(np.float64), ref["W"])
    dmax = float(np.abs(gpu["D"].astype(np.float64) - ref["D"]).max()) if len(rb) else 0.0
    assert dmax <= d_tol, f"max |D - D_ref| = {dmax}"
    if exact_color:
        np.testing.assert_array_equal(gpu["C"].astype(np.float64), ref["C"])
        cmax = 0.0
    else:
        cmax = float(np.abs(gpu["C"].astype(np.float64) - ref["C"]).max()) if len(rb) else 0.0
        assert cmax <= c_tol, f"max |C - C_ref| = {cmax}"
    print(f"[parity] {len(rb)} blocks identical, W identical, max |D - D_oracle| = {dmax:.2e} m, "
          f"max |C - C_oracle| = {cmax:.2e}", flush=True)
    return dmax
