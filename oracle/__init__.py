"""FP64 CPU oracle of the surface-correction hot path.

TEST INFRASTRUCTURE ONLY: tests/, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` are the only callers.  The product path
(``paper_1709_03763_amd``) never imports this package, and this package never
imports the product path; both share only the seeded input generator.

The heavy per-voxel and per-pixel loops live in ``scsurf_oracle.c`` (plain C,
FP64 values, FP32 decisions in a written order, ``-ffp-contract=off``);
selection (Eq. 3) and the adjoint are NumPy (``selection.py``,
``adjoint.py``).

Parity unpinned: ``blur`` (the blurriness w_b) reads an unresolved citation
as the re-blur metric of Crete et al.; it is pinned by that metric's closed
forms and invariants, not by a value of the paper.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "scsurf_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

OK, EINVAL, ENOMEM, ENOTALLOC, EWEIGHT = 0, -1, -2, -5, -6


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (no FMA contraction, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
                               "-fopenmp", "-shared", "-fPIC", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        i64, i32, f32 = ctypes.c_int64, ctypes.c_int, ctypes.c_float
        L.ov_create.restype = P
        L.ov_create.argtypes = [f32, f32, i32]
        L.ov_destroy.argtypes = [P]
        L.ov_n_blocks.restype = i64
        L.ov_n_blocks.argtypes = [P]
        L.ov_op.restype = i32
        L.ov_op.argtypes = [P, P, P, P, P, i32, i32, P, P, P, i32, P, P]
        L.ov_record.restype = i64
        L.ov_record.argtypes = [P, P, P, i32, i32, P, P, P, i64, P, P, P, P, P]
        L.ov_touch_one.restype = i32
        L.ov_touch_one.argtypes = [P, P, P, i32, i32, P, P, P, P, P, P]
        L.ov_export.restype = i64
        L.ov_export.argtypes = [P, i64, P, P, P, P]
        L.ov_import.restype = i32
        L.ov_import.argtypes = [P, i64, P, P, P, P]
        L.of_depth_weight.restype = None
        L.of_depth_weight.argtypes = [P, i32, i32, P, f32, f32, f32, P]
        L.of_fuse_depth.restype = None
        L.of_fuse_depth.argtypes = [P, P, i32, i32, i32, P, P, P, i32, P, P]
        L.of_sharpen.restype = None
        L.of_sharpen.argtypes = [P, i32, i32, P]
        L.of_blur.restype = ctypes.c_double
        L.of_blur.argtypes = [P, i32, i32, P]
        L.of_fuse_color.restype = None
        L.of_fuse_color.argtypes = [P, P, P, P, i32, i32, i32, P, P, P, i32, f32, P, P, P]
        L.ov_threads.restype = i32
        L.ov_set_threads.restype = i32
        L.ov_set_threads.argtypes = [i32]
        L.ov_voxel_sequence.restype = i32
        L.ov_voxel_sequence.argtypes = [P, P, P, P, i32, i32, P, i32, P, P, P, P, P, P, P, P]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _intr(intr) -> np.ndarray:
    if hasattr(intr, "fx"):
        return np.array([intr.fx, intr.fy, intr.cx, intr.cy], np.float32)
    return _c(intr, np.float32)


class Volume:
    """Sparse voxel-hashed TSDF held on the host in FP64 (Sec. 3, SDF volume)."""

    def __init__(self, voxel_size: float, trunc: float, color_f32: bool = False):
        self.voxel_size = float(np.float32(voxel_size))
        self.trunc = float(np.float32(trunc))
        self.color_f32 = bool(color_f32)
        self._h = lib().ov_create(voxel_size, trunc, int(color_f32))
        if not self._h:
            raise MemoryError("oracle volume")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().ov_destroy(h)
            self._h = None

    @property
    def n_blocks(self) -> int:
        return int(lib().ov_n_blocks(self._h))

    def _op(self, kf, intr, R, t, sign, box=None):
        Z = _c(kf["depth"], np.float32)
        Wk = _c(kf["weight"], np.float32)
        H, W = Z.shape
        rgba = rgbf = None
        if self.color_f32:
            rgbf = _c(kf["color"], np.float32)
        else:
            rgba = _c(kf["color"], np.uint8)
        Rm = _c(R, np.float64).reshape(9)
        tv = _c(t, np.float64).reshape(3)
        it = _intr(intr)
        lo = hi = None
        if box is not None:
            lo = _c(box[0], np.int64)
            hi = _c(box[1], np.int64)
        return int(lib().ov_op(self._h, _p(Z), _p(Wk), _p(rgba) if rgba is not None else None,
                               _p(rgbf) if rgbf is not None else None, W, H, _p(it), _p(Rm), _p(tv), sign,
                               _p(lo) if lo is not None else None, _p(hi) if hi is not None else None))

    def integrate(self, kf, intr, R, t, box=None) -> int:
        """Running weighted average of one keyframe at pose (R, t) (Sec. 3)."""
        return self._op(kf, intr, R, t, +1, box)

    def deintegrate(self, kf, intr, R, t, box=None) -> int:
        """Exact reversal of integration, Eq. (2) (Sec. 4.3)."""
        return self._op(kf, intr, R, t, -1, box)

    def export(self):
        """All allocated blocks sorted by (x, y, z) block coordinate."""
        n = self.n_blocks
        b = np.zeros((n, 3), np.int64)
        D = np.zeros((n, 512), np.float64)
        W = np.zeros((n, 512), np.float64)
        C = np.zeros((n, 512, 3), np.float64)
        lib().ov_export(self._h, n, _p(b), _p(D), _p(W), _p(C))
        order = np.lexsort((b[:, 2], b[:, 1], b[:, 0]))
        return {"blocks": b[order], "D": D[order], "W": W[order], "C": C[order]}

    def load(self, field):
        b = _c(field["blocks"], np.int64)
        n = len(b)
        rc = lib().ov_import(self._h, n, _p(b), _p(_c(field["D"], np.float64)), _p(_c(field["W"], np.float64)),
                             _p(_c(field["C"], np.float64)))
        if rc != OK:
            raise MemoryError("oracle import")

    def record(self, kf, intr, R, t):
        """Touched voxels of (keyframe, pose) without updating: coordinates,
        keyframe pixel, quantised weight, FP64 distance, FP32 camera point."""
        Z = _c(kf["depth"], np.float32)
        Wk = _c(kf["weight"], np.float32)
        H, W = Z.shape
        it = _intr(intr)
        Rm = _c(R, np.float64).reshape(9)
        tv = _c(t, np.float64).reshape(3)
        L = lib()
        cnt = int(L.ov_record(self._h, _p(Z), _p(Wk), W, H, _p(it), _p(Rm), _p(tv), 0, None, None, None, None, None))
        n = np.zeros((cnt, 3), np.int32)
        pix = np.zeros(cnt, np.int32)
        w = np.zeros(cnt, np.float32)
        d = np.zeros(cnt, np.float64)
        pf = np.zeros((cnt, 3), np.float32)
        L.ov_record(self._h, _p(Z), _p(Wk), W, H, _p(it), _p(Rm), _p(tv), cnt, _p(n), _p(pix), _p(w), _p(d), _p(pf))
        return {"n": n, "pix": pix, "w": w, "d": d, "p": pf}

    def voxel_sequence(self, kfs, intr, ops, n):
        """Final (D, W, C, touches) of voxel n after operations ops = [(kf index,
        sign, R, t), ...] applied in order from the empty state (RGBA8 colour)."""
        Z = [_c(k["depth"], np.float32) for k in kfs]
        Wk = [_c(k["weight"], np.float32) for k in kfs]
        C = [_c(k["color"], np.uint8) for k in kfs]
        H, W = Z[0].shape
        PZ = (ctypes.c_void_p * len(kfs))(*[z.ctypes.data for z in Z])
        PW = (ctypes.c_void_p * len(kfs))(*[w.ctypes.data for w in Wk])
        PC = (ctypes.c_void_p * len(kfs))(*[c.ctypes.data for c in C])
        kf = np.array([o[0] for o in ops], np.int32)
        sg = np.array([o[1] for o in ops], np.int32)
        R = np.ascontiguousarray(np.array([o[2] for o in ops], np.float64).reshape(-1, 9))
        t = np.ascontiguousarray(np.array([o[3] for o in ops], np.float64).reshape(-1, 3))
        nn = _c(n, np.int64)
        D = np.zeros(1)
        Wv = np.zeros(1)
        Cv = np.zeros(3)
        rc = lib().ov_voxel_sequence(self._h, PZ, PW, PC, W, H, _p(_intr(intr)), len(ops), _p(kf), _p(sg), _p(R),
                                     _p(t), _p(nn), _p(D), _p(Wv), _p(Cv))
        return float(D[0]), float(Wv[0]), Cv, int(rc)

    def touch_one(self, kf, intr, R, t, n):
        Z = _c(kf["depth"], np.float32)
        Wk = _c(kf["weight"], np.float32)
        H, W = Z.shape
        it = _intr(intr)
        nn = _c(n, np.int64)
        pix = np.zeros(1, np.int32)
        pf = np.zeros(3, np.float32)
        hit = lib().ov_touch_one(self._h, _p(Z), _p(Wk), W, H, _p(it), _p(_c(R, np.float64)), _p(_c(t, np.float64)),
                                 _p(nn), _p(pix), _p(pf))
        return bool(hit), int(pix[0]), pf


# ----------------------------------------------------------------------------
# keyframe fusion
# ----------------------------------------------------------------------------


def depth_weight(Z, intr, z_min=0.3, z_max=4.0, disc_rel=0.05):
    """w_z = cos(theta) Z^-2 on the 2^-10 grid, 0 = rejected (Sec. 3, Keyframe Fusion)."""
    Z = _c(Z, np.float32)
    H, W = Z.shape
    out = np.zeros_like(Z)
    lib().of_depth_weight(_p(Z), W, H, _p(_intr(intr)), z_min, z_max, disc_rel, _p(out))
    return out


def fuse_depth(Z, wz, intr, R, t, ref=0):
    """Eq. (1) over a group of frames -> (Z*, W*)."""
    Z = _c(Z, np.float32)
    wz = _c(wz, np.float32)
    n, H, W = Z.shape
    Zs = np.zeros((H, W), np.float32)
    Ws = np.zeros((H, W), np.float32)
    lib().of_fuse_depth(_p(Z), _p(wz), n, W, H, _p(_intr(intr)), _p(_c(R, np.float64)), _p(_c(t, np.float64)), ref,
                        _p(Zs), _p(Ws))
    return Zs, Ws


def sharpen(rgb):
    """Unsharp mask in units of 1/256 (uint16), Sec. 3 colour fusion."""
    rgb = _c(rgb, np.uint8)
    H, W, _ = rgb.shape
    out = np.zeros((H, W, 3), np.uint16)
    lib().of_sharpen(_p(rgb), W, H, _p(out))
    return out


def blur(rgb):
    """Blur measure in [0,1] and its four integer sums."""
    rgb = _c(rgb, np.uint8)
    H, W, _ = rgb.shape
    sums = np.zeros(4, np.int64)
    b = lib().of_blur(_p(rgb), W, H, _p(sums))
    return float(b), sums


def fuse_color(Z, wz, cs, wb, intr, R, t, Zs, Ws, ref=0, occ_rel=0.05):
    """Weighted-median colour fusion; returns (Z*, W*, RGBA8) with pixels that
    have no valid colour observation invalidated."""
    Z = _c(Z, np.float32)
    n, H, W = Z.shape
    Zs = _c(Zs, np.float32).copy()
    Ws = _c(Ws, np.float32).copy()
    rgba = np.zeros((H, W, 4), np.uint8)
    lib().of_fuse_color(_p(Z), _p(_c(wz, np.float32)), _p(_c(cs, np.uint16)), _p(_c(wb, np.float64)), n, W, H,
                        _p(_intr(intr)), _p(_c(R, np.float64)), _p(_c(t, np.float64)), ref, occ_rel, _p(Zs),
                        _p(Ws), _p(rgba))
    return Zs, Ws, rgba


def kf_fuse(depth, rgb, intr, R, t, ref=0, z_min=0.3, z_max=4.0, disc_rel=0.05, occ_rel=0.05):
    """The whole keyframe fusion of a group of frames (Sec. 3, Keyframe Fusion)."""
    depth = _c(depth, np.float32)
    n = depth.shape[0]
    wz = np.stack([depth_weight(depth[i], intr, z_min, z_max, disc_rel) for i in range(n)])
    Zs, Ws = fuse_depth(depth, wz, intr, R, t, ref)
    cs = np.stack([sharpen(rgb[i]) for i in range(n)])
    wb = np.array([1.0 - blur(rgb[i])[0] for i in range(n)])
    Zs, Ws, rgba = fuse_color(depth, wz, cs, wb, intr, R, t, Zs, Ws, ref, occ_rel)
    return {"depth": Zs, "weight": Ws, "color": rgba, "wz": wz, "wb": wb, "cs": cs}


def threads() -> int:
    return int(lib().ov_threads())


def set_threads(n: int) -> int:
    """Thread count of the oracle's OpenMP loops (for timing); returns it."""
    return int(lib().ov_set_threads(int(n)))
