"""Thin Python binding of libscsurf (C ABI in include/scsurf.h).

Argument marshalling only: torch supplies device memory and streams, every
step of the hot path runs in the library's HIP kernels.  The binding fails
loudly when the library is missing or the device is not gfx950; there is no
fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libscsurf.so")

SC_OK, SC_EINVAL, SC_ENOMEM, SC_EHASHFULL, SC_EPOOLFULL, SC_ENOTALLOC, SC_EWEIGHT, SC_EDEVICE, SC_ENOLIB = (
    0, -1, -2, -3, -4, -5, -6, -7, -8)
SC_ERANGE, SC_ESCRATCH = -9, -10
STATUS = {0: "SC_OK", -1: "SC_EINVAL", -2: "SC_ENOMEM", -3: "SC_EHASHFULL", -4: "SC_EPOOLFULL",
          -5: "SC_ENOTALLOC", -6: "SC_EWEIGHT", -7: "SC_EDEVICE", -8: "SC_ENOLIB", -9: "SC_ERANGE",
          -10: "SC_ESCRATCH"}
COLOR_RGBA8, COLOR_F32 = 0, 1
SEL_EQ3, SEL_TOPM, SEL_ALL_ORDERED = 0, 1, 2


class ScError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {STATUS.get(status, status)}")
        self.status = status


class sc_intrinsics(ctypes.Structure):
    _fields_ = [("fx", ctypes.c_float), ("fy", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32)]


class sc_pose(ctypes.Structure):
    _fields_ = [("R", ctypes.c_double * 9), ("t", ctypes.c_double * 3)]


class sc_volume_params(ctypes.Structure):
    _fields_ = [("voxel_size", ctypes.c_float), ("trunc", ctypes.c_float), ("n_buckets", ctypes.c_int64),
                ("max_blocks", ctypes.c_int64), ("color_mode", ctypes.c_int32), ("max_batch_ops", ctypes.c_int32)]


class sc_keyframe(ctypes.Structure):
    _fields_ = [("depth", ctypes.c_void_p), ("weight", ctypes.c_void_p), ("color", ctypes.c_void_p),
                ("packed", ctypes.c_void_p)]


class sc_fuse_params(ctypes.Structure):
    _fields_ = [("z_min", ctypes.c_float), ("z_max", ctypes.c_float), ("disc_rel", ctypes.c_float),
                ("occ_rel", ctypes.c_float)]


class sc_schedule(ctypes.Structure):
    _fields_ = [("vpl", ctypes.c_int32), ("waves_per_wg", ctypes.c_int32), ("wgs_per_cu", ctypes.c_int32),
                ("compact", ctypes.c_int32)]


EXPORTS = ["sc_version", "sc_volume_create", "sc_volume_destroy", "sc_volume_reset", "sc_volume_query",
           "sc_volume_export", "sc_depth_weight", "sc_color_prep", "kf_fuse", "kf_fuse_noalloc", "hash_alloc", "tsdf_integrate",
           "tsdf_integrate_batch",
           "tsdf_deintegrate", "sc_select", "sc_select_dist", "sc_relative_motion", "reintegrate_batch",
           "reintegrate_plain",
           "sc_set_schedule", "sc_get_schedule", "sc_autotune", "sc_autotune_clear", "sc_batch_timing", "sc_batch_timing_read",
           "sc_volume_stats", "tsdf_integrate_backward", "sc_keyframe_pack", "sc_keyframe_pack_bytes", "sc_overlap",
           "sc_volume_mesh", "sc_mesh_vertices", "sc_nn_distance", "sc_mesh_table",
           "sc_volume_import", "sc_stream_enable", "sc_stream_out", "sc_stream_in_all", "sc_stream_stats",
           "sc_stream_export"]

_lib = None


def lib():
    """Loads libscsurf.so (built in-tree by __graft_entry__.build())."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libscsurf.so is not built ({LIB_PATH}); run __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    P, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    L.sc_version.restype = ctypes.c_char_p
    L.sc_volume_create.argtypes = [ctypes.POINTER(sc_volume_params), ctypes.POINTER(P)]
    L.sc_volume_destroy.argtypes = [P]
    L.sc_volume_destroy.restype = None
    L.sc_volume_reset.argtypes = [P, P]
    L.sc_volume_query.argtypes = [P, P, ctypes.POINTER(i64), ctypes.POINTER(i32)]
    L.sc_volume_export.argtypes = [P, P, P, P, P, P, i64, ctypes.POINTER(i64)]
    L.sc_depth_weight.argtypes = [P, i32, ctypes.POINTER(sc_intrinsics), ctypes.POINTER(sc_fuse_params), P, P]
    L.sc_color_prep.argtypes = [P, i32, i32, i32, P, P, P]
    for f in (L.kf_fuse, L.kf_fuse_noalloc):
        f.argtypes = [P, P, ctypes.POINTER(sc_pose), i32, i32, ctypes.POINTER(sc_intrinsics),
                      ctypes.POINTER(sc_fuse_params), P, P, P, P]
    L.hash_alloc.argtypes = [P, P, i64, P, P]
    for f in (L.tsdf_integrate, L.tsdf_deintegrate):
        f.argtypes = [P, ctypes.POINTER(sc_keyframe), ctypes.POINTER(sc_intrinsics), ctypes.POINTER(sc_pose), P]
    L.sc_select.argtypes = [ctypes.POINTER(sc_pose), ctypes.POINTER(sc_pose), i32, i32, i32, P, P]
    L.sc_select_dist.argtypes = [P, i32, i32, i32, P]
    L.sc_stream_enable.argtypes = [P, i32]
    L.sc_stream_out.argtypes = [P, P, ctypes.c_double, P]
    L.sc_stream_in_all.argtypes = [P, P]
    L.sc_stream_stats.argtypes = [P, P, P]
    L.sc_stream_export.argtypes = [P, P, P, P, P, i64, ctypes.POINTER(i64)]
    L.sc_relative_motion.argtypes = [ctypes.POINTER(sc_pose), ctypes.POINTER(sc_pose), ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_double)]
    for f in (L.reintegrate_batch, L.reintegrate_plain):
        f.argtypes = [P, ctypes.POINTER(sc_keyframe), i32, ctypes.POINTER(sc_intrinsics), ctypes.POINTER(sc_pose),
                      ctypes.POINTER(sc_pose), i32, i32, P, ctypes.POINTER(i32), P]
    L.sc_set_schedule.argtypes = [P, ctypes.POINTER(sc_schedule)]
    L.sc_get_schedule.argtypes = [P, ctypes.POINTER(sc_schedule)]
    L.sc_autotune.argtypes = [P, ctypes.POINTER(sc_keyframe), i32, ctypes.POINTER(sc_intrinsics),
                              ctypes.POINTER(sc_pose), ctypes.POINTER(sc_pose), i32, i32, ctypes.POINTER(sc_schedule),
                              ctypes.POINTER(ctypes.c_float), P]
    L.sc_autotune_clear.argtypes = []
    L.sc_autotune_clear.restype = None
    L.sc_batch_timing.argtypes = [P, i32]
    L.sc_batch_timing_read.argtypes = [P, P, ctypes.POINTER(i32)]
    L.sc_volume_stats.argtypes = [P, P, P]
    L.sc_keyframe_pack.argtypes = [ctypes.POINTER(sc_keyframe), i32, i32, P, i64, P]
    L.sc_keyframe_pack_bytes.argtypes = [i32, i32]
    L.sc_keyframe_pack_bytes.restype = i64
    L.sc_overlap.argtypes = [P, ctypes.POINTER(sc_intrinsics), ctypes.POINTER(sc_pose), ctypes.POINTER(sc_pose),
                             ctypes.c_float, ctypes.c_float, P, P]
    L.sc_volume_mesh.argtypes = [P, P, P, P, i64, ctypes.POINTER(i64)]
    L.sc_mesh_vertices.argtypes = [P, P, i64, P, i64, ctypes.POINTER(i64), P]
    L.sc_nn_distance.argtypes = [P, i64, P, i64, ctypes.c_float, P, P, P]
    L.sc_mesh_table.argtypes = [P, P]
    L.sc_volume_import.argtypes = [P, P, P, P, P, P, i64]
    L.tsdf_integrate_backward.argtypes = [P, ctypes.POINTER(sc_keyframe), i32, ctypes.POINTER(sc_intrinsics),
                                          ctypes.POINTER(sc_pose), P, P, P, P, P, P, P, P]
    for name in EXPORTS:
        if name != "sc_version" and name != "sc_volume_destroy":
            getattr(L, name).restype = i32
    _lib = L
    return L


def check(status: int, what: str):
    if status != SC_OK:
        raise ScError(status, what)


# ----------------------------------------------------------------------------
# marshalling helpers
# ----------------------------------------------------------------------------


def stream_handle(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def dptr(t: torch.Tensor, dtype=None, what="tensor") -> int:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{what} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{what} must be {dtype}, got {t.dtype}")
    return t.data_ptr()


def _check_shape(t: torch.Tensor, shape, what: str):
    """The library takes plain pointers and sizes: shapes are checked here,
    before a kernel could read past a buffer."""
    if tuple(t.shape) != tuple(int(x) for x in shape):
        raise ValueError(f"{what} must have shape {tuple(shape)}, got {tuple(t.shape)}")


def _image_size(intr):
    return int(intr.height), int(intr.width)


def intrinsics(intr) -> sc_intrinsics:
    return sc_intrinsics(float(intr.fx), float(intr.fy), float(intr.cx), float(intr.cy), int(intr.width),
                         int(intr.height))


def pose(R, t) -> sc_pose:
    p = sc_pose()
    p.R[:] = [float(x) for x in np.asarray(R, np.float64).reshape(9)]
    p.t[:] = [float(x) for x in np.asarray(t, np.float64).reshape(3)]
    return p


def poses(R, t):
    """(N,3,3) rotations and (N,3) translations -> ctypes sc_pose array (one
    copy through a contiguous (N,12) buffer)."""
    R = np.asarray(R, np.float64).reshape(-1, 9)
    t = np.asarray(t, np.float64).reshape(-1, 3)
    buf = np.ascontiguousarray(np.concatenate([R, t], axis=1))
    arr = (sc_pose * len(buf)).from_buffer_copy(buf.tobytes())
    return arr


def poses_to_numpy(arr):
    buf = np.frombuffer(arr, dtype=np.float64).reshape(len(arr), 12)
    return buf[:, :9].reshape(-1, 3, 3).copy(), buf[:, 9:].copy()


@dataclass
class Keyframe:
    """A fused keyframe on the device: depth Z* (H,W) f32, weight W* (H,W) f32,
    colour RGBA8 (H,W,4) u8 or F32 (H,W,3) f32."""
    depth: torch.Tensor
    weight: torch.Tensor
    color: torch.Tensor
    packed: Optional[torch.Tensor] = None  # (H,W,4) int32 interleaved copy from keyframe_pack

    def image_size(self):
        """(H, W) after checking that the keyframe's tensors agree."""
        if self.depth.dim() != 2:
            raise ValueError("keyframe depth must be (H, W)")
        H, W = (int(x) for x in self.depth.shape)
        _check_shape(self.weight, (H, W), "keyframe weight")
        if self.color.dtype == torch.uint8:
            _check_shape(self.color, (H, W, 4), "RGBA8 keyframe colour")
        elif self.color.dtype == torch.float32:
            _check_shape(self.color, (H, W, 3), "FP32 keyframe colour")
        else:
            raise ValueError("keyframe colour must be uint8 (H, W, 4) or float32 (H, W, 3)")
        if self.packed is not None:
            _check_shape(self.packed, (H, W, 4), "packed keyframe")
            # the cell depth ranges must follow the records in the same storage
            have = self.packed.untyped_storage().nbytes() - 4 * self.packed.storage_offset()
            if not self.packed.is_contiguous() or have < int(lib().sc_keyframe_pack_bytes(W, H)):
                raise ValueError("packed keyframe: not a buffer written by keyframe_pack (cell ranges missing)")
        return H, W

    def c(self) -> sc_keyframe:
        packed = None if self.packed is None else dptr(self.packed, torch.int32, "packed")
        return sc_keyframe(dptr(self.depth, torch.float32, "depth"), dptr(self.weight, torch.float32, "weight"),
                           dptr(self.color, None, "color"), packed)


class KeyframeSet:
    """A fixed list of keyframes marshalled once for repeated updates: holds
    the ctypes array of their device pointers and references to the tensors
    (so they stay alive).  Rebuild it if a keyframe's tensors are replaced."""

    def __init__(self, kfs):
        self.kfs = list(kfs)
        sizes = {k.image_size() for k in self.kfs}
        kinds = {k.color.dtype for k in self.kfs}
        if len(sizes) > 1 or len(kinds) > 1:
            raise ValueError("the keyframes of one call must share their image size and colour type")
        self.size = sizes.pop() if sizes else None
        self.color_dtype = kinds.pop() if kinds else None
        self.arr = (sc_keyframe * len(self.kfs))()
        for i, k in enumerate(self.kfs):
            self.arr[i] = k.c()

    def __len__(self):
        return len(self.kfs)


def keyframes(kfs) -> KeyframeSet:
    return kfs if isinstance(kfs, KeyframeSet) else KeyframeSet(kfs)


def fuse_params(z_min=0.3, z_max=4.0, disc_rel=0.05, occ_rel=0.05) -> sc_fuse_params:
    return sc_fuse_params(z_min, z_max, disc_rel, occ_rel)


# ----------------------------------------------------------------------------
# API
# ----------------------------------------------------------------------------


def version() -> str:
    return lib().sc_version().decode()


class Volume:
    """Voxel-hashed TSDF owned by the library (Sec. 3, SDF volume)."""

    def __init__(self, voxel_size: float, trunc: float, n_buckets: int, max_blocks: int, color_mode: int = COLOR_RGBA8,
                 max_batch_ops: int = 512):
        self.params = sc_volume_params(voxel_size, trunc, n_buckets, max_blocks, color_mode, max_batch_ops)
        self.color_mode = color_mode
        self._h = ctypes.c_void_p()
        check(lib().sc_volume_create(ctypes.byref(self.params), ctypes.byref(self._h)), "sc_volume_create")

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().sc_volume_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def reset(self, stream=None):
        check(lib().sc_volume_reset(self._h, stream_handle(stream)), "sc_volume_reset")

    def query(self, stream=None):
        n = ctypes.c_int64()
        e = ctypes.c_int32()
        check(lib().sc_volume_query(self._h, stream_handle(stream), ctypes.byref(n), ctypes.byref(e)),
              "sc_volume_query")
        return int(n.value), int(e.value)

    def export(self, stream=None):
        """Allocated blocks in pool order: dict of device tensors."""
        n, _ = self.query(stream)
        dev = torch.device("cuda")
        xyz = torch.empty((max(n, 1), 3), dtype=torch.int32, device=dev)
        D = torch.empty((max(n, 1), 512), dtype=torch.float32, device=dev)
        W = torch.empty((max(n, 1), 512), dtype=torch.float32, device=dev)
        if self.color_mode == COLOR_RGBA8:
            C = torch.empty((max(n, 1), 512, 4), dtype=torch.uint8, device=dev)
        else:
            C = torch.empty((max(n, 1), 3, 512), dtype=torch.float32, device=dev)
        nout = ctypes.c_int64()
        check(lib().sc_volume_export(self._h, stream_handle(stream), xyz.data_ptr(), D.data_ptr(), W.data_ptr(),
                                     C.data_ptr(), n, ctypes.byref(nout)), "sc_volume_export")
        return {"blocks": xyz[:n], "D": D[:n], "W": W[:n], "C": C[:n]}

    def import_field(self, field, stream=None):
        """Loads blocks {"blocks" (n,3) int32, "D" (n,512) f32, "W" (n,512) f32,
        optional "C" (n,512,4) uint8 or (n,3,512) f32} given as device
        tensors, in the layout `export` returns."""
        xyz = field["blocks"].to(torch.int32).contiguous()
        n = int(xyz.shape[0])
        D = field["D"].to(torch.float32).contiguous()
        W = field["W"].to(torch.float32).contiguous()
        C = field.get("C")
        if C is not None:
            C = C.contiguous()
        if xyz.dim() != 2 or xyz.shape[1] != 3:
            raise ValueError("blocks must be (n, 3)")
        if D.shape != (n, 512) or W.shape != (n, 512):
            raise ValueError("D and W must be (n, 512)")
        if C is not None:
            if self.color_mode == COLOR_RGBA8:
                if C.dtype != torch.uint8:
                    raise ValueError("RGBA8 colour must be uint8")
                _check_shape(C, (n, 512, 4), "C")
            else:
                if C.dtype != torch.float32:
                    raise ValueError("FP32 colour must be float32")
                _check_shape(C, (n, 3, 512), "C")
        check(lib().sc_volume_import(self._h, stream_handle(stream), xyz.data_ptr() if n else None,
                                     D.data_ptr() if n else None, W.data_ptr() if n else None,
                                     C.data_ptr() if (C is not None and n) else None, n), "sc_volume_import")

    def mesh(self, stream=None):
        """Marching Cubes of the volume: (tri_xyz (T,3,3) f32, tri_keys
        (T,3,4) int32) device tensors, triangles in the library's fixed order
        (blocks in pool order, cubes in voxel order)."""
        n = ctypes.c_int64()
        check(lib().sc_volume_mesh(self._h, stream_handle(stream), None, None, 0, ctypes.byref(n)), "sc_volume_mesh")
        T = n.value
        dev = torch.device("cuda")
        xyz = torch.empty((max(T, 1), 3, 3), dtype=torch.float32, device=dev)
        keys = torch.empty((max(T, 1), 3, 4), dtype=torch.int32, device=dev)
        check(lib().sc_volume_mesh(self._h, stream_handle(stream), xyz.data_ptr(), keys.data_ptr(), T,
                                   ctypes.byref(n)), "sc_volume_mesh")
        if n.value != T:
            raise ScError(SC_EDEVICE, "sc_volume_mesh: triangle count changed between calls")
        return xyz[:T], keys[:T]

    def stream_export(self):
        """Blocks held by the host store (streaming mode): dict of NumPy
        arrays in export's layout."""
        n = ctypes.c_int64()
        check(lib().sc_stream_export(self._h, None, None, None, None, 0, ctypes.byref(n)), "sc_stream_export")
        m = int(n.value)
        xyz = np.zeros((m, 3), np.int32)
        D = np.zeros((m, 512), np.float32)
        W = np.zeros((m, 512), np.float32)
        C = np.zeros((m, 512, 4), np.uint8) if self.color_mode == COLOR_RGBA8 else np.zeros((m, 3, 512), np.float32)
        check(lib().sc_stream_export(self._h, xyz.ctypes.data, D.ctypes.data, W.ctypes.data, C.ctypes.data, m,
                                     ctypes.byref(n)), "sc_stream_export")
        return {"blocks": xyz, "D": D, "W": W, "C": C}

    def export_sorted(self, stream=None, with_host=False):
        """Allocated blocks sorted by (x, y, z) as NumPy arrays; colour as
        (n, 512, 3) in RGB order.  with_host: also the blocks the host store
        holds (streaming mode), i.e. the whole field."""
        f = {k: v.cpu().numpy() for k, v in self.export(stream).items()}
        if with_host:
            h = self.stream_export()
            f = {k: np.concatenate([f[k], h[k]]) for k in f}
        b = f["blocks"].astype(np.int64)
        order = np.lexsort((b[:, 2], b[:, 1], b[:, 0]))
        C = f["C"][order]
        C = C[..., :3] if self.color_mode == COLOR_RGBA8 else np.transpose(C, (0, 2, 1))
        return {"blocks": b[order], "D": f["D"][order], "W": f["W"][order], "C": C}

    def check_error(self, stream=None):
        n, e = self.query(stream)
        check(e, "device error")
        return n

    def _check_keyframes(self, kset: KeyframeSet, intr, *pose_sets):
        """Keyframe images of the intrinsics' size, colour of the volume's
        mode, one pose per keyframe in each pose array."""
        if kset.size is not None and kset.size != _image_size(intr):
            raise ValueError(f"keyframes are {kset.size}, the intrinsics say {_image_size(intr)}")
        want = torch.uint8 if self.color_mode == COLOR_RGBA8 else torch.float32
        if kset.color_dtype is not None and kset.color_dtype != want:
            raise ValueError(f"this volume takes {want} keyframe colour, got {kset.color_dtype}")
        for ps in pose_sets:
            if len(ps) != len(kset):
                raise ValueError(f"{len(ps)} poses for {len(kset)} keyframes")

    def integrate(self, kf: Keyframe, intr, R, t, stream=None):
        self._check_keyframes(KeyframeSet([kf]), intr)
        k = kf.c()
        check(lib().tsdf_integrate(self._h, ctypes.byref(k), ctypes.byref(intrinsics(intr)), ctypes.byref(pose(R, t)),
                                   stream_handle(stream)), "tsdf_integrate")

    def integrate_batch(self, kfs, intr, R, t, stream=None):
        """Integrates keyframes at poses (R (n,3,3), t (n,3)) in order, in one
        batched pass: the same volume as integrate() called on each in turn."""
        kset = keyframes(kfs)
        T = poses(R, t)
        self._check_keyframes(kset, intr, T)
        check(lib().tsdf_integrate_batch(self._h, kset.arr, len(kset), ctypes.byref(intrinsics(intr)), T,
                                         stream_handle(stream)), "tsdf_integrate_batch")

    def deintegrate(self, kf: Keyframe, intr, R, t, stream=None):
        self._check_keyframes(KeyframeSet([kf]), intr)
        k = kf.c()
        check(lib().tsdf_deintegrate(self._h, ctypes.byref(k), ctypes.byref(intrinsics(intr)),
                                     ctypes.byref(pose(R, t)), stream_handle(stream)), "tsdf_deintegrate")

    def hash_alloc(self, block_xyz: torch.Tensor, want_slots=True, stream=None):
        if block_xyz.dim() != 2 or block_xyz.shape[1] != 3:
            raise ValueError("block_xyz must be (n, 3)")
        n = block_xyz.shape[0]
        slots = torch.empty(n, dtype=torch.int32, device=block_xyz.device) if want_slots else None
        check(lib().hash_alloc(self._h, dptr(block_xyz, torch.int32, "block_xyz"), n,
                               slots.data_ptr() if slots is not None else None, stream_handle(stream)), "hash_alloc")
        return slots

    def _reint(self, fn, kfs, intr, T_int, T_new, m, mode, stream):
        kset = keyframes(kfs)
        Ti = poses(*T_int)
        Tn = poses(*T_new)
        self._check_keyframes(kset, intr, Ti, Tn)
        karr = kset.arr
        sel = (ctypes.c_int32 * len(kfs))()
        ns = ctypes.c_int32()
        check(fn(self._h, karr, len(kfs), ctypes.byref(intrinsics(intr)), Ti, Tn, m, mode, sel, ctypes.byref(ns),
                 stream_handle(stream)), fn.__name__)
        R, t = poses_to_numpy(Ti)
        return list(sel[:ns.value]), (R, t)

    def reintegrate_batch(self, kfs, intr, T_int, T_new, m, mode=SEL_EQ3, stream=None):
        """One pose-graph update, batched.  Returns (processing order, updated
        integration poses (R, t))."""
        return self._reint(lib().reintegrate_batch, kfs, intr, T_int, T_new, m, mode, stream)

    def reintegrate_plain(self, kfs, intr, T_int, T_new, m, mode=SEL_EQ3, stream=None):
        return self._reint(lib().reintegrate_plain, kfs, intr, T_int, T_new, m, mode, stream)

    def set_schedule(self, vpl, waves_per_wg, wgs_per_cu, compact=0):
        s = sc_schedule(vpl, waves_per_wg, wgs_per_cu, compact)
        check(lib().sc_set_schedule(self._h, ctypes.byref(s)), "sc_set_schedule")

    def get_schedule(self):
        s = sc_schedule()
        check(lib().sc_get_schedule(self._h, ctypes.byref(s)), "sc_get_schedule")
        return (s.vpl, s.waves_per_wg, s.wgs_per_cu, s.compact)

    def autotune(self, kfs, intr, T_int, T_new, m, mode=SEL_EQ3, stream=None):
        kset = keyframes(kfs)
        Ti, Tn = poses(*T_int), poses(*T_new)
        self._check_keyframes(kset, intr, Ti, Tn)
        best = sc_schedule()
        ms = ctypes.c_float()
        check(lib().sc_autotune(self._h, kset.arr, len(kfs), ctypes.byref(intrinsics(intr)), Ti, Tn, m, mode,
                                ctypes.byref(best), ctypes.byref(ms), stream_handle(stream)), "sc_autotune")
        return (best.vpl, best.waves_per_wg, best.wgs_per_cu, best.compact), float(ms.value)

    @staticmethod
    def autotune_clear():
        """Empties the process's autotuning cache."""
        lib().sc_autotune_clear()

    def batch_timing(self, capacity: int):
        """Record HIP events around the voxel pass of the next `capacity` batched launches."""
        self._timing_cap = capacity
        check(lib().sc_batch_timing(self._h, capacity), "sc_batch_timing")

    def batch_timing_read(self):
        cap = max(getattr(self, "_timing_cap", 0), 1)
        ms = (ctypes.c_float * cap)()
        n = ctypes.c_int32()
        check(lib().sc_batch_timing_read(self._h, ms, ctypes.byref(n)), "sc_batch_timing_read")
        return list(ms[:n.value])

    def stream_enable(self, enable=True):
        """Streaming mode (Sec. 3): operations stream in the host-held blocks
        among their candidates before running."""
        check(lib().sc_stream_enable(self._h, int(bool(enable))), "sc_stream_enable")

    def stream_out(self, center, radius: float, stream=None):
        """Moves the device blocks outside the sphere (center, radius) to the
        host store."""
        c = (ctypes.c_double * 3)(*[float(x) for x in np.asarray(center, np.float64).reshape(3)])
        check(lib().sc_stream_out(self._h, c, float(radius), stream_handle(stream)), "sc_stream_out")

    def stream_in_all(self, stream=None):
        check(lib().sc_stream_in_all(self._h, stream_handle(stream)), "sc_stream_in_all")

    def stream_stats(self, stream=None):
        """(device blocks, host blocks, blocks out, blocks in, bytes out, bytes in)."""
        out = (ctypes.c_int64 * 6)()
        check(lib().sc_stream_stats(self._h, stream_handle(stream), out), "sc_stream_stats")
        return tuple(int(x) for x in out)

    def stats(self, stream=None):
        """(candidate blocks, block-operation pairs, voxel updates, blocks written), cumulative."""
        out = (ctypes.c_int64 * 4)()
        check(lib().sc_volume_stats(self._h, stream_handle(stream), out), "sc_volume_stats")
        return tuple(int(x) for x in out)

    def integrate_backward(self, kfs, intr, R, t, grad_D, grad_C, grad_depth, grad_color, grad_xi, grad_D0=None,
                           grad_C0=None, stream=None):
        """Adjoint of integrating `kfs` at (R, t) into the field the volume
        holds (see tsdf_integrate_backward): accumulates into grad_depth,
        grad_color and grad_xi; writes grad_D0 / grad_C0 (pool order) if
        given."""
        kset = keyframes(kfs)
        T = poses(R, t)
        self._check_keyframes(kset, intr, T)
        n_blocks, _ = self.query(stream)
        H, W = _image_size(intr)
        _check_shape(grad_D, (n_blocks, 512), "grad_D")
        if grad_C is not None:
            _check_shape(grad_C, (n_blocks, 3, 512), "grad_C")
        _check_shape(grad_depth, (len(kset), H, W), "grad_depth")
        if grad_color is not None:
            _check_shape(grad_color, (len(kset), H, W, 3), "grad_color")
        _check_shape(grad_xi, (len(kset), 6), "grad_xi")
        if grad_D0 is not None:
            _check_shape(grad_D0, (n_blocks, 512), "grad_D0")
        if grad_C0 is not None:
            _check_shape(grad_C0, (n_blocks, 3, 512), "grad_C0")

        def opt(x, what):
            return dptr(x, torch.float32, what) if x is not None else None

        check(lib().tsdf_integrate_backward(
            self._h, kset.arr, len(kset), ctypes.byref(intrinsics(intr)), T, dptr(grad_D, torch.float32, "grad_D"),
            opt(grad_C, "grad_C"), dptr(grad_depth, torch.float32, "grad_depth"), opt(grad_color, "grad_color"),
            dptr(grad_xi, torch.float32, "grad_xi"), opt(grad_D0, "grad_D0"), opt(grad_C0, "grad_C0"),
            stream_handle(stream)), "tsdf_integrate_backward")


def relative_motion(R_kf, t_kf, R, t):
    """(translation norm, rotation angle in radians) of T_kf^-1 T, computed by
    the library (the distance keyframe strategy, Sec. 4.2)."""
    tr, ang = ctypes.c_double(), ctypes.c_double()
    check(lib().sc_relative_motion(ctypes.byref(pose(R_kf, t_kf)), ctypes.byref(pose(R, t)), ctypes.byref(tr),
                                   ctypes.byref(ang)), "sc_relative_motion")
    return float(tr.value), float(ang.value)


def select(T_int, T_new, m, mode=SEL_EQ3):
    """Host selection (Sec. 4.3): (processing order, distances)."""
    Ti = poses(*T_int)
    Tn = poses(*T_new)
    K = len(Ti)
    out = (ctypes.c_int32 * max(K, 1))()
    dist = (ctypes.c_double * max(K, 1))()
    n = lib().sc_select(Ti, Tn, K, m, mode, out, dist)
    if n < 0:
        raise ScError(n, "sc_select")
    return list(out[:n]), np.array(dist[:K])


def select_dist(dist, m, mode=SEL_EQ3):
    d = np.ascontiguousarray(dist, np.float64)
    K = len(d)
    out = (ctypes.c_int32 * max(K, 1))()
    n = lib().sc_select_dist(d.ctypes.data_as(ctypes.c_void_p), K, m, mode, out)
    if n < 0:
        raise ScError(n, "sc_select_dist")
    return list(out[:n])


def keyframe_pack(kf: Keyframe, stream=None) -> Keyframe:
    """The keyframe with its interleaved {depth', q(weight), RGBA8, 0} copy
    attached (RGBA8 keyframes; the voxel passes then gather from it): the
    weight quantised to 2^-10 and the depth replaced by -inf where that weight
    is not positive."""
    H, W = kf.depth.shape
    if kf.color.dtype != torch.uint8 or tuple(kf.color.shape) != (H, W, 4):
        raise ValueError("keyframe_pack needs an RGBA8 keyframe")
    nbytes = int(lib().sc_keyframe_pack_bytes(W, H))
    if nbytes <= 0:
        raise ValueError(f"keyframe size {W} x {H} outside 1 .. 16384")
    buf = torch.empty(nbytes // 4, dtype=torch.int32, device=kf.depth.device)
    check(lib().sc_keyframe_pack(ctypes.byref(kf.c()), W, H, buf.data_ptr(), nbytes, stream_handle(stream)),
          "sc_keyframe_pack")
    # the records as an (H, W, 4) view; the cell ranges follow them in `buf`
    return Keyframe(kf.depth, kf.weight, kf.color, buf[:H * W * 4].view(H, W, 4))


def overlap(depth: torch.Tensor, intr, R, t, R_ref, t_ref, z_min=0.3, z_max=4.0, stream=None):
    """(valid, visible) pixel counts of a frame's depth against a reference
    view (the overlap strategy of Sec. 4.2).  Synchronises."""
    if depth.numel() != int(intr.width) * int(intr.height):
        raise ValueError(f"depth has {depth.numel()} pixels, the intrinsics say {intr.width} x {intr.height}")
    counts = torch.empty(2, dtype=torch.int32, device=depth.device)
    check(lib().sc_overlap(dptr(depth, torch.float32, "depth"), ctypes.byref(intrinsics(intr)),
                           ctypes.byref(pose(R, t)), ctypes.byref(pose(R_ref, t_ref)), float(z_min), float(z_max),
                           counts.data_ptr(), stream_handle(stream)), "sc_overlap")
    c = counts.cpu().numpy()
    return int(c[0]), int(c[1])


def depth_weight(depth: torch.Tensor, intr, params=None, stream=None) -> torch.Tensor:
    depth = depth if depth.dim() == 3 else depth[None]
    _check_shape(depth, (depth.shape[0],) + _image_size(intr), "depth")
    out = torch.empty_like(depth)
    p = params or fuse_params()
    check(lib().sc_depth_weight(dptr(depth, torch.float32, "depth"), depth.shape[0], ctypes.byref(intrinsics(intr)),
                                ctypes.byref(p), out.data_ptr(), stream_handle(stream)), "sc_depth_weight")
    return out


def color_prep(rgb: torch.Tensor, stream=None):
    rgb = rgb if rgb.dim() == 4 else rgb[None]
    if rgb.dim() != 4 or rgb.shape[3] != 3:
        raise ValueError("rgb must be (n, H, W, 3) or (H, W, 3)")
    n, H, W, _ = rgb.shape
    sharp = torch.empty((n, H, W, 3), dtype=torch.uint16, device=rgb.device)
    wb = torch.empty(n, dtype=torch.float64, device=rgb.device)
    check(lib().sc_color_prep(dptr(rgb, torch.uint8, "rgb"), n, W, H, sharp.data_ptr(), wb.data_ptr(),
                              stream_handle(stream)), "sc_color_prep")
    return sharp, wb


def _fuse(entry: str, depth: torch.Tensor, rgb: torch.Tensor, R, t, intr, params, ref, stream, out) -> Keyframe:
    if depth.dim() != 3:
        raise ValueError("depth must be (n, H, W)")
    n, H, W = depth.shape
    _check_shape(depth, (n,) + _image_size(intr), "depth")
    _check_shape(rgb, (n, H, W, 3), "rgb")
    T = poses(R, t)
    if len(T) != n:
        raise ValueError(f"{len(T)} poses for {n} frames")
    dev = depth.device
    if out is None:
        out = Keyframe(torch.empty((H, W), dtype=torch.float32, device=dev),
                       torch.empty((H, W), dtype=torch.float32, device=dev),
                       torch.empty((H, W, 4), dtype=torch.uint8, device=dev))
    _check_shape(out.depth, (H, W), "out.depth")
    _check_shape(out.weight, (H, W), "out.weight")
    _check_shape(out.color, (H, W, 4), "out.color")
    p = params or fuse_params()
    check(getattr(lib(), entry)(dptr(depth, torch.float32, "depth"), dptr(rgb, torch.uint8, "rgb"), T, n, ref,
                                ctypes.byref(intrinsics(intr)), ctypes.byref(p),
                                dptr(out.depth, torch.float32, "out.depth"),
                                dptr(out.weight, torch.float32, "out.weight"),
                                dptr(out.color, torch.uint8, "out.color"), stream_handle(stream)), entry)
    return out


def kf_fuse(depth: torch.Tensor, rgb: torch.Tensor, R, t, intr, params=None, ref=0, stream=None, out=None) -> Keyframe:
    """Fuses frames (n,H,W) / (n,H,W,3) at poses (R, t) into one keyframe."""
    return _fuse("kf_fuse", depth, rgb, R, t, intr, params, ref, stream, out)


def kf_fuse_noalloc(depth: torch.Tensor, rgb: torch.Tensor, R, t, intr, params=None, ref=0, stream=None,
                    out=None) -> Keyframe:
    """kf_fuse whose library side allocates nothing (fixed per-device
    scratch); pass `out` (a Keyframe of preallocated tensors) for a call that
    allocates nothing on the Python side either."""
    return _fuse("kf_fuse_noalloc", depth, rgb, R, t, intr, params, ref, stream, out)
