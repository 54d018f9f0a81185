"""Surface extraction and the surface metrics of Sec. 5 ("Surface evaluation
methods and metrics") over the library's calls: the Marching Cubes mesh of a
volume, its vertices, and the mean absolute deviation of capped
nearest-neighbour distances, CORR (mesh vertices to a reference cloud) and
COMPL (reference vertices to the mesh vertices).  Every step runs in the
library's kernels; this module only marshals tensors."""
from __future__ import annotations

import ctypes

import torch

from . import scsurf


def _dptr(t: torch.Tensor, dtype, what):
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"{what}: expected a contiguous {dtype} device tensor")
    return t.data_ptr() if t.numel() else None


def mesh_table():
    """The library's Marching Cubes case table: per case, a list of
    (edges in loop order, fanned around a centre vertex), and the triangle
    counts."""
    import numpy as np
    loops = np.zeros((256, 16), np.uint8)
    ntri = np.zeros(256, np.uint8)
    scsurf.check(scsurf.lib().sc_mesh_table(loops.ctypes.data, ntri.ctypes.data), "sc_mesh_table")
    out = []
    for c in range(256):
        row, p, cur = loops[c], 0, []
        while p < 16 and row[p]:
            n = int(row[p] & 0x7F)
            cur.append(([int(e) for e in row[p + 1:p + 1 + n]], bool(row[p] & 0x80)))
            p += 1 + n
        out.append(cur)
    return out, ntri.astype(int).tolist()


def mesh_vertices(tri_xyz: torch.Tensor, tri_keys: torch.Tensor, stream=None) -> torch.Tensor:
    """Distinct vertices (V,3) of a triangle soup from `Volume.mesh`."""
    n_tri = int(tri_xyz.shape[0])
    x = tri_xyz.reshape(-1, 3).contiguous()
    k = tri_keys.reshape(-1, 4).contiguous()
    cap = 3 * n_tri
    out = torch.empty((max(cap, 1), 3), dtype=torch.float32, device=tri_xyz.device)
    n = ctypes.c_int64()
    scsurf.check(scsurf.lib().sc_mesh_vertices(_dptr(x, torch.float32, "tri_xyz"), _dptr(k, torch.int32, "tri_keys"),
                                               n_tri, out.data_ptr(), cap, ctypes.byref(n),
                                               scsurf.stream_handle(stream)), "sc_mesh_vertices")
    return out[:n.value]


def nn_distance(ref: torch.Tensor, query: torch.Tensor, radius: float, stream=None):
    """(distances (Q,) f32, their FP64 sum) from every query point to its
    nearest reference point, capped at `radius`."""
    ref = ref.reshape(-1, 3).contiguous()
    query = query.reshape(-1, 3).contiguous()
    dist = torch.empty(max(query.shape[0], 1), dtype=torch.float32, device=query.device)
    total = torch.zeros(1, dtype=torch.float64, device=query.device)
    scsurf.check(scsurf.lib().sc_nn_distance(_dptr(ref, torch.float32, "ref"), ref.shape[0],
                                             _dptr(query, torch.float32, "query"), query.shape[0], float(radius),
                                             dist.data_ptr(), total.data_ptr(), scsurf.stream_handle(stream)),
                 "sc_nn_distance")
    return dist[:query.shape[0]], float(total.item())


def corr(mesh_vertices: torch.Tensor, reference: torch.Tensor, radius: float, stream=None) -> float:
    """CORR: mean distance from the mesh vertices to the reference cloud."""
    n = mesh_vertices.reshape(-1, 3).shape[0]
    return nn_distance(reference, mesh_vertices, radius, stream)[1] / n if n else 0.0


def compl(reference_vertices: torch.Tensor, mesh_vertices: torch.Tensor, radius: float, stream=None) -> float:
    """COMPL: mean distance from the reference vertices to the mesh vertices."""
    n = reference_vertices.reshape(-1, 3).shape[0]
    return nn_distance(mesh_vertices, reference_vertices, radius, stream)[1] / n if n else 0.0
