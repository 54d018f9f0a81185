"""Iso-surface extraction and surface metrics — test infrastructure (the oracle).

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline may use this
module; the product path never does.

* Marching Cubes (Sec. 3 "SDF volume": the iso-surface of the SDF volume is
  extracted with Marching Cubes).  The cube of voxel n has corners
  n + (k & 1, (k >> 1) & 1, (k >> 2) & 1), k = 0..7; a cube is meshed only
  when all eight corner voxels are allocated and observed (W > 0).  A corner
  is inside when D < 0 (behind the surface).  Edge e = 4 a + o1 + 2 o2 runs
  along axis a from the corner whose offsets on the other two axes (in
  increasing axis order) are (o1, o2).  The vertex on an edge from its lower
  corner p (D0) to its upper corner q (D1) is p + t e_a with
  t = D0 / (D0 - D1), in voxel units, scaled by the voxel size, in FP64.
  The case table is derived from a rule, not copied: on every face, seen
  from outside the cube with its corners in counter-clockwise order, each
  run of inside corners is cut off by one segment from the edge where the
  walk enters the run to the edge where it leaves it (so two diagonal inside
  corners of a face stay separate, the same on both cubes sharing the face,
  which keeps the surface closed).  Segments chain across faces into loops,
  ordered by their smallest edge, each rotated to start at its smallest
  edge.  A loop with two segments on one face is fanned from an added centre
  vertex (the mean of its vertices, summed in loop order), so that no
  triangle side lies inside a face; every other loop is fanned from its
  first vertex.  Triangles then face the outside (their right-hand normal
  points towards increasing D).
* Surface metrics (Sec. 5 "Surface evaluation methods and metrics"): the
  mean absolute deviation of nearest-neighbour distances between two point
  sets, CORR from the mesh vertices to a reference cloud and COMPL from the
  reference to the mesh vertices.  Distances are capped at a radius (a
  point with no neighbour within it counts as the radius).
"""
from __future__ import annotations

import numpy as np

CORNER_OFF = np.array([(k & 1, (k >> 1) & 1, (k >> 2) & 1) for k in range(8)], np.int64)


def _edge_of(k_lo: int, axis: int) -> int:
    o = [int(CORNER_OFF[k_lo][b]) for b in range(3) if b != axis]
    return 4 * axis + o[0] + 2 * o[1]


def _corner(off) -> int:
    return int(off[0]) + 2 * int(off[1]) + 4 * int(off[2])


def edge_corners(e: int):
    """(lower corner, upper corner, axis) of edge e."""
    a, r = divmod(e, 4)
    others = [b for b in range(3) if b != a]
    off = [0, 0, 0]
    off[others[0]] = r & 1
    off[others[1]] = r >> 1
    lo = _corner(off)
    off[a] = 1
    return lo, _corner(off), a


def _edge_between(k0: int, k1: int) -> int:
    d = CORNER_OFF[k1] - CORNER_OFF[k0]
    a = int(np.nonzero(d)[0][0])
    return _edge_of(k0 if d[a] > 0 else k1, a)


def _faces():
    """Corners of the six faces in counter-clockwise order seen from outside
    (right-hand rule about the outward normal)."""
    out = []
    for a in range(3):
        u, v = (a + 1) % 3, (a + 2) % 3
        for s in (0, 1):
            ring = []
            for (pu, pv) in ((0, 0), (1, 0), (1, 1), (0, 1)):  # counter-clockwise about +e_a
                off = [0, 0, 0]
                off[a], off[u], off[v] = s, pu, pv
                ring.append(_corner(off))
            out.append(ring if s == 1 else ring[::-1])
    return out


FACES = _faces()


def case_loops(case: int):
    """Loops of a cube whose inside corners are the set bits of `case`: a
    list of (edges in loop order starting at the smallest, needs a centre
    vertex)."""
    inside = [(case >> k) & 1 for k in range(8)]
    nxt = {}
    face_of = {}
    for f, ring in enumerate(FACES):
        cross = []  # (position on the ring, kind, edge)
        for i in range(4):
            k0, k1 = ring[i], ring[(i + 1) % 4]
            if inside[k0] != inside[k1]:
                cross.append((i, "enter" if inside[k1] else "leave", _edge_between(k0, k1)))
        for j, (i, kind, e) in enumerate(cross):
            if kind != "enter":
                continue
            # the next crossing counter-clockwise leaves this inside run
            _, kind2, e2 = cross[(j + 1) % len(cross)]
            assert kind2 == "leave"
            assert e not in nxt
            nxt[e] = e2
            face_of[e] = f
    loops, seen = [], set()
    for e0 in sorted(nxt):
        if e0 in seen:
            continue
        loop, e = [], e0
        while e not in seen:
            seen.add(e)
            loop.append(e)
            e = nxt[e]
        assert e == e0
        faces = [face_of[x] for x in loop]
        loops.append((loop, len(set(faces)) < len(faces)))
    out = []
    for loop, centre in sorted(loops, key=lambda l: min(l[0])):
        i = loop.index(min(loop))
        out.append((loop[i:] + loop[:i], centre))
    return out


def case_triangles(case: int):
    """Triangles of a cube whose inside corners are the set bits of `case`:
    vertex ids 0..11 are edges, 12 + j the centre of loop j."""
    tris = []
    for j, (loop, centre) in enumerate(case_loops(case)):
        if centre:
            for i in range(len(loop)):
                tris.append((12 + j, loop[i], loop[(i + 1) % len(loop)]))
        else:
            for i in range(1, len(loop) - 1):
                tris.append((loop[0], loop[i], loop[i + 1]))
    return tris


LOOPS = [case_loops(c) for c in range(256)]
TABLE = [case_triangles(c) for c in range(256)]


def _block_key(b):
    b = np.asarray(b, np.int64) + (1 << 20)
    return (b[..., 0] << 42) | (b[..., 1] << 21) | b[..., 2]


def _block_finder(blocks):
    """Index of each queried block coordinate in `blocks`, or -1."""
    key = _block_key(blocks)
    order = np.argsort(key)
    sk = key[order]

    def find(b):
        k = _block_key(b)
        pos = np.minimum(np.searchsorted(sk, k), len(sk) - 1)
        return np.where(sk[pos] == k, order[pos], -1)

    return find


def marching_cubes(field, voxel_size, anchor_blocks=None):
    """Triangle soup of a volume export {'blocks' (n,3), 'D' (n,512),
    'W' (n,512)}: (tri (T,3,3) float64 positions in metres, edges (T,3,4)
    int64 rows (x, y, z, k) naming each vertex: k < 3 the edge along axis k
    from voxel (x, y, z), k = 3 + j the centre of loop j of the cube of
    voxel (x, y, z)).  With `anchor_blocks` (K,3), only the cubes whose
    corner 0 lies in those blocks are meshed (their corners may lie in any
    block of the field).  Triangles come grouped by case."""
    blocks = np.asarray(field["blocks"], np.int64)
    D = np.asarray(field["D"], np.float64)
    W = np.asarray(field["W"], np.float64)
    s = float(np.float32(voxel_size))
    empty = (np.zeros((0, 3, 3)), np.zeros((0, 3, 4), np.int64))
    if len(blocks) == 0:
        return empty
    find = _block_finder(blocks)
    i = np.arange(512)
    local = np.stack([i & 7, (i >> 3) & 7, i >> 6], 1)
    anchors = blocks if anchor_blocks is None else np.asarray(anchor_blocks, np.int64).reshape(-1, 3)
    # every voxel of every anchor block anchors one cube
    vox = (8 * anchors[:, None, :] + local[None, :, :]).reshape(-1, 3)
    Dc = np.zeros((len(vox), 8))
    ok = np.ones(len(vox), bool)
    for k in range(8):
        c = vox + CORNER_OFF[k]
        b = np.floor_divide(c, 8)
        l = c - 8 * b
        bi = find(b)
        li = l[:, 0] + 8 * l[:, 1] + 64 * l[:, 2]
        have = bi >= 0
        w = np.where(have, W[np.maximum(bi, 0), li], 0.0)
        ok &= w > 0
        Dc[:, k] = np.where(have, D[np.maximum(bi, 0), li], 0.0)
    case = np.zeros(len(vox), np.int64)
    for k in range(8):
        case |= (Dc[:, k] < 0).astype(np.int64) << k
    meshed = np.nonzero(ok & (case != 0) & (case != 255))[0]
    tri, edg = [], []
    for c in np.unique(case[meshed]):
        sel = meshed[case[meshed] == c]
        g = vox[sel]
        pos, key = {}, {}
        for e in range(12):
            lo, hi, a = edge_corners(e)
            if ((c >> lo) & 1) == ((c >> hi) & 1):
                continue
            p = g + CORNER_OFF[lo]
            d0, d1 = Dc[sel, lo], Dc[sel, hi]
            t = d0 / (d0 - d1)
            x = s * p.astype(np.float64)
            x[:, a] = s * (p[:, a].astype(np.float64) + t)
            pos[e] = x
            key[e] = np.concatenate([p, np.full((len(sel), 1), a)], 1)
        for j, (loop, centre) in enumerate(LOOPS[c]):
            if centre:
                acc = np.zeros((len(sel), 3))
                for e in loop:
                    acc = acc + pos[e]
                pos[12 + j] = acc / len(loop)
                key[12 + j] = np.concatenate([g, np.full((len(sel), 1), 3 + j)], 1)
        for t3 in TABLE[c]:
            tri.append(np.stack([pos[v] for v in t3], 1))
            edg.append(np.stack([key[v] for v in t3], 1))
    if not tri:
        return empty
    return np.concatenate(tri), np.concatenate(edg).astype(np.int64)


def unique_vertices(tri, edges):
    """Mesh vertices, one per key: (V,3) positions sorted by key."""
    e = np.asarray(edges, np.int64).reshape(-1, 4)
    p = np.asarray(tri, np.float64).reshape(-1, 3)
    if len(e) == 0:
        return np.zeros((0, 3))
    _, first = np.unique(e, axis=0, return_index=True)
    return p[first]


def nn_distance(ref, query, radius):
    """Distance from every query point to its nearest reference point, capped
    at `radius` (FP64; a k-d tree query bounded by the radius)."""
    from scipy.spatial import cKDTree
    q = np.asarray(query, np.float64).reshape(-1, 3)
    r = np.asarray(ref, np.float64).reshape(-1, 3)
    if len(q) == 0:
        return np.zeros(0)
    if len(r) == 0:
        return np.full(len(q), float(radius))
    d, _ = cKDTree(r).query(q, k=1, distance_upper_bound=float(radius))
    return np.minimum(d, float(radius))


def nn_distance_brute(ref, query, radius):
    """The same by exhaustive search (small sets)."""
    q = np.asarray(query, np.float64).reshape(-1, 3)
    r = np.asarray(ref, np.float64).reshape(-1, 3)
    if len(r) == 0:
        return np.full(len(q), float(radius))
    d = np.sqrt(((q[:, None, :] - r[None, :, :]) ** 2).sum(-1)).min(1)
    return np.minimum(d, float(radius))


def corr(mesh_vertices, reference, radius):
    """CORR: mean distance from the mesh vertices to the reference cloud."""
    return float(nn_distance(reference, mesh_vertices, radius).mean()) if len(mesh_vertices) else 0.0


def compl(reference_vertices, mesh_vertices, radius):
    """COMPL: mean distance from the reference vertices to the mesh vertices."""
    return float(nn_distance(mesh_vertices, reference_vertices, radius).mean()) if len(reference_vertices) else 0.0
