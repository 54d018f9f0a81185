"""Pins of the oracle's Marching Cubes and surface metrics against closed
forms and invariants: the case table covers exactly the crossing edges,
closed fields give closed, consistently oriented meshes with the right Euler
characteristic and enclosed volume, linear fields are reproduced exactly,
random fields give a manifold mesh away from the domain boundary, and the
capped nearest-neighbour distances match exhaustive search and closed
forms."""
import math

import numpy as np
import pytest

from oracle import mesh as M


def _field(fn, lo_blk, hi_blk, s, w=None):
    """Volume export of blocks lo_blk..hi_blk (inclusive) with D = fn(x) at
    voxel centres x = s n (metres) and W = 1 (or w(x))."""
    rng = [range(lo_blk[a], hi_blk[a] + 1) for a in range(3)]
    blocks = np.array([(x, y, z) for x in rng[0] for y in rng[1] for z in rng[2]], np.int64)
    i = np.arange(512)
    local = np.stack([i & 7, (i >> 3) & 7, i >> 6], 1)
    vox = 8 * blocks[:, None, :] + local[None]
    X = s * vox.astype(np.float64)
    D = fn(X)
    W = np.ones(D.shape) if w is None else w(X)
    return {"blocks": blocks, "D": D, "W": W}


def _directed_edges(edges):
    """Triangle sides as pairs of vertex keys (tuples), in triangle order."""
    out = []
    for t in edges.tolist():
        k = [tuple(v) for v in t]
        out += [(k[0], k[1]), (k[1], k[2]), (k[2], k[0])]
    return out


def _closed_and_oriented(edges):
    cnt = {}
    for a, b in _directed_edges(edges):
        cnt[(a, b)] = cnt.get((a, b), 0) + 1
    for (a, b), c in cnt.items():
        assert c == 1, "a directed side is used twice (inconsistent orientation)"
        assert cnt.get((b, a), 0) == 1, "an open side"
    return len(cnt) // 2


def _euler(edges):
    V = len({tuple(v) for t in edges.tolist() for v in t})
    E = _closed_and_oriented(edges)
    F = len(edges)
    return V - E + F


def _volume(tri):
    # divergence theorem: sum of signed tetrahedra against the origin
    a, b, c = tri[:, 0], tri[:, 1], tri[:, 2]
    return float(np.einsum("ij,ij->i", a, np.cross(b, c)).sum() / 6.0)


def test_table_uses_exactly_the_crossing_edges():
    assert M.TABLE[0] == [] and M.TABLE[255] == []
    for c in range(256):
        ins = [(c >> k) & 1 for k in range(8)]
        cross = {e for e in range(12) if ins[M.edge_corners(e)[0]] != ins[M.edge_corners(e)[1]]}
        used = [e for t in M.TABLE[c] for e in t if e < 12]
        assert set(used) == cross, c
        # every crossing edge is on exactly one loop; a loop of k vertices
        # gives k - 2 triangles, or k around an added centre vertex
        loops = M.LOOPS[c]
        assert sorted(e for l, _ in loops for e in l) == sorted(cross)
        assert len(M.TABLE[c]) == sum(len(l) if ce else len(l) - 2 for l, ce in loops)
        assert all(len(l) >= 3 for l, _ in loops)
        # a centre vertex only where a loop crosses one face twice (at least 6 vertices)
        assert all(len(l) >= 6 for l, ce in loops if ce)
        # the complementary case has the same crossing edges
        assert {e for t in M.TABLE[255 - c] for e in t if e < 12} == cross


def test_edge_numbering():
    assert [M.edge_corners(e) for e in (0, 3, 4, 7, 8, 11)] == [(0, 1, 0), (6, 7, 0), (0, 2, 1), (5, 7, 1),
                                                             (0, 4, 2), (3, 7, 2)]


def test_single_corner_faces_away_from_it():
    # corner 0 inside: one triangle on edges 0, 4, 8 whose normal is +(1,1,1)
    assert M.TABLE[1] == [(0, 4, 8)]
    f = _field(lambda X: X.sum(-1) - 0.5, (0, 0, 0), (0, 0, 0), 1.0)
    f["D"][:] = 1.0
    f["D"][0, 0] = -1.0  # voxel (0,0,0)
    tri, edges = M.marching_cubes(f, 1.0)
    assert len(tri) == 1
    n = np.cross(tri[0, 1] - tri[0, 0], tri[0, 2] - tri[0, 0])
    assert np.all(n > 0)
    np.testing.assert_allclose(tri[0], [[0.5, 0, 0], [0, 0.5, 0], [0, 0, 0.5]])


def test_sphere_is_closed_with_genus_zero_and_its_volume():
    s, r, c = 0.01, 0.1, np.array([0.123, 0.087, 0.104])
    f = _field(lambda X: np.linalg.norm(X - c, axis=-1) - r, (-1, -1, -1), (3, 3, 3), s)
    tri, edges = M.marching_cubes(f, s)
    assert len(tri) > 500
    assert _euler(edges) == 2
    vol = _volume(tri)
    assert abs(vol - 4 / 3 * math.pi * r ** 3) < 0.01 * 4 / 3 * math.pi * r ** 3
    d = np.abs(np.linalg.norm(tri.reshape(-1, 3) - c, axis=1) - r)
    assert d.max() < s / 16  # linear interpolation of a curved SDF along one edge


def test_torus_has_euler_characteristic_zero():
    s, R, rr, c = 0.01, 0.12, 0.04, np.array([0.2, 0.2, 0.1])

    def sdf(X):
        p = X - c
        q = np.sqrt(p[..., 0] ** 2 + p[..., 1] ** 2) - R
        return np.sqrt(q ** 2 + p[..., 2] ** 2) - rr

    f = _field(sdf, (0, 0, 0), (5, 5, 3), s)
    tri, edges = M.marching_cubes(f, s)
    assert _euler(edges) == 0
    assert abs(_volume(tri) - 2 * math.pi ** 2 * R * rr ** 2) < 0.02 * 2 * math.pi ** 2 * R * rr ** 2


def test_linear_field_vertices_lie_on_the_plane():
    s = float(np.float32(0.01))  # the voxel size as the volume stores it
    n = np.array([0.3, -0.5, 0.81])
    n /= np.linalg.norm(n)
    f = _field(lambda X: X @ n - 0.0437, (0, 0, 0), (1, 1, 1), s)
    tri, edges = M.marching_cubes(f, s)
    assert len(tri) > 100
    assert np.abs(tri.reshape(-1, 3) @ n - 0.0437).max() < 1e-16
    # every normal faces +n
    nn = np.cross(tri[:, 1] - tri[:, 0], tri[:, 2] - tri[:, 0])
    assert np.all(nn @ n > 0)


def test_random_field_is_manifold_inside_the_domain():
    rng = np.random.default_rng(3)
    f = _field(lambda X: rng.normal(size=X.shape[:-1]), (0, 0, 0), (1, 1, 1), 1.0)
    tri, edges = M.marching_cubes(f, 1.0)
    cnt = {}
    for a, b in _directed_edges(edges):
        cnt[(a, b)] = cnt.get((a, b), 0) + 1

    def on_boundary(a, b):
        for ax in range(3):
            for plane in (0, 15):
                # an edge vertex (k < 3) off axis `ax` lies in the plane of its coordinate
                if all(v[3] < 3 and v[3] != ax and v[ax] == plane for v in (a, b)):
                    return True
        return False

    n_boundary = 0
    for (a, b), c in cnt.items():
        assert c == 1
        if on_boundary(a, b):
            n_boundary += 1
            assert (b, a) not in cnt
        else:
            assert cnt.get((b, a), 0) == 1, (a, b)
    assert n_boundary > 0
    assert any(v[3] >= 3 for t in edges.tolist() for v in t), "the field exercises loops with a centre vertex"


def test_unobserved_corners_skip_the_cube():
    s = 0.01
    f = _field(lambda X: X[..., 0] - 0.0405, (0, 0, 0), (0, 0, 0), s)
    tri, _ = M.marching_cubes(f, s)
    # the plane x = 4.05 voxels cuts the 7 x 7 cubes between x = 4 and x = 5
    assert len(tri) == 2 * 7 * 7
    f["W"][0, 4 + 8 * 3 + 64 * 3] = 0.0  # voxel (4, 3, 3) unobserved: four cubes touch it
    tri, _ = M.marching_cubes(f, s)
    assert len(tri) == 2 * (7 * 7 - 4)


def test_unique_vertices_one_per_edge():
    s, r, c = 0.01, 0.025, np.array([0.035, 0.036, 0.034])  # inside the block's cubes
    f = _field(lambda X: np.linalg.norm(X - c, axis=-1) - r, (0, 0, 0), (0, 0, 0), s)
    tri, edges = M.marching_cubes(f, s)
    v = M.unique_vertices(tri, edges)
    assert len(v) == len({tuple(x) for x in edges.reshape(-1, 4).tolist()})
    # Euler: V - E + F = 2 with E = 3F / 2 on a closed triangle mesh
    assert len(v) - len(tri) // 2 == 2


def test_nn_distance_matches_exhaustive_search():
    rng = np.random.default_rng(9)
    ref = rng.uniform(0, 1, (700, 3))
    q = rng.uniform(-0.2, 1.2, (300, 3))
    for radius in (0.02, 0.05, 0.3, 10.0):
        np.testing.assert_allclose(M.nn_distance(ref, q, radius), M.nn_distance_brute(ref, q, radius), rtol=0,
                                   atol=1e-15)
    assert np.all(M.nn_distance(np.zeros((0, 3)), q, 0.05) == 0.05)
    assert len(M.nn_distance(ref, np.zeros((0, 3)), 0.05)) == 0


def test_mad_closed_forms():
    h, delta = 0.01, 0.002
    g = np.arange(0, 1, h)
    X, Y = np.meshgrid(g, g, indexing="ij")
    plane = np.stack([X.ravel(), Y.ravel(), np.zeros(X.size)], 1)
    lifted = plane + [0, 0, delta]
    assert M.corr(lifted, plane, 0.05) == pytest.approx(delta, abs=1e-15)
    assert M.compl(plane, lifted, 0.05) == pytest.approx(delta, abs=1e-15)
    # half of the reference is missing from the model: those points count the cap
    half = lifted[plane[:, 0] < 0.5 - 1e-9]
    cap = 0.05
    far = plane[:, 0] >= 0.5 + cap - 1e-9
    exp_far = far.mean() * cap
    got = M.compl(plane, half, cap)
    assert got > exp_far
    assert M.corr(half, plane, cap) == pytest.approx(delta, abs=1e-15)
