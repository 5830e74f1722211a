"""Pins of the oracle's surface extraction (marching tetrahedra over the
optimised cells): hand-counted cases, a plane, and a closed sphere."""
import numpy as np

import oracle


def _one_cell(values):
    """A single cell (grid 1x1x1 over [0,1]^3) with the given corner values,
    corner (a,b,c) at index 4a + 2b + c, every vertex optimised."""
    dims, lo, hi = (1, 1, 1), (0.0, 0.0, 0.0), (1.0, 1.0, 1.0)
    D = np.zeros(8)
    for a in range(2):
        for b in range(2):
            for c in range(2):
                D[(a * 2 + b) * 2 + c] = values[4 * a + 2 * b + c]
    return oracle.extract_surface(dims, lo, hi, D, np.ones(8, np.uint8))


def test_single_negative_corner_counts():
    # corner 0 and corner 7 lie in all six tetrahedra, corner 4 (x) in two,
    # so one negative corner gives 6, 6 and 2 triangles
    for corner, expect in [(0, 6), (7, 6), (4, 2), (2, 2), (1, 2), (6, 2), (5, 2), (3, 2)]:
        v = np.ones(8)
        v[corner] = -1.0
        keys, tri = _one_cell(v)
        assert len(keys) == expect, (corner, len(keys))
        # every triangle vertex is the midpoint of an edge from that corner (values -1 / 1)
        cx = np.array([corner >> 2 & 1, corner >> 1 & 1, corner & 1], float)
        d = np.abs(tri.reshape(-1, 3) - cx).max(axis=1)
        assert np.allclose(d, 0.5)


def test_no_sign_change_and_all_inside():
    assert len(_one_cell(np.ones(8))[0]) == 0
    assert len(_one_cell(-np.ones(8))[0]) == 0


def test_checkerboard_of_two_and_two():
    # x < 0.5 inside: value = x - 0.5 at the corners: every tetrahedron has
    # two corners each side or one and three; the cut is the plane x = 0.5
    v = np.array([(a - 0.5) for a in (0, 0, 0, 0, 1, 1, 1, 1)], float)
    keys, tri = _one_cell(v)
    assert len(keys) > 0
    assert np.allclose(tri[..., 0], 0.5)
    # the triangles cover the unit square of the plane exactly once
    e1 = tri[:, 1] - tri[:, 0]
    e2 = tri[:, 2] - tri[:, 0]
    area = 0.5 * np.linalg.norm(np.cross(e1, e2), axis=1).sum()
    assert abs(area - 1.0) < 1e-12


def test_plane_in_a_dense_band():
    # D = z - c over a 6x5x7 grid, every cell optimised: all vertices on the
    # plane and the area equals the domain's x-y extent
    dims, lo, hi = (6, 5, 7), (-1.0, -0.5, -0.75), (0.5, 0.75, 1.0)
    c = 0.1234
    V = np.array(dims) + 1
    z = lo[2] + np.arange(V[2]) * ((hi[2] - lo[2]) / dims[2])
    D = np.broadcast_to(z - c, (V[0], V[1], V[2])).reshape(-1).astype(np.float64)
    keys, tri = oracle.extract_surface(dims, lo, hi, D, np.ones(int(V.prod()), np.uint8))
    assert np.abs(tri[..., 2] - c).max() < 1e-12
    e1 = tri[:, 1] - tri[:, 0]
    e2 = tri[:, 2] - tri[:, 0]
    area = 0.5 * np.linalg.norm(np.cross(e1, e2), axis=1).sum()
    assert abs(area - (hi[0] - lo[0]) * (hi[1] - lo[1])) < 1e-9
    assert np.all(np.diff(keys) > 0)


def test_sphere_is_closed_and_near():
    # closed-form sphere SDF over a band around it: the mesh is watertight
    # (every edge in exactly two triangles) and its vertices lie within the
    # linear-interpolation error of the sphere along a cell's longest edge
    R, r = 24, 0.55
    dims, lo, hi = (R, R, R), (-1.0, -1.0, -1.0), (1.0, 1.0, 1.0)
    h = 2.0 / R
    g = lo[0] + np.arange(R + 1) * h
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    D = (np.sqrt(X * X + Y * Y + Z * Z) - r).reshape(-1)
    vf = (np.abs(D) < 3 * h).astype(np.uint8)
    keys, tri = oracle.extract_surface(dims, lo, hi, D, vf)
    v = tri.reshape(-1, 3)
    err = np.abs(np.linalg.norm(v, axis=1) - r)
    # chord error of |x| along an edge of length L at distance >= r - L: L^2 / (8 (r - L))
    L = np.sqrt(3) * h
    assert err.max() <= L * L / (8 * (r - L)) + 1e-12
    # watertight: canonical edges (vertex coordinates are computed identically
    # in every tetrahedron sharing a grid edge)
    edges = {}
    for t in tri:
        pts = [tuple(p) for p in t]
        for a, b in ((0, 1), (1, 2), (2, 0)):
            e = (min(pts[a], pts[b]), max(pts[a], pts[b]))
            edges[e] = edges.get(e, 0) + 1
    counts = np.array(list(edges.values()))
    assert np.all(counts == 2), np.bincount(counts)


def test_metrics_on_the_exact_sphere_mesh():
    """The measures of the extracted mesh of the exact sphere SDF: near zero
    distance, normals consistent, F-score 1 at a threshold above the
    interpolation error; a shifted sphere is measured as far."""
    from paper_2308_13175_amd import metrics

    R, r = 32, 0.5
    h = 2.0 / R
    g = -1.0 + np.arange(R + 1) * h
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    D = (np.sqrt(X * X + Y * Y + Z * Z) - r).reshape(-1)
    vf = (np.abs(D) < 3 * h).astype(np.uint8)
    _, tri = oracle.extract_surface((R, R, R), (-1.0,) * 3, (1.0,) * 3, D, vf)
    rng = np.random.default_rng(3)
    s = rng.normal(size=(20_000, 3))
    surf = r * s / np.linalg.norm(s, axis=1, keepdims=True)
    sdf, grad = metrics.sphere_sdf(r)
    m = metrics.reconstruction_metrics(tri, surf, sdf, grad, tau=0.01, n_samples=50_000)
    assert m["accuracy"] < 2e-3 and m["completeness"] < 5e-3
    assert m["nc"] > 0.995
    assert m["fscore"] > 0.99
    sdf2, grad2 = metrics.sphere_sdf(r, centre=(0.05, 0.0, 0.0))
    m2 = metrics.reconstruction_metrics(tri, surf + np.array([0.05, 0.0, 0.0]), sdf2, grad2, tau=0.01,
                                        n_samples=50_000)
    assert m2["cd_l1"] > 5 * m["cd_l1"] and m2["fscore"] < 0.5


# ---------------------------------------------------------------------------
# Marching cubes (the paper's mesh step)
# ---------------------------------------------------------------------------

def _mc_one_cell(inside):
    """One cell over [0,1]^3, corner (a,b,c) at index 4a + 2b + c, value -1
    at the inside corners and +1 elsewhere."""
    v = np.ones(8)
    for i in inside:
        v[i] = -1.0
    D = np.zeros(8)
    for a in range(2):
        for b in range(2):
            for c in range(2):
                D[(a * 2 + b) * 2 + c] = v[4 * a + 2 * b + c]
    return oracle.marching_cubes((1, 1, 1), (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), D, np.ones(8, np.uint8))


def _area(tri):
    e1 = tri[:, 1] - tri[:, 0]
    e2 = tri[:, 2] - tri[:, 0]
    return 0.5 * np.linalg.norm(np.cross(e1, e2), axis=1).sum()


def _edge_uses(tri):
    """Directed and undirected uses of every triangle edge (by exact vertex coordinates)."""
    directed, undirected = {}, {}
    for t in tri:
        pts = [tuple(p) for p in t]
        for a, b in ((0, 1), (1, 2), (2, 0)):
            directed[(pts[a], pts[b])] = directed.get((pts[a], pts[b]), 0) + 1
            e = (min(pts[a], pts[b]), max(pts[a], pts[b]))
            undirected[e] = undirected.get(e, 0) + 1
    return directed, undirected


def test_mc_hand_counted_cells():
    """Counted by hand: a corner cut off is one triangle; two corners sharing
    an edge, or a whole face, a quad (two); a corner with its three edge
    neighbours, a hexagon (four); two diagonal corners of a face, or two
    opposite corners of the cube, are cut off separately (two); complements
    of a single corner, one."""
    cases = [((), 0), ((0,), 1), ((7,), 1), ((0, 4), 2), ((0, 1, 2, 3), 2), ((0, 1, 2, 4), 4),
             ((0, 3), 2), ((0, 6), 2), ((0, 7), 2), (tuple(range(1, 8)), 1), (tuple(range(8)), 0)]
    for inside, expect in cases:
        keys, tri = _mc_one_cell(inside)
        assert len(keys) == expect, (inside, len(keys))
    # values -1 / +1: every vertex is an edge midpoint; corner 0 alone gives the
    # triangle of the three midpoints next to it
    keys, tri = _mc_one_cell((0,))
    assert {tuple(p) for p in tri[0]} == {(0.5, 0.0, 0.0), (0.0, 0.5, 0.0), (0.0, 0.0, 0.5)}
    counts = oracle.marching_cubes_counts()
    assert counts.max() == 5 and counts[0] == 0 and counts[255] == 0


def test_mc_plane_area_exact():
    """A tilted plane z = 0.3 + 0.2 x through a dense band over [-1, 1]^3:
    linear interpolation of a linear field is exact, so every vertex lies on
    the plane and the mesh covers exactly the plane inside the box,
    4 sqrt(1 + 0.2^2)."""
    R = 14
    dims, lo, hi = (R, R, R), (-1.0,) * 3, (1.0,) * 3
    g = -1.0 + np.arange(R + 1) * (2.0 / R)
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    D = (Z - (0.3 + 0.2 * X)).reshape(-1)
    keys, tri = oracle.marching_cubes(dims, lo, hi, D, np.ones(D.size, np.uint8))
    v = tri.reshape(-1, 3)
    assert np.abs(v[:, 2] - (0.3 + 0.2 * v[:, 0])).max() < 1e-14
    assert abs(_area(tri) - 4 * np.sqrt(1.04)) < 1e-12
    assert np.all(np.diff(keys) > 0)


def test_mc_sphere_closed_oriented_genus_zero():
    """The closed-form sphere SDF over a band: the mesh is watertight (every
    edge in exactly two triangles), consistently oriented (each edge once
    each way), has the Euler characteristic of a sphere, and its vertices
    lie within the interpolation error; its area is within that error of
    4 pi r^2."""
    R, r = 24, 0.55
    dims, lo, hi = (R, R, R), (-1.0,) * 3, (1.0,) * 3
    h = 2.0 / R
    g = -1.0 + np.arange(R + 1) * h
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    D = (np.sqrt(X * X + Y * Y + Z * Z) - r).reshape(-1)
    vf = (np.abs(D) < 3 * h).astype(np.uint8)
    keys, tri = oracle.marching_cubes(dims, lo, hi, D, vf)
    L = h
    err = np.abs(np.linalg.norm(tri.reshape(-1, 3), axis=1) - r)
    assert err.max() <= L * L / (8 * (r - L)) + 1e-12
    directed, undirected = _edge_uses(tri)
    assert set(undirected.values()) == {2}
    assert set(directed.values()) == {1}
    V = len({tuple(p) for p in tri.reshape(-1, 3)})
    assert V - len(undirected) + len(tri) == 2
    assert abs(_area(tri) / (4 * np.pi * r * r) - 1) < 0.02


def test_mc_random_field_has_no_cracks():
    """A random field (many ambiguous faces) over a dense band: every mesh
    edge not on the domain's boundary is shared by exactly two triangles,
    once each way; the face rule is the same from both cells of a face."""
    rng = np.random.default_rng(11)
    R = 9
    dims, lo, hi = (R, R, R), (0.0,) * 3, (1.0,) * 3
    D = rng.normal(size=(R + 1) ** 3)
    keys, tri = oracle.marching_cubes(dims, lo, hi, D, np.ones(D.size, np.uint8))
    assert len(tri) > 500
    directed, undirected = _edge_uses(tri)
    on_boundary = lambda p: any(abs(x) < 1e-15 or abs(x - 1.0) < 1e-15 for x in p)
    for (a, b), n in undirected.items():
        if on_boundary(a) and on_boundary(b):
            assert n in (1, 2)
        else:
            assert n == 2 and directed.get((a, b)) == 1 and directed.get((b, a)) == 1, (a, b, n)
