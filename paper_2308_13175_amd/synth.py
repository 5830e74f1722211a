"""Seeded synthetic inputs for the GridPull pull step.

This module produces the inputs that both the HIP path and the CPU oracle
consume: point clouds, grid domains, query batches and initial fields.  It
contains none of the method's arithmetic (no interpolation, pulling, loss,
band or optimiser code); it only draws random geometry.

The shapes stand in for the paper's datasets (Sec. 4: ShapeNet, FAMOUS, SRB,
3D scenes, KITTI), which are not available: they have the same kind of
content (closed surfaces sampled by area, noisy room-scale scenes) and span
the same point counts (10K to 20M) and grid resolutions (64^3 to 1024^3).

Every generator is deterministic in its seed (numpy PCG64).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np


# ---------------------------------------------------------------------------
# Grid domains
# ---------------------------------------------------------------------------

@dataclasses.dataclass(frozen=True)
class Domain:
    """A grid of R_x x R_y x R_z cells over the box [lo, hi]."""

    dims: tuple
    lo: tuple
    hi: tuple

    @property
    def h(self):
        return tuple((self.hi[a] - self.lo[a]) / self.dims[a] for a in range(3))

    @property
    def n_cells(self) -> int:
        return int(self.dims[0]) * int(self.dims[1]) * int(self.dims[2])

    @property
    def vdims(self):
        return tuple(int(d) + 1 for d in self.dims)

    @property
    def n_vertices(self) -> int:
        v = self.vdims
        return v[0] * v[1] * v[2]

    @property
    def diagonal(self) -> float:
        return math.sqrt(sum((self.hi[a] - self.lo[a]) ** 2 for a in range(3)))


def cube_domain(res: int, half: float = 1.0) -> Domain:
    return Domain((res, res, res), (-half, -half, -half), (half, half, half))


def vertex_positions(dom: Domain, vertex_ids: np.ndarray) -> np.ndarray:
    """World positions lo + (i, j, k) * h of x-major vertex ids, float64 [n, 3]."""
    vy, vz = dom.vdims[1], dom.vdims[2]
    vid = np.asarray(vertex_ids, dtype=np.int64)
    i = vid // (vy * vz)
    j = (vid // vz) % vy
    k = vid % vz
    h = dom.h
    return np.stack([dom.lo[0] + i * h[0], dom.lo[1] + j * h[1], dom.lo[2] + k * h[2]], axis=1)


# ---------------------------------------------------------------------------
# Surface samplers (area-uniform)
# ---------------------------------------------------------------------------

def _unit_sphere(rng, n):
    v = rng.standard_normal((n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v


def sphere_points(n: int, radius: float = 0.5, seed: int = 0) -> np.ndarray:
    """Uniform points on a sphere at the origin (normalised Gaussian vectors)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return (_unit_sphere(rng, n) * radius).astype(np.float32)


@dataclasses.dataclass(frozen=True)
class Primitive:
    """An axis-aligned ellipsoid, box or z-axis torus."""

    kind: str                 # "ellipsoid" | "box" | "torus"
    centre: tuple
    size: tuple               # half-axes (ellipsoid, box) or (R, r, 0) (torus)

    def area(self) -> float:
        if self.kind == "box":
            a, b, c = self.size
            return 8.0 * (a * b + a * c + b * c)
        if self.kind == "torus":
            R, r = self.size[0], self.size[1]
            return 4.0 * math.pi ** 2 * R * r
        a, b, c = self.size          # Knud Thomsen's approximation; only a weight
        p = 1.6075
        return 4 * math.pi * (((a * b) ** p + (a * c) ** p + (b * c) ** p) / 3) ** (1 / p)

    def bounds(self):
        c = np.asarray(self.centre, dtype=np.float64)
        if self.kind == "torus":
            R, r = self.size[0], self.size[1]
            e = np.array([R + r, R + r, r])
        else:
            e = np.asarray(self.size, dtype=np.float64)
        return c - e, c + e

    def overlaps(self, other: "Primitive") -> bool:
        a0, a1 = self.bounds()
        b0, b1 = other.bounds()
        return bool(np.all(a0 < b1) and np.all(b0 < a1))

    def inside(self, x: np.ndarray) -> np.ndarray:
        """Strictly inside (points on the surface are outside)."""
        d = x - np.asarray(self.centre)
        if self.kind == "box":
            return np.all(np.abs(d) < np.asarray(self.size), axis=1)
        if self.kind == "torus":
            R, r = self.size[0], self.size[1]
            rho = np.sqrt(d[:, 0] ** 2 + d[:, 1] ** 2)
            return (rho - R) ** 2 + d[:, 2] ** 2 < r * r
        s = np.asarray(self.size)
        return np.sum((d / s) ** 2, axis=1) < 1.0

    def sample(self, rng, n: int) -> np.ndarray:
        c = np.asarray(self.centre)
        if n <= 0:
            return np.zeros((0, 3))
        if self.kind == "box":
            a, b, cz = self.size
            areas = np.array([b * cz, b * cz, a * cz, a * cz, a * b, a * b])
            face = rng.choice(6, size=n, p=areas / areas.sum())
            u = rng.uniform(-1.0, 1.0, size=(n, 3))
            axis = face // 2
            sign = np.where(face % 2 == 0, -1.0, 1.0)
            u[np.arange(n), axis] = sign
            return c + u * np.asarray(self.size)
        if self.kind == "torus":
            R, r = self.size[0], self.size[1]
            out = []
            got = 0
            while got < n:
                m = int((n - got) * (R + r) / R * 1.2) + 16
                uu = rng.uniform(0, 2 * math.pi, m)
                vv = rng.uniform(0, 2 * math.pi, m)
                keep = rng.uniform(0, 1, m) < (R + r * np.cos(vv)) / (R + r)
                uu, vv = uu[keep], vv[keep]
                pts = np.stack([(R + r * np.cos(vv)) * np.cos(uu),
                                (R + r * np.cos(vv)) * np.sin(uu),
                                r * np.sin(vv)], axis=1)
                out.append(pts)
                got += len(pts)
            return c + np.concatenate(out)[:n]
        a, b, cz = self.size
        out = []
        got = 0
        wmax = max(b * cz, a * cz, a * b)
        while got < n:
            m = int((n - got) * 2.0) + 16
            u = _unit_sphere(rng, m)
            w = np.sqrt((b * cz * u[:, 0]) ** 2 + (a * cz * u[:, 1]) ** 2 + (a * b * u[:, 2]) ** 2)
            keep = rng.uniform(0, wmax, m) < w
            out.append(u[keep] * np.asarray(self.size))
            got += int(keep.sum())
        return c + np.concatenate(out)[:n]


def union_surface_points(prims: Sequence[Primitive], n: int, rng,
                         extra_inside: Sequence[Primitive] = ()) -> np.ndarray:
    """Area-uniform points on the boundary of a union of primitives.

    Candidates are drawn on each primitive in proportion to its area; those
    strictly inside another primitive are rejected, and the draw repeats until
    n points remain.
    """
    areas = np.array([p.area() for p in prims])
    probs = areas / areas.sum()
    chunks: List[np.ndarray] = []
    got = 0
    while got < n:
        want = int((n - got) * 1.3) + 64
        counts = rng.multinomial(want, probs)
        for i, (p, k) in enumerate(zip(prims, counts)):
            if k == 0:
                continue
            x = p.sample(rng, int(k))
            keep = np.ones(len(x), dtype=bool)
            for j, o in enumerate(prims):
                if j != i and p.overlaps(o):
                    keep &= ~o.inside(x)
            for o in extra_inside:
                keep &= ~o.inside(x)
            x = x[keep]
            chunks.append(x)
            got += len(x)
    pts = np.concatenate(chunks)
    idx = rng.permutation(len(pts))[:n]
    return pts[idx]


def torus_points(n: int, R: float = 0.5, r: float = 0.15, jitter: float = 0.002,
                 seed: int = 1) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    t = Primitive("torus", (0.0, 0.0, 0.0), (R, r, 0.0))
    pts = t.sample(rng, n)
    pts = pts + rng.normal(0.0, jitter, size=pts.shape)
    return pts.astype(np.float32)


def random_primitives(rng, count: int, kinds: Sequence[str], centre_half: float,
                      half_axes=(0.05, 0.3), torus_R=(0.15, 0.4), torus_r=(0.03, 0.1)):
    prims = []
    for _ in range(count):
        kind = kinds[int(rng.integers(len(kinds)))]
        c = tuple(rng.uniform(-centre_half, centre_half, 3))
        if kind == "torus":
            size = (float(rng.uniform(*torus_R)), float(rng.uniform(*torus_r)), 0.0)
        else:
            size = tuple(float(s) for s in rng.uniform(half_axes[0], half_axes[1], 3))
        prims.append(Primitive(kind, c, size))
    return prims


def union24_points(n: int = 2_000_000, seed: int = 2) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    prims = random_primitives(rng, 24, ("ellipsoid", "box"), 0.7)
    return union_surface_points(prims, n, rng).astype(np.float32)


def room_points(n: int = 20_000_000, n_furniture: int = 200, noise: float = 0.005,
                seed: int = 4) -> np.ndarray:
    """A 10 x 8 x 3 room (floor, ceiling, four walls) with furniture on the floor."""
    rng = np.random.Generator(np.random.PCG64(seed))
    room = Primitive("box", (5.0, 4.0, 1.5), (5.0, 4.0, 1.5))
    furn = []
    for _ in range(n_furniture):
        kind = "box" if rng.uniform() < 0.5 else "ellipsoid"
        hx, hy = rng.uniform(0.1, 0.6, 2)
        hz = rng.uniform(0.1, 0.5)
        cx, cy = rng.uniform(0.7, 9.3), rng.uniform(0.7, 7.3)
        furn.append(Primitive(kind, (float(cx), float(cy), float(hz)),
                              (float(hx), float(hy), float(hz))))
    areas = np.array([room.area()] + [p.area() for p in furn])
    probs = areas / areas.sum()
    bl = np.array([p.bounds()[0] for p in furn])
    bh = np.array([p.bounds()[1] for p in furn])
    overlap = np.all((bl[:, None, :] < bh[None, :, :]) & (bl[None, :, :] < bh[:, None, :]), axis=2)
    np.fill_diagonal(overlap, False)
    chunks = []
    got = 0
    while got < n:
        want = int((n - got) * 1.2) + 1024
        counts = rng.multinomial(want, probs)
        x = room.sample(rng, int(counts[0]))
        # room points strictly inside a piece of furniture are hidden: test each
        # piece only against the points in its footprint (x-sorted slices)
        keep = np.ones(len(x), dtype=bool)
        order = np.argsort(x[:, 0], kind="stable")
        xs = x[order, 0]
        for i, o in enumerate(furn):
            a, b = np.searchsorted(xs, bl[i, 0], "right"), np.searchsorted(xs, bh[i, 0], "left")
            if b <= a:
                continue
            cand = order[a:b]
            y = x[cand]
            sel = (y[:, 1] > bl[i, 1]) & (y[:, 1] < bh[i, 1]) & (y[:, 2] < bh[i, 2])
            if np.any(sel):
                c2 = cand[sel]
                keep[c2[o.inside(x[c2])]] = False
        chunks.append(x[keep])
        got += int(keep.sum())
        for i, p in enumerate(furn):
            k = int(counts[i + 1])
            if k == 0:
                continue
            y = p.sample(rng, k)
            keep = (y[:, 2] >= 0.0)
            for j in np.nonzero(overlap[i])[0]:
                keep &= ~furn[j].inside(y)
            chunks.append(y[keep])
            got += int(keep.sum())
    pts = np.concatenate(chunks)
    pts = pts[rng.permutation(len(pts))[:n]]
    pts = pts + rng.normal(0.0, noise, size=pts.shape)
    return pts.astype(np.float32)


def room_domain(dims=(1024, 820, 308), size=(10.0, 8.0, 3.0), pad_cells: int = 4) -> Domain:
    """Room bounds padded by pad_cells cells per side, so noisy points stay inside."""
    h = [size[a] / (dims[a] - 2 * pad_cells) for a in range(3)]
    lo = tuple(-pad_cells * h[a] for a in range(3))
    hi = tuple(size[a] + pad_cells * h[a] for a in range(3))
    return Domain(tuple(dims), lo, hi)


# ---------------------------------------------------------------------------
# Per-point sampling scale
# ---------------------------------------------------------------------------

def knn_sigma(points: np.ndarray, k: int = 50) -> np.ndarray:
    """Distance from each point to its k-th nearest other point (float32)."""
    from scipy.spatial import cKDTree

    tree = cKDTree(points.astype(np.float64))
    d, _ = tree.query(points.astype(np.float64), k=k + 1)
    return d[:, k].astype(np.float32)


# ---------------------------------------------------------------------------
# Queries and initial fields for tests
# ---------------------------------------------------------------------------

def host_queries(points: np.ndarray, n_queries: int, sigma, seed: int,
                 stratified: bool = True) -> np.ndarray:
    """Queries = a source point plus sigma * N(0, I3), float32 [n, 3].

    With stratified sources, query k uses point floor(k * J / Q); otherwise the
    sources are drawn uniformly with replacement.  sigma is a scalar or a
    per-point array.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    J = len(points)
    if stratified:
        src = (np.arange(n_queries, dtype=np.int64) * J) // max(n_queries, 1)
    else:
        src = rng.integers(0, J, n_queries)
    z = rng.standard_normal((n_queries, 3))
    sig = np.asarray(sigma, dtype=np.float64)
    sig = sig[src][:, None] if sig.ndim else float(sig)
    q = points[src].astype(np.float64) + sig * z
    return q.astype(np.float32)


def sphere_sdf_field(dom: Domain, radius: float, noise: float = 0.0, seed: int = 0,
                     centre=(0.0, 0.0, 0.0)) -> np.ndarray:
    """|x_v - centre| - radius (+ U(-noise, noise)) at every vertex, x-major, float32."""
    vx, vy, vz = dom.vdims
    h = dom.h
    xs = dom.lo[0] + np.arange(vx) * h[0] - centre[0]
    ys = dom.lo[1] + np.arange(vy) * h[1] - centre[1]
    zs = dom.lo[2] + np.arange(vz) * h[2] - centre[2]
    d = np.sqrt(xs[:, None, None] ** 2 + ys[None, :, None] ** 2 + zs[None, None, :] ** 2) - radius
    d = d.reshape(-1)
    if noise > 0:
        rng = np.random.Generator(np.random.PCG64(seed))
        d = d + rng.uniform(-noise, noise, size=d.shape)
    return d.astype(np.float32)


# ---------------------------------------------------------------------------
# The five workloads
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Shape:
    points: np.ndarray            # float32 [J, 3]
    domain: Domain
    n_queries: int
    sigma: object                 # float or float32 [J]


@dataclasses.dataclass
class Workload:
    name: str
    shapes: List[Shape]
    m1: int = 3
    m2: int = 3
    iters: int = 20
    # Adam's initial learning rate in world units: lr0_cells cells of the
    # smallest cell size when given (the sphere workload starts at the
    # closed-form field), else 1.0 in the units of the domain scaled to
    # [-1, 1] on its longest side (half that side)
    lr0_cells: Optional[float] = None

    def lr0(self) -> float:
        d = self.shapes[0].domain
        if self.lr0_cells is not None:
            return self.lr0_cells * min(min(s.domain.h) for s in self.shapes)
        return 0.5 * max(d.hi[a] - d.lo[a] for a in range(3))

    @property
    def n_points(self) -> int:
        return sum(len(s.points) for s in self.shapes)

    @property
    def n_queries(self) -> int:
        return sum(s.n_queries for s in self.shapes)


def sphere_workload() -> Workload:
    """10K points on a sphere r=0.5, 64^3 over [-1,1]^3, 50K queries, sigma 0.02."""
    pts = sphere_points(10_000, 0.5, seed=0)
    return Workload("sphere-10k-64^3-q50k", [Shape(pts, cube_domain(64), 50_000, 0.02)],
                    iters=20, lr0_cells=0.1)


def torus_workload(n_points: int = 200_000, n_queries: int = 1_000_000) -> Workload:
    """200K noisy torus points, 128^3, 1M queries, sigma = 50th-NN distance."""
    pts = torus_points(n_points, seed=1)
    return Workload("torus-200k-128^3-q1M", [Shape(pts, cube_domain(128), n_queries, knn_sigma(pts, 50))])


def union24_workload() -> Workload:
    """2M points on a union of 24 ellipsoids/boxes, 256^3, 4M queries, sigma = 2h."""
    pts = union24_points(2_000_000, seed=2)
    dom = cube_domain(256)
    return Workload("union24-2M-256^3-q4M", [Shape(pts, dom, 4_000_000, 2 * dom.h[0])], iters=200)


def batched_workload(n_shapes: int = 64, seed: int = 3, scale: float = 1.0) -> Workload:
    """64 shapes, J log-uniform in [5K, 300K], grid by J, Q_i = 10 J_i, sigma = 2 h_i."""
    rng = np.random.Generator(np.random.PCG64(seed))
    shapes = []
    for _ in range(n_shapes):
        J = int(round(math.exp(rng.uniform(math.log(5e3), math.log(3e5))) * scale))
        J = max(J, 16)
        res = 64 if J < 19_600 * scale else (128 if J < 76_600 * scale else 256)
        nprim = int(rng.integers(1, 5))
        prims = random_primitives(rng, nprim, ("ellipsoid", "box", "torus"), 0.5)
        pts = union_surface_points(prims, J, rng).astype(np.float32)
        dom = cube_domain(res)
        shapes.append(Shape(pts, dom, 10 * J, 2 * dom.h[0]))
    return Workload("batched64-5k..300k", shapes)


def room_workload(n_points: int = 20_000_000, n_queries: int = 32_000_000) -> Workload:
    """20M noisy room points, 1024x820x308 cells, 32M queries, sigma = 2h."""
    pts = room_points(n_points, seed=4)
    dom = room_domain()
    return Workload("room-20M-1024x820x308-q32M", [Shape(pts, dom, n_queries, 2 * min(dom.h))])


WORKLOADS = {
    1: sphere_workload,
    2: torus_workload,
    3: union24_workload,
    4: batched_workload,
    5: room_workload,
}
