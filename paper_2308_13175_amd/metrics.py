"""Reconstruction quality of an extracted mesh against a closed-form surface
(the paper's evaluation measures, Sec. 4: Chamfer distance, normal
consistency and F-score), computed on the host from samples.

- accuracy: |sdf(x)| of points x sampled uniformly by area on the mesh, the
  exact distance to the closed-form surface;
- completeness: distance from points on the true surface to the nearest mesh
  sample (a k-d tree over the samples);
- CD-L1 = (mean accuracy + mean completeness) / 2;
- NC = mean |n_face . grad sdf / |grad sdf|| at the mesh samples (the mesh's
  triangles are not oriented, so the absolute cosine);
- F-score at tau = 2 P R / (P + R), P = share of accuracies below tau,
  R = share of completenesses below tau.

This is evaluation, not the optimisation path.
"""
from __future__ import annotations

from typing import Callable, Dict

import numpy as np


def sample_mesh(tri: np.ndarray, n: int, seed: int = 0):
    """n points uniformly by area on triangles tri [m, 3, 3], with the unit
    normal of the triangle each comes from."""
    tri = np.asarray(tri, dtype=np.float64)
    e1 = tri[:, 1] - tri[:, 0]
    e2 = tri[:, 2] - tri[:, 0]
    cr = np.cross(e1, e2)
    area = 0.5 * np.linalg.norm(cr, axis=1)
    keep = area > 0
    tri, e1, e2, cr, area = tri[keep], e1[keep], e2[keep], cr[keep], area[keep]
    rng = np.random.default_rng(seed)
    f = rng.choice(len(tri), size=n, p=area / area.sum())
    u, v = rng.random(n), rng.random(n)
    flip = u + v > 1.0
    u[flip], v[flip] = 1.0 - u[flip], 1.0 - v[flip]
    x = tri[f, 0] + u[:, None] * e1[f] + v[:, None] * e2[f]
    nrm = cr[f] / np.linalg.norm(cr[f], axis=1, keepdims=True)
    return x, nrm


def sphere_sdf(r: float, centre=(0.0, 0.0, 0.0)):
    c = np.asarray(centre, dtype=np.float64)

    def sdf(x):
        return np.linalg.norm(x - c, axis=1) - r

    def grad(x):
        d = x - c
        return d / np.linalg.norm(d, axis=1, keepdims=True)

    return sdf, grad


def torus_sdf(R: float, r: float):
    """z-axis torus at the origin: sqrt((sqrt(x^2 + y^2) - R)^2 + z^2) - r."""

    def sdf(x):
        q = np.hypot(x[:, 0], x[:, 1]) - R
        return np.hypot(q, x[:, 2]) - r

    def grad(x):
        rho = np.hypot(x[:, 0], x[:, 1])
        q = rho - R
        s = np.hypot(q, x[:, 2])
        g = np.stack([q * x[:, 0] / rho, q * x[:, 1] / rho, x[:, 2]], axis=1)
        return g / s[:, None]

    return sdf, grad


def reconstruction_metrics(tri: np.ndarray, surface_points: np.ndarray, sdf: Callable, grad: Callable,
                           tau: float, n_samples: int = 100_000, seed: int = 0) -> Dict[str, float]:
    from scipy.spatial import cKDTree

    x, nrm = sample_mesh(tri, n_samples, seed)
    acc = np.abs(sdf(x))
    comp, _ = cKDTree(x).query(np.asarray(surface_points, dtype=np.float64))
    g = grad(x)
    nc = np.abs(np.sum(nrm * g / np.linalg.norm(g, axis=1, keepdims=True), axis=1))
    p = float(np.mean(acc < tau))
    rr = float(np.mean(comp < tau))
    return {"cd_l1": float(0.5 * (acc.mean() + comp.mean())), "accuracy": float(acc.mean()),
            "completeness": float(comp.mean()), "nc": float(nc.mean()),
            "fscore": 2 * p * rr / (p + rr) if p + rr > 0 else 0.0, "precision": p, "recall": rr, "tau": tau}
