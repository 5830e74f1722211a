"""FP64 CPU oracle of the GridPull pull step -- test infrastructure only.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may use
this package.  It is the checker for the HIP library and shares no code with
it: the C source next to this file is compiled on its own with gcc and loaded
through ctypes.  Each wrapper names the part of the paper it computes; the
C file states the readings taken where the paper is silent.

Domains are passed as plain (dims, lo, hi) triples so that nothing here
depends on the product package.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gridpull_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-shared", "-fPIC"]

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C, FP64, no contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build(force=True)   # missing or older than its source
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    i64, i32, u32, u64, f64 = ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double
    lib.og_build_band.restype = i64
    lib.og_build_band.argtypes = [P, P, P, P, P, P, i64, i32, i32, P, P]
    lib.og_nn_bruteforce.restype = None
    lib.og_nn_bruteforce.argtypes = [P, P, P, i64, P, P, P, i64, P]
    lib.og_eval.restype = ctypes.c_int
    lib.og_eval.argtypes = [P, P, P, P, f64, f64, f64, P, P]
    lib.og_loss_grad.restype = i64
    lib.og_loss_grad.argtypes = [P, P, P, P, P, P, P, P, P, P, i64, P, P, P,
                                 f64, f64, f64, f64, P, P, P, P]
    lib.og_adam.restype = None
    lib.og_adam.argtypes = [i64, P, P, P, P, P, i32, f64, f64, i32, f64, f64, f64]
    lib.og_philox4x32_10.restype = None
    lib.og_philox4x32_10.argtypes = [P, P, P]
    lib.og_query_offsets.restype = None
    lib.og_query_offsets.argtypes = [u64, u32, u32, i64, i64, P]
    lib.og_extract_surface.restype = i64
    lib.og_extract_surface.argtypes = [P, P, P, P, P, i64, P, P]
    lib.og_marching_cubes.restype = i64
    lib.og_marching_cubes.argtypes = [P, P, P, P, P, i64, P, P]
    lib.og_mc_counts.restype = None
    lib.og_mc_counts.argtypes = [P]
    lib.og_normal_term.restype = i64
    lib.og_normal_term.argtypes = [P, P, P, P, P, P, P, P, P, i64, P, P, P, P, P, P, f64, f64, P, P]
    _lib = lib
    return lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _grid(dims, lo, hi):
    R = np.ascontiguousarray(dims, dtype=np.int32)
    L = np.ascontiguousarray(lo, dtype=np.float64)
    H = np.ascontiguousarray(hi, dtype=np.float64)
    return R, L, H


def _soa(x: np.ndarray):
    x = np.asarray(x, dtype=np.float32)
    return (np.ascontiguousarray(x[:, 0]), np.ascontiguousarray(x[:, 1]),
            np.ascontiguousarray(x[:, 2]))


class DomainError(ValueError):
    pass


def build_band(dims, lo, hi, points: np.ndarray, m1: int, m2: int):
    """Base cells, M1 and M2 bands (Sec. 3 band paragraphs) as dense flags.

    Returns (cell_flags [R_x*R_y*R_z], vert_flags [(R+1)^3]) -- see the C file
    for the bit meanings.  Raises DomainError for a point outside [lo, hi].
    """
    lib = _load()
    R, L, H = _grid(dims, lo, hi)
    nc = int(np.prod(R.astype(np.int64)))
    nv = int(np.prod(R.astype(np.int64) + 1))
    cf = np.zeros(nc, dtype=np.uint8)
    vf = np.zeros(nv, dtype=np.uint8)
    px, py, pz = _soa(points)
    bad = lib.og_build_band(_p(R), _p(L), _p(H), _p(px), _p(py), _p(pz), len(px),
                            int(m1), int(m2), _p(cf), _p(vf))
    if bad >= 0:
        raise DomainError("point %d lies outside the grid domain" % bad)
    return cf, vf


def nn_bruteforce(queries: np.ndarray, points: np.ndarray) -> np.ndarray:
    """argmin_j |q - s_j|^2 (Eq. 4's NN(q)), ties to the lowest j, int32."""
    lib = _load()
    qx, qy, qz = _soa(queries)
    px, py, pz = _soa(points)
    out = np.empty(len(qx), dtype=np.int32)
    lib.og_nn_bruteforce(_p(qx), _p(qy), _p(qz), len(qx), _p(px), _p(py), _p(pz), len(px), _p(out))
    return out


def eval_field(dims, lo, hi, D: np.ndarray, x) -> Optional[tuple]:
    """f(x) and grad f(x) of the trilinear field (Eq. 1), or None outside."""
    lib = _load()
    R, L, H = _grid(dims, lo, hi)
    D = np.ascontiguousarray(D, dtype=np.float64)
    f = np.zeros(1)
    g = np.zeros(3)
    ok = lib.og_eval(_p(R), _p(L), _p(H), _p(D), float(x[0]), float(x[1]), float(x[2]), _p(f), _p(g))
    return (float(f[0]), g) if ok else None


def loss_grad(dims, lo, hi, cell_flags, vert_flags, D, queries, nn, points,
              alpha=1.0, beta=1.0, gamma=0.005, eps_n=1e-12,
              want_grad=True, per_query=False, want_tau=False) -> dict:
    """Total loss of Eq. 8 with its terms, the valid-query count and dL/dD."""
    lib = _load()
    R, L, H = _grid(dims, lo, hi)
    D = np.ascontiguousarray(D, dtype=np.float64)
    qx, qy, qz = _soa(queries)
    px, py, pz = _soa(points)
    nn = np.ascontiguousarray(nn, dtype=np.int32)
    terms = np.zeros(5)
    grad = np.zeros(len(D)) if want_grad else None
    pq = np.zeros((len(qx), 4)) if per_query else None
    tau = np.zeros(len(D)) if want_tau else None
    cf = np.ascontiguousarray(cell_flags, dtype=np.uint8)
    vf = np.ascontiguousarray(vert_flags, dtype=np.uint8)
    nvalid = lib.og_loss_grad(_p(R), _p(L), _p(H), _p(cf), _p(vf), _p(D),
                              _p(qx), _p(qy), _p(qz), _p(nn), len(qx), _p(px), _p(py), _p(pz),
                              float(alpha), float(beta), float(gamma), float(eps_n), _p(terms),
                              _p(grad) if grad is not None else None,
                              _p(pq) if pq is not None else None,
                              _p(tau) if tau is not None else None)
    if nvalid < 0:
        raise DomainError("a nearest point lies outside the grid domain")
    out = {"total": terms[0], "pull": terms[1], "tv": terms[2], "surf": terms[3], "grad": terms[4],
           "terms": terms, "n_valid": int(nvalid)}
    if grad is not None:
        out["dD"] = grad
    if pq is not None:
        out["per_query"] = pq
    if tau is not None:
        out["tau"] = tau
    return out


def adam(D, G, m, v, vert_flags, t: int, lr0: float, decay: float = 0.3, decay_every: int = 400,
         beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8) -> None:
    """One Adam step (Sec. 4 "Details") on the optimised vertices, in place (float64 arrays)."""
    lib = _load()
    for a in (D, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    G = np.ascontiguousarray(G, dtype=np.float64)
    vf = np.ascontiguousarray(vert_flags, dtype=np.uint8)
    lib.og_adam(len(D), _p(D), _p(G), _p(m), _p(v), _p(vf), int(t), float(lr0), float(decay),
                int(decay_every), float(beta1), float(beta2), float(eps))


def philox4x32_10(ctr: Sequence[int], key: Sequence[int]) -> np.ndarray:
    lib = _load()
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib.og_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def query_offsets(seed: int, iteration: int, stream: int, k0: int, n: int) -> np.ndarray:
    """Standard-normal offsets z_k (Philox4x32-10 + Box-Muller), float64 [n, 3]."""
    lib = _load()
    z = np.zeros((n, 3))
    lib.og_query_offsets(int(seed), int(iteration), int(stream), int(k0), int(n), _p(z))
    return z


def nn_exact(queries: np.ndarray, points: np.ndarray, k: int = 16, workers: int = -1) -> np.ndarray:
    """The same NN(q) as nn_bruteforce, for inputs too large for brute force.

    A k-d tree (scipy, a library primitive) proposes the k nearest candidates;
    they are re-ranked with the exact double distance and lowest-index tie rule
    of og_nn_bruteforce.  Queries whose k-th candidate is not clearly farther
    than the best (a possible tie or near tie beyond k) are re-run by brute
    force, so the result does not depend on the tree's own rounding.
    """
    from scipy.spatial import cKDTree

    q = np.asarray(queries, np.float32)
    p = np.asarray(points, np.float32)
    J = len(p)
    if J == 0:
        return np.full(len(q), -1, np.int32)
    k = min(k, J)
    tree = cKDTree(p.astype(np.float64))
    d, idx = tree.query(q.astype(np.float64), k=k, workers=workers)
    if k == 1:
        d = d[:, None]
        idx = idx[:, None]
    qd = q.astype(np.float64)
    pd = p.astype(np.float64)
    dx = qd[:, None, 0] - pd[idx, 0]
    dy = qd[:, None, 1] - pd[idx, 1]
    dz = qd[:, None, 2] - pd[idx, 2]
    d2 = (dx * dx + dy * dy) + dz * dz
    best = d2.min(axis=1)
    cand = np.where(d2 == best[:, None], idx, np.iinfo(np.int64).max)
    out = cand.min(axis=1).astype(np.int32)
    unsafe = (d[:, -1] <= np.sqrt(best) * (1 + 1e-7) + 1e-12) & (k < J)
    if np.any(unsafe):
        sel = np.nonzero(unsafe)[0]
        out[sel] = nn_bruteforce(q[sel], p)
    return out


def extract_surface(dims, lo, hi, D: np.ndarray, vert_flags: np.ndarray):
    """Zero level set of the field over the cells whose eight corners are
    optimised (the mesh step after the optimisation, Sec. 3/4), by marching
    tetrahedra (six per cell along its main diagonal; the C file states the
    reading).  Returns (keys int64 [n] = cell_id * 16 + tet * 2 + triangle,
    triangles float64 [n, 3, 3]) in key order."""
    lib = _load()
    R, L, H = _grid(dims, lo, hi)
    Dd = np.ascontiguousarray(D, dtype=np.float64)
    vf = np.ascontiguousarray(vert_flags, dtype=np.uint8)
    n = lib.og_extract_surface(_p(R), _p(L), _p(H), _p(Dd), _p(vf), 0, None, None)
    keys = np.zeros(max(n, 1), dtype=np.int64)
    xyz = np.zeros((max(n, 1), 3, 3), dtype=np.float64)
    lib.og_extract_surface(_p(R), _p(L), _p(H), _p(Dd), _p(vf), n, _p(keys), _p(xyz))
    return keys[:n], xyz[:n]


def marching_cubes(dims, lo, hi, D: np.ndarray, vert_flags: np.ndarray):
    """Zero level set of the field over the cells whose eight corners are
    optimised, by marching cubes (Sec. 3, last paragraph; Sec. 4 "Details");
    the C file states the face rule that resolves ambiguous faces.  Returns
    (keys int64 [n] = cell_id * 16 + triangle number in the cell, triangles
    float64 [n, 3, 3]) in key order."""
    lib = _load()
    R, L, H = _grid(dims, lo, hi)
    Dd = np.ascontiguousarray(D, dtype=np.float64)
    vf = np.ascontiguousarray(vert_flags, dtype=np.uint8)
    n = lib.og_marching_cubes(_p(R), _p(L), _p(H), _p(Dd), _p(vf), 0, None, None)
    if n < 0:
        raise RuntimeError("marching cubes: a configuration's face segments do not close")
    keys = np.zeros(max(n, 1), dtype=np.int64)
    xyz = np.zeros((max(n, 1), 3, 3), dtype=np.float64)
    lib.og_marching_cubes(_p(R), _p(L), _p(H), _p(Dd), _p(vf), n, _p(keys), _p(xyz))
    return keys[:n], xyz[:n]


def marching_cubes_counts() -> np.ndarray:
    """Triangles per corner configuration (bit i: corner i = 4a + 2b + c inside)."""
    lib = _load()
    out = np.zeros(256, dtype=np.int32)
    lib.og_mc_counts(_p(out))
    return out


def normal_term(dims, lo, hi, cell_flags, D, queries, nn, points, normals, weight: float = 1.0,
                eps_n: float = 1e-12, with_grad: bool = True):
    """Normal supervision (Sec. 4, normals paragraph; the C file states the
    reading): L_N = mean over valid queries of 1 - gh_s . n_s at s = NN(q).
    Returns (L_N, weight * dL_N/dD as a dense vertex array or None, Q_v)."""
    lib = _load()
    R, L, H = _grid(dims, lo, hi)
    qx, qy, qz = _soa(queries)
    px, py, pz = _soa(points)
    nx, ny, nz = _soa(normals)
    nn = np.ascontiguousarray(nn, dtype=np.int32)
    Dd = np.ascontiguousarray(D, dtype=np.float64)
    cf = np.ascontiguousarray(cell_flags, dtype=np.uint8)
    grad = np.zeros(int(np.prod(R.astype(np.int64) + 1)), dtype=np.float64) if with_grad else None
    term = np.zeros(1, dtype=np.float64)
    nv = lib.og_normal_term(_p(R), _p(L), _p(H), _p(cf), _p(Dd), _p(qx), _p(qy), _p(qz), _p(nn), len(qx),
                            _p(px), _p(py), _p(pz), _p(nx), _p(ny), _p(nz), float(weight), float(eps_n),
                            _p(term), _p(grad) if grad is not None else None)
    if nv < 0:
        raise DomainError("a nearest point lies outside the grid")
    return float(term[0]), grad, int(nv)
