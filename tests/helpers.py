"""Shared helpers of the GPU parity tests (no method arithmetic here)."""
import sys

import numpy as np

import oracle
from paper_2308_13175_amd import synth


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def make_problem(specs, m1=3, m2=3, weights=(1.0, 1.0, 0.005), adam=None):
    from paper_2308_13175_amd.problem import Problem

    return Problem(specs, m1=m1, m2=m2, weights=weights, adam=adam)


def spec(points, dom, n_queries, sigma):
    from paper_2308_13175_amd.problem import ShapeSpec

    return ShapeSpec(points, dom.dims, dom.lo, dom.hi, n_queries, sigma)


def slot_flags_by_vertex(prob, shape_index, dom):
    """Per vertex id of one shape: the slot flags the library exported (or -1 if no slot)."""
    vid, flags = prob.layout()
    b, e = prob.slot_begin[shape_index], prob.slot_begin[shape_index + 1]
    vid, flags = vid[b:e], flags[b:e]
    have = vid >= 0
    out = np.full(dom.n_vertices, -1, dtype=np.int16)
    assert len(np.unique(vid[have])) == int(have.sum()), "a vertex appears in two slots"
    out[vid[have]] = flags[have]
    return out


def compare_band(prob, shape_index, dom, cf, vf):
    """Bit-exact comparison of the exported band with the oracle's dense flags."""
    got = slot_flags_by_vertex(prob, shape_index, dom)
    V = np.asarray(dom.vdims)
    R = np.asarray(dom.dims)
    # vertex sets: optimised (1) and TV (2)
    in_slot = got >= 0
    g = np.where(in_slot, got, 0).astype(np.uint8)
    assert np.array_equal((g & 1) > 0, (vf & 1) > 0), "optimised vertex set differs"
    assert np.array_equal((g & 2) > 0, (vf & 2) > 0), "TV vertex set differs"
    # cell sets: bits 4 (M1), 8 (M2), 16 (point cells) on the cell's lowest corner
    ijk = np.stack(np.meshgrid(np.arange(R[0]), np.arange(R[1]), np.arange(R[2]), indexing="ij"), -1).reshape(-1, 3)
    lower = (ijk[:, 0] * V[1] + ijk[:, 1]) * V[2] + ijk[:, 2]
    gc = np.where(got[lower] >= 0, got[lower], 0).astype(np.uint8)
    assert np.array_equal((gc & 16) > 0, (cf & 1) > 0), "point-cell set differs"
    assert np.array_equal((gc & 4) > 0, (cf & 2) > 0), "M1 band differs"
    assert np.array_equal((gc & 8) > 0, (cf & 4) > 0), "M2 band differs"


def loss_terms(prob):
    return prob.loss.cpu().numpy(), prob.n_valid.cpu().numpy()


def assert_terms_close(got, ref, rtol=1e-5):
    names = ("total", "pull", "tv", "surf", "grad")
    for i, k in enumerate(names):
        err = abs(got[i] - ref[k])
        assert err <= rtol * abs(ref[k]) + 1e-12, "%s: got %.10e oracle %.10e (rel %.2e)" % (
            k, got[i], ref[k], err / max(abs(ref[k]), 1e-300))


def assert_grad_close(got, ref, rtol=1e-5):
    gmax = np.abs(ref).max()
    err = np.abs(got - ref).max()
    assert err <= rtol * gmax, "gradient: max err %.3e vs max |g| %.3e (rel %.2e)" % (err, gmax, err / gmax)
