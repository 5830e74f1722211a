"""Shared helpers of the GPU parity tests (no method arithmetic here)."""
import sys

import numpy as np

import oracle
from paper_2308_13175_amd import synth


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def make_problem(specs, m1=3, m2=3, weights=(1.0, 1.0, 0.005), adam=None, brick=8):
    from paper_2308_13175_amd.problem import Problem

    return Problem(specs, m1=m1, m2=m2, weights=weights, adam=adam, brick=brick)


def spec(points, dom, n_queries, sigma):
    from paper_2308_13175_amd.problem import ShapeSpec

    return ShapeSpec(points, dom.dims, dom.lo, dom.hi, n_queries, sigma)


def _cell_of_vertex(dom, vid):
    V = np.asarray(dom.vdims, dtype=np.int64)
    R = np.asarray(dom.dims, dtype=np.int64)
    i = vid // (V[1] * V[2])
    j = (vid // V[2]) % V[1]
    k = vid % V[2]
    ok = (i < R[0]) & (j < R[1]) & (k < R[2])
    return ok, (i * R[1] + j) * R[2] + k


def compare_band(prob, shape_index, dom, cf, vf):
    """Bit-exact comparison of the exported band with the oracle's dense flags.

    Compares sorted id sets: optimised and TV vertices, point cells, M1 and M2
    cells (a cell is reported on the slot of its lowest corner).
    """
    vid, flags = prob.layout()
    b, e = prob.slot_begin[shape_index], prob.slot_begin[shape_index + 1]
    vid, flags = vid[b:e], flags[b:e]
    have = vid >= 0
    vid, flags = vid[have], flags[have]
    assert len(np.unique(vid)) == len(vid), "a vertex appears in two slots"
    for bit, obit, what in ((1, 1, "optimised vertex"), (2, 2, "TV vertex")):
        got = np.sort(vid[(flags & bit) > 0])
        ref = np.nonzero(vf & obit)[0]
        assert np.array_equal(got, ref), "%s set differs (%d vs %d)" % (what, len(got), len(ref))
    for bit, obit, what in ((16, 1, "point cell"), (4, 2, "M1 cell"), (8, 4, "M2 cell")):
        sel = (flags & bit) > 0
        ok, cid = _cell_of_vertex(dom, vid[sel])
        assert np.all(ok), "%s flag on a vertex with no cell" % what
        got = np.sort(cid)
        ref = np.nonzero(cf & obit)[0]
        assert np.array_equal(got, ref), "%s set differs (%d vs %d)" % (what, len(got), len(ref))


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
    log("  gradient: max err %.3e / max |g| %.3e = %.2e" % (err, gmax, err / gmax))
    assert err <= rtol * gmax, "gradient: max err %.3e vs max |g| %.3e (rel %.2e)" % (err, gmax, err / gmax)
