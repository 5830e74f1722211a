"""Full-size parity: the workloads at their real grid, point and query counts.

Nearest neighbours of the oracle come from oracle.nn_exact (a k-d tree
proposes candidates, the exact double distance and lowest-index rule decide),
which is pinned against the brute force in the CPU tests.
"""
import numpy as np
import pytest

import oracle
from paper_2308_13175_amd import synth
from helpers import assert_grad_close, assert_terms_close, compare_band, log, loss_terms, make_problem, spec

pytestmark = pytest.mark.gpu


def _full_parity(pts, dom, q, D, sigma=0.0, m1=3, m2=3, check_band=True):
    prob = make_problem([spec(pts, dom, len(q), sigma)], m1=m1, m2=m2)
    prob.set_dense_field([D])
    prob.set_queries(q)
    prob.nearest()
    prob.forward()
    prob.backward()
    prob.sync()
    log("  gpu done: %d slots" % prob.n_slots)
    cf, vf = oracle.build_band(dom.dims, dom.lo, dom.hi, pts, m1, m2)
    if check_band:
        compare_band(prob, 0, dom, cf, vf)
    log("  band ok")
    nn_ref = oracle.nn_exact(q, pts)
    got_nn = prob.nn[: len(q)].cpu().numpy()
    bad = np.nonzero(got_nn != nn_ref)[0]
    assert len(bad) == 0, "%d of %d nearest neighbours differ, e.g. query %d: %d vs %d" % (
        len(bad), len(q), bad[0], got_nn[bad[0]], nn_ref[bad[0]])
    log("  nn ok")
    ref = oracle.loss_grad(dom.dims, dom.lo, dom.hi, cf, vf, D.astype(np.float64), q, nn_ref, pts)
    got, nv = loss_terms(prob)
    assert int(nv[0]) == ref["n_valid"]
    assert_terms_close(got[0], ref)
    assert_grad_close(prob.dense_grad()[0], ref["dD"])
    log("  loss/grad ok: L=%.6e valid=%d" % (ref["total"], ref["n_valid"]))
    prob.close()


def test_torus_200k_128_full_size():
    log("case: torus 200k points, 128^3, 1M queries, per-point sigma")
    wl = synth.torus_workload()
    s = wl.shapes[0]
    q = synth.host_queries(s.points, s.n_queries, s.sigma, seed=5)
    D = synth.sphere_sdf_field(s.domain, 0.5, noise=0.01, seed=2)
    _full_parity(s.points, s.domain, q, D, sigma=s.sigma)


def test_union24_2M_256_full_size():
    log("case: union of 24 primitives, 2M points, 256^3, 4M queries")
    wl = synth.union24_workload()
    s = wl.shapes[0]
    q = synth.host_queries(s.points, s.n_queries, s.sigma, seed=6)
    D = synth.sphere_sdf_field(s.domain, 0.6, noise=0.005, seed=3)
    _full_parity(s.points, s.domain, q, D, sigma=s.sigma)


def test_room_20M_full_grid_sampler_stream():
    """The room at its full grid: a 2M-query slice of the GPU sampler's own
    stream for the workload's 32M queries (stratified sources over the
    cell-sorted points, sigma = 2h), block-aligned, so that the gradient
    pass's blocks see the windows and slabs of the real run at full-grid
    coordinates."""
    log("case: room, 20M points, 1024x820x308, 2M queries of the sampler's 32M stream")
    wl = synth.room_workload()
    s = wl.shapes[0]
    stream = make_problem([spec(s.points, s.domain, s.n_queries, s.sigma)])
    stream.sample(seed=11, iteration=3)
    k0, n = 10 * 1024 * 1024, 2_000_000
    q = stream.queries()[k0:k0 + n].copy()
    stream.close()
    log("  sampled")
    ctr = [0.5 * (s.domain.lo[a] + s.domain.hi[a]) for a in range(3)]
    D = synth.sphere_sdf_field(s.domain, 2.0, noise=0.002, seed=4, centre=ctr)
    _full_parity(s.points, s.domain, q, D, sigma=s.sigma)


def test_batched_64_shapes_vs_single_and_oracle():
    """64 uneven shapes in one context, Q_i = 10 J_i queries each from the GPU
    sampler's stream (sigma = 2 h_i): each shape equals its own single-shape
    run (1e-5 relative) and the oracle."""
    log("case: 64 shapes batched, queries = 10 x points per shape")
    wl = synth.batched_workload()
    specs = [spec(s.points, s.domain, s.n_queries, s.sigma) for s in wl.shapes]
    Ds = [synth.sphere_sdf_field(s.domain, 0.4, noise=0.01, seed=i) for i, s in enumerate(wl.shapes)]
    batch = make_problem(specs)
    batch.set_dense_field(Ds)
    batch.sample(seed=21, iteration=2)
    batch.nearest()
    batch.forward()
    batch.backward()
    batch.sync()
    qall = batch.queries()
    bl, bn = loss_terms(batch)
    bg = batch.dense_grad()
    bnn = batch.nn[: batch.n_queries].cpu().numpy()
    batch.close()
    log("  batch done: %d queries" % len(qall))
    off = 0
    for i, s in enumerate(wl.shapes):
        q = qall[off:off + s.n_queries]
        single = make_problem([specs[i]])
        single.set_dense_field([Ds[i]])
        single.set_queries(q)
        single.nearest()
        single.forward()
        single.backward()
        sl, sn = loss_terms(single)
        assert bn[i] == sn[0]
        assert np.array_equal(bnn[off:off + len(q)], single.nn[: len(q)].cpu().numpy())
        rel = np.abs(bl[i] - sl[0]) / np.maximum(np.abs(sl[0]), 1e-30)
        assert np.max(rel) <= 1e-5, (i, rel)
        sg = single.dense_grad()[0]
        assert np.max(np.abs(bg[i] - sg)) <= 1e-5 * np.abs(sg).max()
        single.close()
        dom = s.domain
        cf, vf = oracle.build_band(dom.dims, dom.lo, dom.hi, s.points, 3, 3)
        nn_ref = oracle.nn_exact(q, s.points)
        assert np.array_equal(bnn[off:off + len(q)], nn_ref)
        ref = oracle.loss_grad(dom.dims, dom.lo, dom.hi, cf, vf, Ds[i].astype(np.float64), q, nn_ref, s.points)
        assert int(bn[i]) == ref["n_valid"]
        assert_terms_close(bl[i], ref)
        assert_grad_close(bg[i], ref["dD"])
        log("  shape %d (J=%d, Q=%d, R=%d) ok" % (i, len(s.points), len(q), dom.dims[0]))
        off += len(q)
