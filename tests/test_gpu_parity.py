"""HIP path vs the FP64 oracle, element by element, on seeded inputs.

Bar: bit-exact for band sets, valid-query counts and nearest-neighbour
indices; per-step loss terms within 1e-5 relative; gradients within 1e-5 of
the largest oracle gradient entry (norm-relative).
"""
import math

import numpy as np
import pytest

import oracle
from paper_2308_13175_amd import synth
from helpers import (assert_grad_close, assert_terms_close, compare_band, log, loss_terms, make_problem, spec)

pytestmark = pytest.mark.gpu


def _sphere_case(res=64, J=10_000, Q=50_000, sigma=0.02, m1=3, m2=3, seed=0):
    dom = synth.cube_domain(res)
    pts = synth.sphere_points(J, 0.5, seed=seed)
    q = synth.host_queries(pts, Q, sigma, seed=seed + 100)
    D = synth.sphere_sdf_field(dom, 0.5, noise=0.01, seed=seed)
    return dom, pts, q, D


def _run_gpu(dom, pts, q, D, m1=3, m2=3, weights=(1.0, 1.0, 0.005), brick=8):
    prob = make_problem([spec(pts, dom, len(q), 0.0)], m1=m1, m2=m2, weights=weights, brick=brick)
    prob.set_dense_field([D])
    prob.set_queries(q)
    prob.nearest()
    prob.forward()
    prob.grad.zero_()
    prob.backward()
    prob.sync()
    return prob


def _oracle(dom, pts, q, D, m1=3, m2=3, weights=(1.0, 1.0, 0.005)):
    cf, vf = oracle.build_band(dom.dims, dom.lo, dom.hi, pts, m1, m2)
    nn = oracle.nn_bruteforce(q, pts)
    ref = oracle.loss_grad(dom.dims, dom.lo, dom.hi, cf, vf, D.astype(np.float64), q, nn, pts, *weights)
    return cf, vf, nn, ref


@pytest.mark.parametrize("m1,m2,brick", [(3, 3, 8), (1, 4, 8), (4, 2, 8), (3, 14, 8), (3, 3, 4), (4, 2, 4),
                                         (3, 14, 16), (1, 4, 16)])
def test_sphere_64_parity(m1, m2, brick):
    """Band sets, NN, loss terms and gradient on the 64^3 sphere for several
    band widths and every brick size."""
    log("case: sphere 64^3 J=10k Q=50k m1=%d m2=%d brick %d" % (m1, m2, brick))
    dom, pts, q, D = _sphere_case()
    prob = _run_gpu(dom, pts, q, D, m1, m2, brick=brick)
    cf, vf, nn, ref = _oracle(dom, pts, q, D, m1, m2)
    compare_band(prob, 0, dom, cf, vf)
    assert prob.n_active == int((vf & 1).sum())
    from paper_2308_13175_amd import gridpull as gp
    cells = gp.gp_export_active_cells(prob.ctx, 0).cpu().numpy()
    assert np.array_equal(cells, np.nonzero(cf & 2)[0])
    assert np.array_equal(prob.nn[: len(q)].cpu().numpy(), nn)
    got, nv = loss_terms(prob)
    assert int(nv[0]) == ref["n_valid"]
    assert_terms_close(got[0], ref)
    assert_grad_close(prob.dense_grad()[0], ref["dD"])
    prob.close()


@pytest.mark.parametrize("brick", [4, 16])
def test_brick_sizes_through_the_path(brick):
    """Bricks of 4^3 and 16^3 vertices through the rest of the path: the
    anisotropic grid with random values (bricks cut by the grid boundary) and
    a wide TV band, the fused forward + backward (the TV kernels in their
    block layout whatever layout is asked), Adam steps, surface extraction by
    marching cubes and the normal term, each against the oracle."""
    from paper_2308_13175_amd import gridpull as gp
    from paper_2308_13175_amd.problem import AdamConfig

    log("case: brick %d, anisotropic grid, fused pass, both TV layout requests" % brick)
    rng = np.random.default_rng(5)
    adom = synth.Domain((24, 17, 31), (-1.125, -0.625, -0.875), (0.875, 0.8125, 1.0625))
    apts = (synth.sphere_points(3000, 0.45, seed=3) + np.float32(0.05)).astype(np.float32)
    aq = synth.host_queries(apts, 9000, 0.05, seed=7)
    aD = rng.normal(size=adom.n_vertices).astype(np.float32) * 0.2
    cf, vf, nn, ref = _oracle(adom, apts, aq, aD, 2, 5)
    prob = make_problem([spec(apts, adom, len(aq), 0.0)], m1=2, m2=5, brick=brick)
    compare_band(prob, 0, adom, cf, vf)
    prob.set_dense_field([aD])
    prob.set_queries(aq)
    prob.nearest()
    assert np.array_equal(prob.nn[: len(aq)].cpu().numpy(), nn)
    for layout in (0, 2, 1):
        gp.gp_set_tv_layout(prob.ctx, layout)
        prob.grad.zero_()
        prob.forward_backward()
        prob.sync()
        got, nv = loss_terms(prob)
        assert int(nv[0]) == ref["n_valid"]
        assert_terms_close(got[0], ref)
        assert_grad_close(prob.dense_grad()[0], ref["dD"])
    prob.close()

    log("case: brick %d, Adam steps against the oracle's" % brick)
    import torch
    dom, pts, q, D = _sphere_case(res=32, J=2000, Q=4000, sigma=0.04, seed=6)
    prob = make_problem([spec(pts, dom, len(q), 0.0)], brick=brick)
    prob.set_dense_field([D])
    cf, vf = oracle.build_band(dom.dims, dom.lo, dom.hi, pts, 3, 3)
    rng = np.random.default_rng(0)
    Dd = D.astype(np.float64)
    m = np.zeros(dom.n_vertices)
    v = np.zeros(dom.n_vertices)
    act = (vf & 1) > 0
    for t in (1, 2, 401):
        G = (rng.normal(size=dom.n_vertices) * 10.0 ** rng.uniform(-6, -2, dom.n_vertices)).astype(np.float32)
        gp.gp_gather_vertices(prob.ctx, torch.from_numpy(G).cuda(), prob.grad)
        prob.step(t, lr0=0.01)
        oracle.adam(Dd, G.astype(np.float64), m, v, vf, t, lr0=0.01)
        got = prob.dense_field()[0]
        assert np.max(np.abs(got[act] - Dd[act])) <= 1e-5 * 0.01 * min(t, 20) + 1e-7, t
    prob.close()

    log("case: brick %d, marching cubes" % brick)
    dom, pts, q, D = _sphere_case()
    prob = make_problem([spec(pts, dom, 0, 0.0)], brick=brick)
    prob.set_dense_field([D])
    tri, key = gp.gp_extract_surface(prob.ctx, 0, prob.field, method=0)
    tri, key = tri.cpu().numpy(), key.cpu().numpy()
    cf, vf = oracle.build_band(dom.dims, dom.lo, dom.hi, pts, 3, 3)
    rkey, rtri = oracle.marching_cubes(dom.dims, dom.lo, dom.hi, D.astype(np.float64), vf)
    assert len(rkey) > 100 and np.array_equal(key, rkey)
    assert np.abs(tri.astype(np.float64) - rtri.astype(np.float32).astype(np.float64)).max() == 0.0
    prob.close()


def _row_turns(dom, pts, q, nn, cf, block=256, cap=4096, max_slabs=16, brick=8, linemap=2048):
    """Per block of the gradient pass, (slabs, turns): the slabs of its line
    box and the turns of LDS rows they take in all (0, 0 when the block sends
    its contributions straight to the gradient).  The box covers the cells of
    the block's queries in the M1 band and of their nearest points, plus one
    vertex, in lines of 16 consecutive slots (x, y / (16 / brick), z-brick);
    slabs are whole x layers of at most linemap lines; a slab takes one turn
    per cap / 16 of its distinct corner lines (at least one)."""
    R = np.array(dom.dims)
    S = {4: 2, 8: 3, 16: 4}[brick]
    L = 4 - S
    rows = cap // 16
    cell = lambda x: np.clip(np.floor((x.astype(np.float64) - dom.lo) / dom.h), 0, R - 1).astype(np.int64)
    cq, cs = cell(q), cell(pts[nn])
    ok = (cf[(cq[:, 0] * R[1] + cq[:, 1]) * R[2] + cq[:, 2]] & 2) != 0
    offs = np.array([[i >> 2, (i >> 1) & 1, i & 1] for i in range(8)])
    out = []
    for b in range(0, len(q), block):
        m = ok[b:b + block]
        if not m.any():
            continue
        c = np.concatenate([cq[b:b + block][m], cs[b:b + block][m]])
        lo, hi = c.min(0), c.max(0)
        nx = hi[0] - lo[0] + 2
        nzb = ((hi[2] + 1) >> S) - (lo[2] >> S) + 1
        nyl = ((hi[1] + 1) >> L) - (lo[1] >> L) + 1
        cross = nzb * nyl
        if cross > linemap:
            out.append((0, 0))
            continue
        layers = min(nx, linemap // cross)
        slabs = -(-nx // layers)
        if slabs > max_slabs:
            out.append((0, 0))
            continue
        v = (c[:, None, :] + offs[None]).reshape(-1, 3)
        line = np.stack([v[:, 0], v[:, 1] >> L, v[:, 2] >> S], 1)
        rx = line[:, 0] - lo[0]
        turns = 0
        for p in range(slabs):
            sel = line[(rx >= p * layers) & (rx < (p + 1) * layers)]
            n = len(np.unique((sel[:, 0] << 42) | (sel[:, 1] << 21) | sel[:, 2]))
            turns += max(1, -(-n // rows))
        out.append((slabs, turns))
    return np.array(out)


@pytest.mark.parametrize("case", ["one turn", "several turns", "several slabs", "no rows"])
def test_gradient_accumulation_paths(case):
    """A block of the gradient pass sums its contributions in LDS rows, one
    per 16-slot line of the gradient it touches: in one turn, in several
    turns when it touches more lines than there are rows, in slabs when its
    box has more lines than the line map, and straight to the gradient when
    it would take more slabs than the limit.  Queries around cell-sorted points with a
    small spread keep every block in one turn; a larger spread with half the
    rows needs two turns; sources drawn at random on a finer grid spread every
    block over the sphere (many slabs, or none under a limit of four).  The
    path of every block is computed on the host; each case against the
    oracle."""
    from paper_2308_13175_amd import gridpull as gp

    log("case: gradient accumulation, %s" % case)
    res, n, sigma, strat, cap, max_slabs = {"one turn": (64, 40_000, 0.01, True, 4096, 16),
                                            "several turns": (64, 80_000, 0.06, True, 2048, 16),
                                            "several slabs": (128, 40_000, 0.01, False, 4096, 16),
                                            "no rows": (128, 40_000, 0.01, False, 4096, 4)}[case]
    dom = synth.cube_domain(res)
    pts = synth.sphere_points(10_000, 0.5, seed=21)
    c = np.minimum(np.floor((pts.astype(np.float64) - dom.lo) / dom.h), res - 1).astype(np.int64)
    pts = pts[np.argsort((c[:, 0] * res + c[:, 1]) * res + c[:, 2], kind="stable")]
    q = synth.host_queries(pts, n, sigma, seed=22, stratified=strat)
    D = synth.sphere_sdf_field(dom, 0.5, noise=0.01, seed=23)
    cf, vf, nn, ref = _oracle(dom, pts, q, D)
    paths = _row_turns(dom, pts, q, nn, cf, cap=cap, max_slabs=max_slabs)
    log("  slabs per block: %s, turns per block: %s" % (np.bincount(paths[:, 0]).tolist(),
                                                        np.bincount(paths[:, 1]).tolist()))
    if case == "one turn":
        assert (paths[:, 1] == 1).all()
    elif case == "several turns":
        assert (paths[:, 0] == 1).all() and (paths[:, 1] >= 2).mean() > 0.3
    elif case == "several slabs":
        assert (paths[:, 0] >= 2).all()
    else:
        assert (paths[:, 0] == 0).mean() > 0.9
    prob = make_problem([spec(pts, dom, len(q), 0.0)])
    gp.gp_set_grad_params(prob.ctx, cap, max_slabs, 2048, 16384)
    prob.set_dense_field([D])
    prob.set_queries(q)
    prob.nearest()
    prob.forward()
    prob.grad.zero_()
    prob.backward()
    prob.sync()
    assert np.array_equal(prob.nn[: len(q)].cpu().numpy(), nn)
    got, nv = loss_terms(prob)
    assert int(nv[0]) == ref["n_valid"]
    assert_terms_close(got[0], ref)
    assert_grad_close(prob.dense_grad()[0], ref["dD"])
    prob.grad.zero_()
    prob.forward_backward()
    prob.sync()
    got, nv = loss_terms(prob)
    assert_terms_close(got[0], ref)
    assert_grad_close(prob.dense_grad()[0], ref["dD"])
    prob.close()


def test_large_contributions_bypass_the_rows():
    """Contributions of 2^19 or more go straight to the gradient (the fixed
    point of the LDS rows would overflow), mixed with small ones that take
    the rows.  A field scaled by 1e-7 has |grad f| near 1e-7, so the
    gradient-consistency adjoint (weight 1) carries 1/|grad f| ~ 1e7 (Eq. 7
    differentiated) while the pull and surface adjoints stay of order one.
    The largest such contribution is bounded below on the host from the
    oracle's per-query cosine term: gamma * sin(theta) / |grad f| * R / 2 per
    unit corner weight, with |grad f| <= 2e-7 for this field."""
    log("case: contributions beyond the fixed-point range")
    dom = synth.cube_domain(32)
    pts = synth.sphere_points(3000, 0.5, seed=31)
    q = synth.host_queries(pts, 12_000, 0.04, seed=32)
    D = (1e-7 * synth.sphere_sdf_field(dom, 0.5, noise=0.01, seed=33).astype(np.float64)).astype(np.float32)
    weights = (1.0, 1.0, 1.0)
    cf, vf = oracle.build_band(dom.dims, dom.lo, dom.hi, pts, 3, 3)
    nn = oracle.nn_bruteforce(q, pts)
    ref = oracle.loss_grad(dom.dims, dom.lo, dom.hi, cf, vf, D.astype(np.float64), q, nn, pts, *weights,
                           per_query=True)
    pq = ref["per_query"]
    lg = pq[pq[:, 3] > 0, 2]
    sin_max = float(np.sqrt(np.clip(lg * (2.0 - lg), 0.0, None)).max())
    # (corner weights of at least 1/8 on some corner of the cell: a factor 8 of margin)
    assert weights[2] * sin_max / 2e-7 * (dom.dims[0] / 2.0) / 8.0 >= 2.0 ** 19
    prob = _run_gpu(dom, pts, q, D, weights=weights)
    assert np.array_equal(prob.nn[: len(q)].cpu().numpy(), nn)
    got, nv = loss_terms(prob)
    assert int(nv[0]) == ref["n_valid"]
    assert_terms_close(got[0], ref)
    assert_grad_close(prob.dense_grad()[0], ref["dD"])
    prob.grad.zero_()
    prob.forward_backward()
    prob.sync()
    got, nv = loss_terms(prob)
    assert_terms_close(got[0], ref)
    assert_grad_close(prob.dense_grad()[0], ref["dD"])
    prob.close()


@pytest.mark.parametrize("cap,max_passes,brick", [(2048, 16, 8), (6144, 64, 8), (4096, 1, 8), (2048, 16, 4),
                                                   (6144, 64, 16), (2048, 4, 16)])
def test_window_settings_and_autotuner(cap, max_passes, brick):
    """The gradient pass at other row counts, slab limits and brick sizes (a
    block touching more lines than there are rows takes them in turns)
    gives the oracle's loss terms and gradient; so does the setting the
    autotuner picks, and out-of-range settings are refused."""
    from paper_2308_13175_amd import gridpull as gp

    log("case: rows of %d vertices, at most %d slabs, brick %d" % (cap, max_passes, brick))
    dom = synth.cube_domain(64)
    pts = synth.sphere_points(10_000, 0.5, seed=21)
    c = np.minimum(np.floor((pts.astype(np.float64) - dom.lo) / dom.h), 63).astype(np.int64)
    pts = pts[np.argsort((c[:, 0] * 64 + c[:, 1]) * 64 + c[:, 2], kind="stable")]
    q = synth.host_queries(pts, 80_000, 0.06, seed=22)
    D = synth.sphere_sdf_field(dom, 0.5, noise=0.01, seed=23)
    cf, vf, nn, ref = _oracle(dom, pts, q, D)
    paths = _row_turns(dom, pts, q, nn, cf, cap=cap, max_slabs=max_passes, brick=brick)
    log("  turns per block: %s" % np.bincount(paths[:, 1]).tolist())
    assert (paths[:, 0] == 1).all()
    if cap == 2048:
        assert (paths[:, 1] >= 2).any()
    prob = make_problem([spec(pts, dom, len(q), 0.0)], brick=brick)
    gp.gp_set_grad_params(prob.ctx, cap, max_passes, 2048, 16384)
    assert gp.gp_get_grad_params(prob.ctx) == (cap, max_passes, 2048, 16384)
    prob.set_dense_field([D])
    prob.set_queries(q)
    prob.nearest()

    def check():
        prob.forward()
        prob.grad.zero_()
        prob.backward()
        prob.sync()
        got, nv = loss_terms(prob)
        assert int(nv[0]) == ref["n_valid"]
        assert_terms_close(got[0], ref)
        assert_grad_close(prob.dense_grad()[0], ref["dD"])
        prob.grad.zero_()
        prob.forward_backward()
        prob.sync()
        got, nv = loss_terms(prob)
        assert_terms_close(got[0], ref)
        assert_grad_close(prob.dense_grad()[0], ref["dD"])

    check()
    log("  autotuner")
    prob.grad.fill_(3.0)
    chosen, ms = prob.autotune_grad(reps=1)
    prob.sync()
    assert chosen[0] in (2048, 4096, 6144) and 1 <= chosen[1] <= 64 and chosen[2] >= 0 and chosen[3] >= 0
    assert ms[0] > 0
    assert (ms[1] > 0 and ms[2] > 0) if brick == 8 else (ms[1] == -1 and ms[2] == -1)   # one TV layout only
    assert gp.gp_get_grad_params(prob.ctx) == chosen
    assert bool((prob.grad == 3.0).all())   # the caller's gradient is left alone
    check()
    for bad in [(4000, 16, 0, 0), (3584, 16, 0, 0), (4096, 0, 0, 0), (4096, 65, 0, 0), (4096, 16, -1, 0),
                (4096, 16, 0, -1)]:
        with pytest.raises(gp.GridPullError) as ei:
            gp.gp_set_grad_params(prob.ctx, *bad)
        assert ei.value.status == 1
    assert gp.gp_get_grad_params(prob.ctx) == chosen
    prob.close()


def test_anisotropic_grid_and_edge_cases():
    """Anisotropic cells, a point on hi, queries outside the domain, duplicate points."""
    log("case: anisotropic 24x17x31 with edge cases")
    # bounds exactly representable in float32, so points placed on lo/hi are inside
    dom = synth.Domain((24, 17, 31), (-1.125, -0.625, -0.875), (0.875, 0.8125, 1.0625))
    rng = np.random.default_rng(5)
    pts = (synth.sphere_points(3000, 0.45, seed=3) + np.float32(0.05)).astype(np.float32)
    pts[0] = np.array(dom.hi, dtype=np.float32)          # exactly on hi
    pts[1] = np.array(dom.lo, dtype=np.float32)          # exactly on lo
    pts[2] = pts[3]                                      # duplicate: NN ties
    q = synth.host_queries(pts, 9000, 0.05, seed=7)
    q[:20] = np.float32(3.0)                             # outside the domain
    q[20:40] = pts[3:23]                                 # exactly on points
    q[40] = pts[2]
    D = rng.normal(size=dom.n_vertices).astype(np.float32) * 0.2
    prob = _run_gpu(dom, pts, q, D, 2, 3)
    cf, vf, nn, ref = _oracle(dom, pts, q, D, 2, 3)
    compare_band(prob, 0, dom, cf, vf)
    got_nn = prob.nn[: len(q)].cpu().numpy()
    assert np.array_equal(got_nn, nn)
    assert got_nn[40] == 2
    got, nv = loss_terms(prob)
    assert int(nv[0]) == ref["n_valid"]
    assert_terms_close(got[0], ref)
    assert_grad_close(prob.dense_grad()[0], ref["dD"])
    prob.close()


@pytest.mark.parametrize("m1,m2", [(12, 12), (100, 3), (3, 1024), (11, 11)])
def test_dense_band_when_m_covers_the_grid(m1, m2):
    log("case: M >= R - 1 (every cell in the band), m1=%d m2=%d" % (m1, m2))
    dom = synth.cube_domain(12)
    pts = synth.sphere_points(500, 0.5, seed=9)
    q = synth.host_queries(pts, 3000, 0.2, seed=10)
    D = synth.sphere_sdf_field(dom, 0.5, noise=0.05, seed=1)
    prob = _run_gpu(dom, pts, q, D, m1, m2)
    cf, vf, nn, ref = _oracle(dom, pts, q, D, m1, m2)
    assert np.all(cf & (2 if m1 >= 11 else 4)) and np.all(vf & 1)
    compare_band(prob, 0, dom, cf, vf)
    got, nv = loss_terms(prob)
    assert int(nv[0]) == ref["n_valid"]
    assert_terms_close(got[0], ref)
    assert_grad_close(prob.dense_grad()[0], ref["dD"])
    prob.close()


def test_constant_field_takes_the_zero_gradient_path():
    log("case: constant field")
    dom = synth.cube_domain(16)
    pts = synth.sphere_points(400, 0.5, seed=11)
    q = synth.host_queries(pts, 2000, 0.05, seed=12)
    D = np.full(dom.n_vertices, 0.25, np.float32)
    prob = _run_gpu(dom, pts, q, D)
    cf, vf, nn, ref = _oracle(dom, pts, q, D)
    got, nv = loss_terms(prob)
    assert got[0][4] == 1.0 and ref["grad"] == 1.0
    assert_terms_close(got[0], ref)
    g = prob.dense_grad()[0]
    assert np.all(np.isfinite(g))
    assert_grad_close(g, ref["dD"])
    prob.close()


@pytest.mark.parametrize("weights", [(1.0, 0.0, 0.0), (0.0, 1.0, 0.0), (0.0, 0.0, 1.0), (2.0, 0.5, 0.3)])
def test_each_term_separately(weights):
    log("case: weights", weights)
    dom, pts, q, D = _sphere_case(res=32, J=3000, Q=12_000, sigma=0.04, seed=4)
    prob = _run_gpu(dom, pts, q, D, 3, 3, weights)
    _, _, _, ref = _oracle(dom, pts, q, D, 3, 3, weights)
    got, _ = loss_terms(prob)
    assert_terms_close(got[0], ref)
    assert_grad_close(prob.dense_grad()[0], ref["dD"])
    prob.close()


def test_adam_step_parity():
    import torch

    log("case: Adam steps")
    dom, pts, q, D = _sphere_case(res=32, J=2000, Q=4000, sigma=0.04, seed=6)
    prob = make_problem([spec(pts, dom, len(q), 0.0)])
    prob.set_dense_field([D])
    cf, vf = oracle.build_band(dom.dims, dom.lo, dom.hi, pts, 3, 3)
    rng = np.random.default_rng(0)
    Dd = D.astype(np.float64)
    m = np.zeros(dom.n_vertices)
    v = np.zeros(dom.n_vertices)
    # the first steps, then across the decays of the schedule (x0.3 at 401, 801, 1201)
    for t in (1, 2, 3, 399, 400, 401, 402, 799, 800, 801, 802, 1200, 1201):
        G = (rng.normal(size=dom.n_vertices) * 10.0 ** rng.uniform(-6, -2, dom.n_vertices)).astype(np.float32)
        dense_g = torch.from_numpy(G).cuda()
        from paper_2308_13175_amd import gridpull as gp
        gp.gp_gather_vertices(prob.ctx, dense_g, prob.grad)
        prob.step(t, lr0=0.01)
        oracle.adam(Dd, G.astype(np.float64), m, v, vf, t, lr0=0.01)
        got = prob.dense_field()[0]
        act = (vf & 1) > 0
        assert np.max(np.abs(got[act] - Dd[act])) <= 1e-5 * 0.01 * min(t, 20) + 1e-7, t
        # the gradient buffer is cleared by the step
        assert float(prob.grad.abs().max()) == 0.0
    # vertices outside the band never move (their slots are not exported)
    prob.close()


def test_init_sphere_matches_its_formula():
    """gp_init_sphere (Sec. 3, geometric initialisation) against the host
    formula |x_v - c| - r in double, rounded to float, at every vertex of the
    band, on an anisotropic grid with an off-centre sphere."""
    log("case: initial sphere")
    dom = synth.Domain((24, 17, 31), (-1.125, -0.625, -0.875), (0.875, 0.8125, 1.0625))
    pts = (synth.sphere_points(3000, 0.45, seed=3) + np.float32(0.05)).astype(np.float32)
    prob = make_problem([spec(pts, dom, 1000, 0.05)], m1=3, m2=5)
    c, r = (0.1, -0.05, 0.2), 0.07
    prob.init_sphere([c], [r])
    got = prob.dense_field(fill=np.nan)[0]
    V = dom.vdims
    idx = np.nonzero(~np.isnan(got))[0]
    i, j, k = idx // (V[1] * V[2]), (idx // V[2]) % V[1], idx % V[2]
    inv_h = np.array(dom.dims, np.float64) / (np.array(dom.hi) - np.array(dom.lo))
    x = [dom.lo[a] + np.array([i, j, k][a], np.float64) / inv_h[a] - c[a] for a in range(3)]
    ref = (np.sqrt(x[0] ** 2 + x[1] ** 2 + x[2] ** 2) - r).astype(np.float32)
    _, vf = oracle.build_band(dom.dims, dom.lo, dom.hi, pts, 3, 5)
    assert np.array_equal(np.sort(idx), np.nonzero(vf & 1)[0])
    ulp = np.spacing(np.abs(ref))
    assert np.all(np.abs(got[idx] - ref) <= ulp), np.max(np.abs(got[idx] - ref) / ulp)
    prob.close()


def test_sampler_offsets_and_stratification():
    import torch

    log("case: sampler")
    dom = synth.cube_domain(32)
    pts = synth.sphere_points(3000, 0.5, seed=13)
    sig = np.linspace(0.01, 0.05, len(pts)).astype(np.float32)
    Q = 7001                                     # not a multiple of J
    prob = make_problem([spec(pts, dom, Q, sig)])
    for it in (1, 2):
        prob.sample(seed=12345, iteration=it)
        prob.sync()
        q = prob.queries().astype(np.float64)
        src = prob.src[:Q].cpu().numpy()
        counts = np.bincount(src, minlength=len(pts))
        assert counts.min() >= Q // len(pts) and counts.max() <= -(-Q // len(pts))
        z = oracle.query_offsets(12345, it, 0, 0, Q)
        expect = pts[src].astype(np.float64) + sig[src][:, None].astype(np.float64) * z
        err = np.abs(q - expect)
        tol = sig[src][:, None] * (1e-5 * (1 + np.abs(z))) + 1e-6
        assert np.all(err <= tol), float(np.max(err / tol))
    prob.close()


def test_batched_equals_single_shape():
    log("case: batched vs single")
    shapes = []
    rng = np.random.default_rng(21)
    for i, res in enumerate((16, 32, 24)):
        dom = synth.Domain((res, res + 3, res - 2), (-1.0, -1.0, -1.0), (1.0, 1.1, 0.95))
        pts = synth.sphere_points(800 * (i + 1), 0.3 + 0.1 * i, seed=30 + i)
        q = synth.host_queries(pts, 3000 * (i + 1), 0.05, seed=40 + i)
        D = synth.sphere_sdf_field(dom, 0.3 + 0.1 * i, noise=0.02, seed=i)
        shapes.append((dom, pts, q, D))
    batch = make_problem([spec(p, d, len(q), 0.0) for d, p, q, D in shapes])
    batch.set_dense_field([D for d, p, q, D in shapes])
    batch.set_queries(np.concatenate([q for d, p, q, D in shapes]))
    batch.nearest()
    batch.forward()
    batch.backward()
    bl, bn = loss_terms(batch)
    bg = batch.dense_grad()
    for i, (dom, pts, q, D) in enumerate(shapes):
        single = _run_gpu(dom, pts, q, D)
        sl, sn = loss_terms(single)
        assert bn[i] == sn[0]
        assert np.max(np.abs(bl[i] - sl[0]) / np.maximum(np.abs(sl[0]), 1e-30)) <= 1e-5
        sg = single.dense_grad()[0]
        assert np.max(np.abs(bg[i] - sg)) <= 1e-5 * np.abs(sg).max()
        _, _, _, ref = _oracle(dom, pts, q, D)
        assert_terms_close(bl[i], ref)
        assert_grad_close(bg[i], ref["dD"])
        single.close()
    batch.close()


@pytest.mark.parametrize("m1,m2", [(3, 3), (1, 4), (4, 2)])
def test_fused_forward_backward(m1, m2):
    """gp_pull_forward_backward = gp_pull_forward + gp_pull_backward = the
    oracle (M1 < M2 puts band vertices outside the TV set, M1 > M2 the other
    way round); a second fused call on a cleared gradient gives the same result
    (its unscaled accumulator starts from zero again)."""
    import torch

    log("case: fused forward+backward, sphere 64^3 m1=%d m2=%d" % (m1, m2))
    dom, pts, q, D = _sphere_case()
    prob = _run_gpu(dom, pts, q, D, m1, m2)
    sep_loss, _ = loss_terms(prob)
    sep_grad = prob.dense_grad()[0]
    cf, vf, nn, ref = _oracle(dom, pts, q, D, m1, m2)
    for rep in range(2):
        prob.grad.zero_()
        prob.forward_backward()
        prob.sync()
        got, nv = loss_terms(prob)
        assert int(nv[0]) == ref["n_valid"]
        assert_terms_close(got[0], ref)
        np.testing.assert_allclose(got[0], sep_loss[0], rtol=1e-12, atol=0)
        g = prob.dense_grad()[0]
        assert_grad_close(g, ref["dD"])
        assert np.abs(g - sep_grad).max() <= 1e-6 * np.abs(sep_grad).max(), rep
    # a scaled upstream gradient scales the query and TV parts alike
    prob.grad.zero_()
    prob.forward_backward(dloss=torch.full((1,), 2.5, dtype=torch.float64, device=prob.device))
    g = prob.dense_grad()[0]
    assert np.abs(g - 2.5 * sep_grad).max() <= 1e-6 * 2.5 * np.abs(sep_grad).max()
    prob.close()


def _tie_case():
    dom = synth.Domain((40, 40, 40), (-1.0, -1.0, -1.0), (1.0, 1.0, 1.0))
    g = np.arange(-4, 5, dtype=np.float32) * np.float32(0.0625)      # lattice step 1/16, exact in float
    lat = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    rng = np.random.default_rng(3)
    pts = lat[rng.permutation(len(lat))].astype(np.float32)
    half = np.float32(0.03125)
    centres = lat[(lat[:, 0] < g[-1]) & (lat[:, 1] < g[-1]) & (lat[:, 2] < g[-1])] + half
    edges = lat[(lat[:, 0] < g[-1])] + np.array([half, 0, 0], np.float32)
    far = np.array([[0.9, 0.9, 0.9], [-0.95, 0.9, -0.9], [0.0, 0.95, 0.0], [0.93, -0.97, 0.11]], np.float32)
    q = np.concatenate([centres, edges, lat[:50], far]).astype(np.float32)
    q = q[rng.permutation(len(q))]
    D = synth.sphere_sdf_field(dom, 0.3, noise=0.02, seed=4)
    return dom, pts, q, D


def test_nn_exact_ties_and_distant_queries():
    """Points on a lattice in shuffled index order, queries at lattice cube
    centres and edge midpoints (8-way and 4-way exact ties: the lowest index
    must win), queries on lattice points, and queries many cells away from
    every point (the box grows to its limit, then the ring search)."""
    log("case: exact ties and distant queries")
    dom, pts, q, D = _tie_case()
    prob = _run_gpu(dom, pts, q, D, 3, 3)
    cf, vf, nn, ref = _oracle(dom, pts, q, D, 3, 3)
    got_nn = prob.nn[: len(q)].cpu().numpy()
    bad = np.nonzero(got_nn != nn)[0]
    assert len(bad) == 0, "%d of %d differ, e.g. query %s: %d vs %d" % (len(bad), len(q), q[bad[0]], got_nn[bad[0]], nn[bad[0]])
    got, nv = loss_terms(prob)
    assert int(nv[0]) == ref["n_valid"]
    assert_terms_close(got[0], ref)
    assert_grad_close(prob.dense_grad()[0], ref["dD"])
    prob.close()


def test_batch_with_a_shape_without_queries_and_a_one_point_shape():
    """A batch of three shapes: one with points but no queries, one with a
    single point, one ordinary; every shape agrees with the oracle."""
    log("case: batch with an empty query set and a one-point shape")
    dom0 = synth.cube_domain(16)
    dom1 = synth.Domain((20, 12, 16), (-0.5, -0.5, -0.5), (1.5, 0.7, 1.1))
    dom2 = synth.cube_domain(24)
    p0 = synth.sphere_points(300, 0.4, seed=50)
    p1 = np.array([[0.25, 0.05, 0.3]], np.float32)
    p2 = synth.sphere_points(900, 0.5, seed=51)
    q1 = synth.host_queries(p1, 500, 0.15, seed=52)
    q2 = synth.host_queries(p2, 4000, 0.05, seed=53)
    D = [synth.sphere_sdf_field(d, 0.4, noise=0.01, seed=i) for i, d in enumerate((dom0, dom1, dom2))]
    batch = make_problem([spec(p0, dom0, 0, 0.0), spec(p1, dom1, len(q1), 0.0), spec(p2, dom2, len(q2), 0.0)])
    batch.set_dense_field(D)
    batch.set_queries(np.concatenate([q1, q2]))
    batch.nearest()
    batch.forward()
    batch.backward()
    batch.sync()
    bl, bn = loss_terms(batch)
    bg = batch.dense_grad()
    nn = batch.nn[: len(q1) + len(q2)].cpu().numpy()
    assert np.all(nn[: len(q1)] == 0)
    for i, (dom, pts, q) in enumerate(((dom0, p0, np.zeros((0, 3), np.float32)), (dom1, p1, q1), (dom2, p2, q2))):
        cf, vf, onn, ref = _oracle(dom, pts, q, D[i])
        if i == 2:
            assert np.array_equal(nn[len(q1):], onn)
        assert int(bn[i]) == ref["n_valid"]
        assert_terms_close(bl[i], ref)
        if np.abs(ref["dD"]).max() > 0:
            assert_grad_close(bg[i], ref["dD"])
        else:
            assert np.abs(bg[i]).max() == 0.0
    batch.close()


def test_nn_search_shapes_and_autotuner():
    """Every NN search shape (group span, first shell, blocks per tile, empty
    cells skipped or not, search grids finer and coarser than the band),
    including the extremes, and the autotuner's choice give the oracle's
    indices exactly, on the exact-tie lattice and on a sparse sphere (few
    points per cell, so most queries leave the lockstep box open and most
    scanned cells are empty)."""
    from paper_2308_13175_amd import gridpull as gp
    sparse = synth.cube_domain(64), synth.sphere_points(1500, 0.5, seed=7)
    cases = [("ties",) + _tie_case()[:3],
             ("sparse sphere", sparse[0], sparse[1], synth.host_queries(sparse[1], 30_000, 0.04, seed=8))]
    for name, dom, pts, q in cases:
        nn = oracle.nn_bruteforce(q, pts)
        prob = make_problem([spec(pts, dom, len(q), 0.0)])
        prob.set_queries(q)
        assert gp.gp_get_nn_params(prob.ctx) == (8, 1, 1, 0, 1, 8)
        for shape in [(1, 0, 1, 0, 1), (2, 0, 4, 1, 0), (3, 2, 2, 0, 1), (8, 1, 4, 1, 1), (8, 1, 1, 1, 0),
                      (16, 0, 2, 1, 1), (64, 4, 1, 0, 0), (64, 4, 4, 1, 1), (8, 1, 1, 0, 1, 1),
                      (8, 1, 2, 1, 1, 256), (4, 0, 1, 1, 1, 4096), (8, 1, 1, 0, 1, 8)]:
            log("case: %s, search shape %s" % (name, shape))
            gp.gp_set_nn_params(prob.ctx, *shape)
            prob.nn.fill_(-7)
            prob.nearest()
            prob.sync()
            got = prob.nn[: len(q)].cpu().numpy()
            bad = np.nonzero(got != nn)[0]
            assert len(bad) == 0, "%s shape %s: %d differ" % (name, shape, len(bad))
        log("case: %s, autotuner" % name)
        gp.gp_set_nn_params(prob.ctx, 8, 1, 1, 0, 1)   # the tuner starts from the current setting
        prob.nn.fill_(-7)
        chosen, ms = prob.autotune(reps=1)
        prob.sync()
        span, shell, parts, skip, sort, cell_points = chosen
        assert span in (4, 6, 8, 12, 16, 24, 32) and shell in (0, 1, 2) and parts in (1, 2, 4)
        assert skip in (0, 1) and sort in (0, 1) and 1 <= cell_points <= 65536
        assert ms > 0
        assert gp.gp_get_nn_params(prob.ctx) == chosen
        assert np.array_equal(prob.nn[: len(q)].cpu().numpy(), nn)
        prob.nearest()
        prob.sync()
        assert np.array_equal(prob.nn[: len(q)].cpu().numpy(), nn)
        for bad_args in [(0, 1, 1, 0, 1), (65, 1, 1, 0, 1), (8, -1, 1, 0, 1), (8, 5, 1, 0, 1), (8, 1, 3, 0, 1),
                         (8, 1, 0, 0, 1), (8, 1, 1, 2, 1), (8, 1, 1, 0, 2), (8, 1, 1, 0, 1, 0),
                         (8, 1, 1, 0, 1, 65537)]:
            with pytest.raises(gp.GridPullError) as ei:
                gp.gp_set_nn_params(prob.ctx, *bad_args)
            assert ei.value.status == 1
        assert gp.gp_get_nn_params(prob.ctx) == chosen
        prob.close()


def _search_level(dom, pts, cell_points):
    """The search grid's level from its definition: k nearest to
    log2(cell_points / m) / 2 within [0, 3], m the mean number of points per
    band cell holding a point (cells by the library's location rule)."""
    lo, hi, R = np.asarray(dom.lo, np.float64), np.asarray(dom.hi, np.float64), np.asarray(dom.dims, np.int64)
    u = (pts.astype(np.float64) - lo) * (R / (hi - lo))
    c = np.clip(np.floor(u), 0, R - 1).astype(np.int64)
    occupied = len(np.unique((c[:, 0] * R[1] + c[:, 1]) * R[2] + c[:, 2]))
    return int(min(3, max(0, round(0.5 * math.log2(cell_points / (len(pts) / occupied))))))


@pytest.mark.parametrize("res", [16, 32, 64, 128, 256])
def test_nn_search_grid_across_band_resolutions(res):
    """The same torus at band resolutions 16 to 256: the search grid takes the
    level its definition gives (the band's cells where the points are dense,
    up to 8 band cells wide where they are sparse), covers the box, and the
    nearest points equal brute force bit for bit at each resolution and at
    three other density targets."""
    from paper_2308_13175_amd import gridpull as gp
    dom = synth.cube_domain(res)
    pts = synth.torus_points(20_000, seed=1)
    q = synth.host_queries(pts, 20_000, 0.03, seed=2)
    ref = oracle.nn_bruteforce(q, pts)
    prob = make_problem([spec(pts, dom, len(q), 0.0)])
    prob.set_queries(q)
    for cell_points in (8, 1, 64, 4096):
        log("case: torus R=%d, cell_points %d" % (res, cell_points))
        gp.gp_set_nn_params(prob.ctx, 8, 1, 1, 0, 1, cell_points)
        dims, level = gp.gp_get_nn_grid(prob.ctx, 0)
        assert level == _search_level(dom, pts, cell_points)
        f = 2.0 ** level
        assert dims == tuple(int(math.ceil(r / f)) for r in dom.dims)
        prob.nn.fill_(-7)
        prob.nearest()
        prob.sync()
        got = prob.nn[: len(q)].cpu().numpy()
        bad = np.nonzero(got != ref)[0]
        assert len(bad) == 0, "R=%d cell_points %d: %d differ" % (res, cell_points, len(bad))
    prob.close()


def test_nn_points_on_search_cell_faces():
    """Points on the faces of coarse search cells (a lattice of band vertices,
    so at levels 1 to 3 every point lies on search-cell faces), queries at the
    lattice's cell centres (8-way ties), on the points themselves and at random:
    the search's cell assignment at a face and its gap bounds still give brute
    force's indices bit for bit at every level."""
    from paper_2308_13175_amd import gridpull as gp
    dom = synth.Domain((32, 32, 32), (-1.0, -1.0, -1.0), (1.0, 1.0, 1.0))
    g = (np.arange(4, 29, 4, dtype=np.float32) * np.float32(0.0625) - np.float32(1.0))   # every 4th vertex
    lat = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3).astype(np.float32)
    rng = np.random.default_rng(11)
    pts = lat[rng.permutation(len(lat))]
    centres = (lat[(lat < g[-1]).all(1)] + np.float32(0.125)).astype(np.float32)
    q = np.concatenate([centres, lat[:100], rng.uniform(-1, 1, (4000, 3)).astype(np.float32)]).astype(np.float32)
    ref = oracle.nn_bruteforce(q, pts)
    prob = make_problem([spec(pts, dom, len(q), 0.0)])
    prob.set_queries(q)
    for cell_points in (1, 4, 16, 64):
        gp.gp_set_nn_params(prob.ctx, 8, 1, 1, 0, 1, cell_points)
        level = gp.gp_get_nn_grid(prob.ctx, 0)[1]
        log("case: lattice on search-cell faces, level %d" % level)
        prob.nn.fill_(-7)
        prob.nearest()
        prob.sync()
        got = prob.nn[: len(q)].cpu().numpy()
        bad = np.nonzero(got != ref)[0]
        assert len(bad) == 0, "level %d: %d differ" % (level, len(bad))
    prob.close()


@pytest.mark.parametrize("layout", [1, 2])
def test_tv_layouts(layout):
    """Both thread layouts of the TV kernels (block per brick, wave per brick)
    give the oracle's loss terms and gradient, through the separate and the
    fused calls: the sphere with a wide TV band (many brick faces inside the
    band) and the anisotropic grid with random values (bricks cut by the grid
    boundary, neighbours outside the grid)."""
    from paper_2308_13175_amd import gridpull as gp

    dom, pts, q, D = _sphere_case()
    rng = np.random.default_rng(5)
    adom = synth.Domain((24, 17, 31), (-1.125, -0.625, -0.875), (0.875, 0.8125, 1.0625))
    apts = (synth.sphere_points(3000, 0.45, seed=3) + np.float32(0.05)).astype(np.float32)
    aq = synth.host_queries(apts, 9000, 0.05, seed=7)
    aD = rng.normal(size=adom.n_vertices).astype(np.float32) * 0.2
    for name, (dm, p_, q_, D_, m1, m2) in [("sphere m2=14", (dom, pts, q, D, 3, 14)),
                                           ("anisotropic", (adom, apts, aq, aD, 2, 3))]:
        log("case: TV layout %d, %s" % (layout, name))
        prob = make_problem([spec(p_, dm, len(q_), 0.0)], m1=m1, m2=m2)
        gp.gp_set_tv_layout(prob.ctx, layout)
        big = 2 ** 63 - 1
        assert gp.gp_get_grad_params(prob.ctx)[2:] == ((big, big) if layout == 1 else (0, 0))
        prob.set_dense_field([D_])
        prob.set_queries(q_)
        prob.nearest()
        cf, vf, nn, ref = _oracle(dm, p_, q_, D_, m1, m2)
        prob.forward()
        prob.grad.zero_()
        prob.backward()
        prob.sync()
        got, nv = loss_terms(prob)
        assert int(nv[0]) == ref["n_valid"]
        assert_terms_close(got[0], ref)
        assert_grad_close(prob.dense_grad()[0], ref["dD"])
        for rep in range(2):
            prob.grad.zero_()
            prob.forward_backward()
            prob.sync()
            got, nv = loss_terms(prob)
            assert_terms_close(got[0], ref)
            assert_grad_close(prob.dense_grad()[0], ref["dD"])
        with pytest.raises(gp.GridPullError) as ei:
            gp.gp_set_tv_layout(prob.ctx, 3)
        assert ei.value.status == 1
        gp.gp_set_tv_layout(prob.ctx, 0)
        assert gp.gp_get_grad_params(prob.ctx)[2:] == (2048, 16384)
        prob.close()


@pytest.mark.parametrize("method", [0, 1], ids=["marching cubes", "marching tetrahedra"])
def test_surface_extraction(method):
    """The zero-level-set mesh over the optimised cells equals the oracle's,
    by marching cubes (the paper's mesh step) and by marching tetrahedra:
    the same triangle keys (cell and the triangle's number in it) and the
    same corner coordinates (both computed in double with the same
    operations, rounded to float), on the noisy sphere and on a random field
    over an anisotropic grid (many sign changes and ambiguous faces, cells
    cut by the band's edge)."""
    import ctypes

    from paper_2308_13175_amd import gridpull as gp

    dom, pts, q, D = _sphere_case()
    rng = np.random.default_rng(11)
    adom = synth.Domain((24, 17, 31), (-1.125, -0.625, -0.875), (0.875, 0.8125, 1.0625))
    apts = (synth.sphere_points(3000, 0.45, seed=3) + np.float32(0.05)).astype(np.float32)
    aD = (rng.normal(size=adom.n_vertices) * 0.2).astype(np.float32)
    ref_fn = oracle.marching_cubes if method == 0 else oracle.extract_surface
    for name, (dm, p_, D_, m1, m2) in [("sphere", (dom, pts, D, 3, 3)), ("anisotropic random", (adom, apts, aD, 2, 4))]:
        log("case: surface extraction (method %d), %s" % (method, name))
        prob = make_problem([spec(p_, dm, 0, 0.0)], m1=m1, m2=m2)
        prob.set_dense_field([D_])
        tri, key = gp.gp_extract_surface(prob.ctx, 0, prob.field, method=method)
        tri, key = tri.cpu().numpy(), key.cpu().numpy()
        cf, vf = oracle.build_band(dm.dims, dm.lo, dm.hi, p_, m1, m2)
        rkey, rtri = ref_fn(dm.dims, dm.lo, dm.hi, D_.astype(np.float64), vf)
        assert len(rkey) > 100
        assert np.array_equal(key, rkey), "%d vs %d triangles" % (len(key), len(rkey))
        diff = np.abs(tri.astype(np.float64) - rtri.astype(np.float32).astype(np.float64))
        assert diff.max() == 0.0, "largest corner difference %g" % diff.max()
        # too small an output: the count comes back with GP_ERR_CAPACITY
        n = ctypes.c_int64(0)
        t1 = prob.field.new_empty((1, 3, 3))
        k1 = prob.field.new_empty((1,), dtype=prob.field.dtype).to(dtype=__import__("torch").int64)
        st = gp.load_library().gp_extract_surface(prob.ctx, 0, gp._ptr(prob.field), gp._ptr(t1), gp._ptr(k1), 1,
                                                  ctypes.byref(n), method)
        assert st == gp.GP_ERR_CAPACITY and n.value == len(rkey)
        with pytest.raises(gp.GridPullError) as e:
            gp.gp_extract_surface(prob.ctx, 0, prob.field, method=2)
        assert e.value.status == 1
        prob.close()


@pytest.mark.parametrize("brick", [8, 16])
def test_normal_supervision(brick):
    """gp_pull_normals against the oracle's normal term: the mean per shape
    and weight * its gradient, with the points' true normals on the noisy
    sphere and with random unit normals on a random anisotropic field."""
    import torch

    from paper_2308_13175_amd import gridpull as gp

    dom, pts, q, D = _sphere_case()
    rng = np.random.default_rng(13)
    adom = synth.Domain((24, 17, 31), (-1.125, -0.625, -0.875), (0.875, 0.8125, 1.0625))
    apts = (synth.sphere_points(3000, 0.45, seed=3) + np.float32(0.05)).astype(np.float32)
    aq = synth.host_queries(apts, 9000, 0.05, seed=7)
    aD = (rng.normal(size=adom.n_vertices) * 0.2).astype(np.float32)
    rn = rng.normal(size=(len(apts), 3))
    cases = [("sphere, true normals", dom, pts, q, D, pts / np.linalg.norm(pts, axis=1, keepdims=True)),
             ("anisotropic, random normals", adom, apts, aq, aD, rn / np.linalg.norm(rn, axis=1, keepdims=True))]
    for name, dm, p_, q_, D_, nrm in cases:
        log("case: normal supervision, %s, brick %d" % (name, brick))
        nrm = nrm.astype(np.float32)
        prob = make_problem([spec(p_, dm, len(q_), 0.0)], brick=brick)
        prob.set_dense_field([D_])
        prob.set_queries(q_)
        prob.nearest()
        dev = prob.device
        nx, ny, nz = (torch.from_numpy(np.ascontiguousarray(nrm[:, a])).to(dev) for a in range(3))
        term = torch.zeros(1, dtype=torch.float64, device=dev)
        prob.grad.zero_()
        n = prob.n_queries
        gp.gp_pull_normals(prob.ctx, prob.qx[:n], prob.qy[:n], prob.qz[:n], prob.nn, prob.field, nx, ny, nz,
                           0.7, None, term, prob.grad)
        prob.sync()
        cf, vf = oracle.build_band(dm.dims, dm.lo, dm.hi, p_, 3, 3)
        nn = oracle.nn_bruteforce(q_, p_)
        rterm, rgrad, nv = oracle.normal_term(dm.dims, dm.lo, dm.hi, cf, D_.astype(np.float64), q_, nn, p_, nrm,
                                              weight=0.7)
        got = float(term.cpu().numpy()[0])
        assert abs(got - rterm) <= 1e-5 * abs(rterm), (got, rterm)
        assert_grad_close(prob.dense_grad()[0], rgrad)
        prob.close()


def test_nearest_points_not_from_the_search():
    """The loss passes read a query's nearest point from the search's record
    when the record names the same point, else from the caller's points in
    their original order.  Nearest indices given by the caller, before any
    search and after one (half of them changed), give the oracle's loss and
    gradient for those indices (Eq. 4, 6, 7 use s = the given point)."""
    import torch

    log("case: caller-given nearest points")
    dom = synth.cube_domain(32)
    pts = synth.sphere_points(3000, 0.5, seed=41)
    q = synth.host_queries(pts, 12_000, 0.04, seed=42)
    D = synth.sphere_sdf_field(dom, 0.5, noise=0.01, seed=43)
    cf, vf = oracle.build_band(dom.dims, dom.lo, dom.hi, pts, 3, 3)
    prob = make_problem([spec(pts, dom, len(q), 0.0)])
    prob.set_dense_field([D])
    prob.set_queries(q)
    rng = np.random.default_rng(44)
    true_nn = oracle.nn_bruteforce(q, pts)
    given = {"before any search": rng.integers(0, len(pts), len(q)).astype(np.int32),
             "after a search": np.where(rng.random(len(q)) < 0.5, true_nn, (true_nn + 1) % len(pts)).astype(np.int32)}
    for case, nn in given.items():
        log("  " + case)
        if case == "after a search":
            prob.nearest()
            assert np.array_equal(prob.nn[: len(q)].cpu().numpy(), true_nn)
        prob.nn[: len(q)].copy_(torch.from_numpy(nn).to(prob.nn.device))
        ref = oracle.loss_grad(dom.dims, dom.lo, dom.hi, cf, vf, D.astype(np.float64), q, nn, pts)
        prob.forward()
        prob.grad.zero_()
        prob.backward()
        prob.sync()
        got, nv = loss_terms(prob)
        assert int(nv[0]) == ref["n_valid"]
        assert_terms_close(got[0], ref)
        assert_grad_close(prob.dense_grad()[0], ref["dD"])
        prob.grad.zero_()
        prob.forward_backward()
        prob.sync()
        got, nv = loss_terms(prob)
        assert_terms_close(got[0], ref)
        assert_grad_close(prob.dense_grad()[0], ref["dD"])
    prob.close()
