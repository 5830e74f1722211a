#!/usr/bin/env python
"""Throughput of the GridPull pull step on one MI355X.

The metric is pulled queries per second of the forward + backward pass (the
pull, surface, gradient-consistency and TV terms of Eq. 4-8, their
hand-written adjoint scattered into the grid, and the per-shape loss
reduction), with the queries and their nearest surface points already
resident in HBM: one step = one gp_pull_forward_backward over the whole batch
of synthetic queries.  value = queries x steps / the timed region's wall
time.  The roofline is that of the dominant kernel of the step (the fused
query pass, k_query_grad), on its algorithmic bytes per launch: 16 B per query
(q and its nearest-point index), 12 B per distinct nearest point, 12 B per
optimised vertex (field read, gradient read and written), timed with HIP
events on the library's stream during the timed region.

Beside it, the whole optimisation iteration (query sampling, nearest points,
forward + backward, Adam), replayed as one captured hipGraph per iteration;
per-kernel event times of that iteration; on the default workload, the 64
uneven shapes of the batched workload in one launch sequence against one
context per shape, at equal accuracy; and cpu_baseline, the FP64 oracle on one
host thread on a bounded sample of the same workload, in the same unit.
The band and the point buckets are built once before timing (setup_ms).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "pulled queries/sec (fwd+bwd) & % HBM peak; batched vs per-shape at 1e-5 rel err"
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3        # MI355X vector FP32 (published)
NN_FLOPS_PER_PAIR = 8           # dx, dy, dz; three squares; two adds
WORKLOAD_KEYS = {1: "sphere10k", 2: "torus200k", 3: "union24", 4: "batched64", 5: "room20m"}
PROFILES = os.path.join(ROOT, "profiles")
KERNEL_SOURCES = {"k_nn": "nn.hip", "k_forward_query": "pull.hip", "k_backward_query": "pull.hip",
                  "k_query_grad": "pull.hip",
                  "k_tv_forward": "pull.hip", "k_tv_backward": "pull.hip", "k_adam": "step.hip",
                  "k_sample": "sample.hip"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_bytes(name, Q, J, V, V2, n_slots, per_point_sigma):
    """Algorithmic bytes per launch of each kernel (the model in the design notes)."""
    mqj = min(Q, J)
    return {
        "k_sample": 12 * Q + 16 * mqj + (4 * mqj if per_point_sigma else 0),
        "k_nn": 16 * Q + 16 * J,
        "k_forward_query": 16 * Q + 12 * mqj + 4 * V,
        "k_backward_query": 16 * Q + 12 * mqj + 12 * V,
        "k_query_grad": 16 * Q + 12 * mqj + 12 * V,
        "k_tv_forward": 8 * V2,
        "k_tv_backward": 16 * V2,
        "k_adam": 28 * V + 4 * n_slots,
    }.get(name)


def nn_required_pairs(points, dom, queries, n_sample=10000, seed=0, max_reach=12):
    """Mean number of (query, point) pairs an exact cell-bucket search must test.

    For a query at exact nearest distance d, every point in a grid cell whose
    box comes within d of the query can be the nearest point (or tie with it),
    so any exact search over the cell buckets has to test it.  Counted on a
    random sample of the queries with a host k-d tree for d.
    """
    import numpy as np
    from scipy.spatial import cKDTree

    R = np.asarray(dom.dims, np.int64)
    lo = np.asarray(dom.lo, np.float64)
    hi = np.asarray(dom.hi, np.float64)
    h = (hi - lo) / R
    inv_h = R / (hi - lo)
    P = np.asarray(points, np.float64)
    pc = np.clip(np.floor((P - lo) * inv_h), 0, R - 1).astype(np.int64)
    ids, counts = np.unique((pc[:, 0] * R[1] + pc[:, 1]) * R[2] + pc[:, 2], return_counts=True)
    rng = np.random.default_rng(seed)
    sel = rng.choice(len(queries), min(n_sample, len(queries)), replace=False)
    Q = np.asarray(queries, np.float64)[sel]
    d, _ = cKDTree(P).query(Q)
    qc = np.clip(np.floor((Q - lo) * inv_h), 0, R - 1).astype(np.int64)
    reach = np.minimum(np.ceil(d[:, None] * inv_h[None, :] + 1).astype(np.int64).max(1), max_reach)
    total = np.zeros(len(Q))
    for M in np.unique(reach):
        m = reach == M
        q, c0, d2 = Q[m], qc[m], d[m] ** 2
        for ox in range(-M, M + 1):
            for oy in range(-M, M + 1):
                for oz in range(-M, M + 1):
                    c = c0 + np.array([ox, oy, oz])
                    ok = np.all((c >= 0) & (c < R), axis=1)
                    blo = lo + c * h
                    g = np.maximum(np.maximum(blo - q, q - (blo + h)), 0.0)
                    ok &= (g * g).sum(1) <= d2
                    cid = (c[ok, 0] * R[1] + c[ok, 1]) * R[2] + c[ok, 2]
                    k = np.minimum(np.searchsorted(ids, cid), len(ids) - 1)
                    hit = ids[k] == cid
                    t = np.zeros(len(cid))
                    t[hit] = counts[k[hit]]
                    total[np.nonzero(m)[0][ok]] += t
    return float(total.mean()), len(Q)


def _source_sha(kernel):
    """sha256 of the kernel's source file followed by the header every kernel
    inlines (gp_internal.h): a change to either changes the kernel."""
    import hashlib

    src = KERNEL_SOURCES.get(kernel)
    if src is None:
        return None
    h = hashlib.sha256()
    for name in (src, "gp_internal.h"):
        with open(os.path.join(ROOT, "paper_2308_13175_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(kernel, config):
    """HBM bytes per launch from the committed counter summary, or None.

    The summary records the sha256 of the kernel's sources (its file and the
    shared header) when the counters were taken; a kernel changed since then
    gets None.
    """
    path = os.path.join(PROFILES, "%s_%s_traffic.txt" % (kernel, WORKLOAD_KEYS.get(config, "")))
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_sha256") != _source_sha(kernel):
        return None
    try:
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def copy_bandwidth(mib=1024, reps=10):
    """Measured device-to-device copy rate (read + write bytes per second)."""
    import torch

    a = torch.empty(mib << 18, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    gbps = 2.0 * (mib << 20) * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    return gbps


def fwd_bwd_median_ms(prob, n=50):
    """Median duration of one fused forward + backward (query pass, TV, loss) by events."""
    import torch

    times = []
    for _ in range(n):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        prob.forward_backward()
        e1.record()
        times.append((e0, e1))
    torch.cuda.synchronize()
    ms = sorted(a.elapsed_time(b) for a, b in times)
    prob.grad.zero_()
    return ms[len(ms) // 2]


def copy_calibration(mib=256, reps=3):
    """A plain device copy of known size, for scaling the HBM counters."""
    import torch

    a = torch.empty(mib << 18, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    log("copy calibration: %d x %d MiB device copy" % (reps, mib))


def batched_vs_per_shape(wl, prob, steps, warmup, autotune=True):
    """The 64-shape batch: one batched launch sequence against one context per shape.

    Times the metric's step (forward + backward on resident queries and
    nearest points) and the whole iteration (as captured graphs) both ways,
    then puts both in the same state (geometric initial field, the batched
    queries) and compares nearest neighbours, loss terms and gradients.
    """
    import numpy as np
    import torch

    from paper_2308_13175_amd import gridpull as gp
    from paper_2308_13175_amd.problem import GraphedIteration, Problem, spec_from_synth

    singles = [Problem([spec_from_synth(sh)], m1=wl.m1, m2=wl.m2, adam=prob.adam) for sh in wl.shapes]
    for p in singles:
        p.init_sphere()
    torch.cuda.synchronize()
    for _ in range(warmup):
        for p in singles:
            p.iteration(None)
    if autotune:
        for p in singles:
            p.autotune(reps=1)
    for p in singles:
        p.iteration(None)
    # the metric's step, both ways (each side on its own resident queries)
    def time_fb(probs):
        for _ in range(warmup):
            for p in probs:
                p.forward_backward()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            for p in probs:
                p.forward_backward()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    fb_single_s = time_fb(singles)
    fb_batch_s = time_fb([prob])
    # whole iterations as captured graphs, both ways
    def time_graphs(probs):
        graphs = [GraphedIteration(p) for p in probs]
        for _ in range(warmup):
            for g in graphs:
                g.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            for g in graphs:
                g.replay()
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / steps
        del graphs
        return el

    it_single_s = time_graphs(singles)
    it_batch_s = time_graphs([prob])

    # same state both ways: initial field, the batched problem's queries
    prob.init_sphere()
    for p in singles:
        p.init_sphere()
    prob.sample(7, 1)
    prob.nearest()
    prob.grad.zero_()
    prob.forward()
    prob.backward()
    sizes = [int(np.prod(np.asarray(sp.dims, np.int64) + 1)) for sp in prob.specs]
    dense_b = torch.zeros(sum(sizes), dtype=torch.float32, device=prob.device)
    gp.gp_scatter_vertices(prob.ctx, prob.grad, dense_b)
    loss_b = prob.loss.cpu().numpy()
    nn_equal = True
    worst_loss, worst_grad = 0.0, 0.0
    off = doff = 0
    for i, p in enumerate(singles):
        n = p.n_queries
        p.qx[:n].copy_(prob.qx[off:off + n])
        p.qy[:n].copy_(prob.qy[off:off + n])
        p.qz[:n].copy_(prob.qz[off:off + n])
        p.nearest()
        p.grad.zero_()
        p.forward()
        p.backward()
        nn_equal = nn_equal and bool(torch.equal(p.nn[:n], prob.nn[off:off + n]))
        l1 = p.loss.cpu().numpy()[0]
        l0 = loss_b[i]
        worst_loss = max(worst_loss, float(np.max(np.abs(l1 - l0) / np.maximum(np.abs(l0), 1e-300))))
        dense_s = torch.zeros(sizes[i], dtype=torch.float32, device=prob.device)
        gp.gp_scatter_vertices(p.ctx, p.grad, dense_s)
        ref = dense_b[doff:doff + sizes[i]]
        gmax = float(ref.abs().max())
        if gmax > 0:
            worst_grad = max(worst_grad, float((dense_s - ref).abs().max()) / gmax)
        off += n
        doff += sizes[i]
        p.close()
    Q = prob.n_queries
    return {"workload": wl.name, "shapes": len(singles), "queries_per_step": Q,
            "fwd_bwd": {"batched_queries_per_s": Q / fb_batch_s, "per_shape_queries_per_s": Q / fb_single_s,
                        "batched_ms": fb_batch_s * 1e3, "per_shape_ms": fb_single_s * 1e3,
                        "speedup": fb_single_s / fb_batch_s},
            "iteration_graph": {"batched_queries_per_s": Q / it_batch_s, "per_shape_queries_per_s": Q / it_single_s,
                                "batched_ms": it_batch_s * 1e3, "per_shape_ms": it_single_s * 1e3,
                                "speedup": it_single_s / it_batch_s},
            "nn_identical": nn_equal, "max_rel_err_loss_terms": worst_loss, "max_rel_err_grad": worst_grad}


def batched_record(args):
    """Build the 64-shape batched workload and compare it against per-shape contexts."""
    import torch

    from paper_2308_13175_amd import gridpull as gp
    from paper_2308_13175_amd import tuning

    wl, prob, setup_ms = build_problem(4)
    for _ in range(args.warmup):
        prob.iteration(None)
    if not args.no_autotune:
        tuning.tune_nn(prob)
    prob.iteration(None)
    rec = batched_vs_per_shape(wl, prob, max(3, args.steps // 5), 2, not args.no_autotune)
    rec["setup_ms"] = setup_ms
    rec["nn_search_shape"] = list(gp.gp_get_nn_params(prob.ctx))
    prob.close()
    del prob
    torch.cuda.empty_cache()
    return rec


def make_workload(config: int):
    """The synthetic workload of a configuration, its shape specifications and Adam settings."""
    from paper_2308_13175_amd import synth
    from paper_2308_13175_amd.problem import AdamConfig, spec_from_synth

    t0 = time.perf_counter()
    wl = synth.WORKLOADS[config]()
    log("inputs: %s, %d points, %d queries/step (%.1f s)" % (wl.name, wl.n_points, wl.n_queries,
                                                              time.perf_counter() - t0))
    adam = AdamConfig(lr0=wl.lr0(), eps=1e-8 * (5e4 / max(wl.n_queries, 1)))
    return wl, [spec_from_synth(s) for s in wl.shapes], adam


def build_problem(config: int, brick: int = 8, made=None):
    """The configuration's problem with bricks of the given edge (made: the
    result of make_workload, to build from the same inputs again)."""
    from paper_2308_13175_amd import synth
    from paper_2308_13175_amd.problem import Problem

    wl, specs, adam = made if made is not None else make_workload(config)
    import torch

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    prob = Problem(specs, m1=wl.m1, m2=wl.m2, adam=adam, brick=brick)
    torch.cuda.synchronize()
    setup_ms = (time.perf_counter() - t0) * 1e3
    if config == 1:
        s = wl.shapes[0]
        prob.set_dense_field([synth.sphere_sdf_field(s.domain, 0.5, noise=0.01, seed=0)])
    else:
        prob.init_sphere()
    return wl, prob, setup_ms


def schedule_sweep(kind: str, iters: int = 1600, n_points: int = 200_000, n_queries: int = 50_000):
    """Whole optimisation runs on the paper's default schedule, one JSON line per setting.

    Sec. 4's defaults: 50 000 queries per iteration, 1600 iterations, Adam with
    lr 1.0 (the domain is [-1, 1]^3) times 0.3 every 400 iterations, a small-sphere initial
    field, M1 = 3 and M2 = 14.  One quantity varies per sweep, as in the
    ablations: the grid resolution R (Tab. 14), the TV band M2 (Tab. 17) or
    the pull band M1 (3 against all cells).  Input: the 200K-point torus,
    sigma = 2 cells.  Iteration 1 runs eagerly with t = 1, the other
    iterations replay one captured graph.
    """
    import torch

    from paper_2308_13175_amd import gridpull as gp
    from paper_2308_13175_amd import tuning
    from paper_2308_13175_amd import synth
    from paper_2308_13175_amd.problem import AdamConfig, GraphedIteration, Problem, ShapeSpec

    pts = synth.torus_points(n_points, seed=1)
    if kind == "res":
        settings = [(r, 3, 14) for r in (32, 64, 128, 256, 512)]
    elif kind == "m2":
        settings = [(256, 3, m2) for m2 in (2, 14, 30, 50, 256)]
    elif kind == "m1":
        settings = [(256, m1, 14) for m1 in (3, 256)]
    else:
        raise SystemExit("unknown sweep %r (res, m2, m1)" % kind)
    for res, m1, m2 in settings:
        dom = synth.cube_domain(res)
        h = dom.h[0]
        spec = ShapeSpec(pts, dom.dims, dom.lo, dom.hi, n_queries, 2.0 * h)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        prob = Problem([spec], m1=m1, m2=m2, adam=AdamConfig(lr0=1.0, eps=1e-8))
        torch.cuda.synchronize()
        setup_s = time.perf_counter() - t0
        prob.iteration(1)
        tuning.tune_nn(prob)   # before the capture: the graph keeps the search shape
        nn_search = gp.gp_get_nn_params(prob.ctx)
        graph = GraphedIteration(prob)
        prob.init_sphere()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        prob.iteration(1)
        for _ in range(iters - 1):
            graph.replay()
        torch.cuda.synchronize()
        run_s = time.perf_counter() - t0
        prob.sync()
        loss = prob.loss.cpu().numpy()[0]
        # per-kernel event times over a few extra eager iterations
        gp.gp_timing_enable(prob.ctx, True)
        gp.gp_timing_report(prob.ctx)
        for _ in range(10):
            prob.iteration(None)
        torch.cuda.synchronize()
        kern = gp.gp_timing_report(prob.ctx)
        gp.gp_timing_enable(prob.ctx, False)
        _, flags = prob.layout()
        print(json.dumps({
            "sweep": kind, "workload": "torus-200k", "res": res, "m1": m1, "m2": m2, "iterations": iters,
            "queries_per_iteration": n_queries, "run_s": run_s, "ms_per_iteration": run_s * 1e3 / iters,
            "setup_s": setup_s, "slots": prob.n_slots, "optimised_vertices": prob.n_active,
            "tv_vertices": int(((flags & 2) > 0).sum()), "final_loss": [float(x) for x in loss],
            "final_valid": int(prob.n_valid.sum()), "nn_search": list(nn_search),
            "kernels_avg_ms": {k: round(ms / max(n, 1), 5) for k, (n, ms) in sorted(kern.items())}}), flush=True)
        del graph
        prob.close()
        del prob
        torch.cuda.empty_cache()


def surface_runs(iters: int = 1600, n_queries: int = 50_000):
    """Whole runs on the paper's schedule, then the mesh and its quality.

    Each setting optimises from the small-sphere initial field (M1 = 3,
    M2 = 14, 50 000 queries per iteration, sigma = 2 cells, 1600 iterations
    with lr 1.0 x 0.3 every 400), extracts the zero level set with
    gp_extract_surface (marching cubes; the tetrahedra mesh is measured
    beside it) and measures it against the closed-form surface the
    points were drawn from: CD-L1, normal consistency and F-score at
    tau = 0.005 (the shapes span about 1.3 units).  The same measures of the
    mesh of the closed-form SDF sampled on the same band are reported beside
    them.  One JSON line each.
    """
    import numpy as np
    import torch

    from paper_2308_13175_amd import gridpull as gp
    from paper_2308_13175_amd import tuning
    from paper_2308_13175_amd import metrics, synth
    from paper_2308_13175_amd.problem import AdamConfig, GraphedIteration, Problem, ShapeSpec

    torus = synth.torus_points(200_000, seed=1)
    torus_ref = synth.torus_points(100_000, jitter=0.0, seed=17)
    sphere = synth.sphere_points(10_000, 0.5, seed=0)
    sphere_ref = synth.sphere_points(100_000, 0.5, seed=18)
    # noisy torus: N(0, 0.01^2) on every point, fitted with alpha = 1 and with
    # the paper's alpha = 2 for noisy inputs (Sec. 4, noise paragraph)
    noisy = synth.torus_points(200_000, jitter=0.01, seed=1)
    # with ground-truth normals (the closed form's gradient at each point),
    # supervised with weight 1 (Sec. 4, normals paragraph)
    tsdf = metrics.torus_sdf(0.5, 0.15)
    tnormals = tsdf[1](torus.astype(np.float64))
    settings = [("torus-200k", torus, torus_ref, tsdf, 128, 1.0, None),
                ("torus-200k", torus, torus_ref, tsdf, 256, 1.0, None),
                ("sphere-10k", sphere, sphere_ref, metrics.sphere_sdf(0.5), 64, 1.0, None),
                ("torus-200k-noise0.01", noisy, torus_ref, tsdf, 128, 1.0, None),
                ("torus-200k-noise0.01", noisy, torus_ref, tsdf, 128, 2.0, None),
                ("torus-200k-normals", torus, torus_ref, tsdf, 128, 1.0, tnormals)]
    for name, pts, ref, (sdf, grad), res, alpha, normals in settings:
        dom = synth.cube_domain(res)
        h = dom.h[0]
        prob = Problem([ShapeSpec(pts, dom.dims, dom.lo, dom.hi, n_queries, 2.0 * h)], m1=3, m2=14,
                       weights=(alpha, 1.0, 0.005), adam=AdamConfig(lr0=1.0, eps=1e-8))
        if normals is not None:
            prob.set_normals(normals, 1.0)
        prob.iteration(1)
        tuning.tune_nn(prob)
        graph = GraphedIteration(prob)
        prob.init_sphere()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        prob.iteration(1)
        for _ in range(iters - 1):
            graph.replay()
        torch.cuda.synchronize()
        run_s = time.perf_counter() - t0
        prob.sync()
        # the mesh of the closed-form field on the same band: what extraction
        # and measurement alone give (the field's own interpolation error)
        g = np.asarray(dom.lo)[:, None] + np.arange(res + 1)[None, :] * h
        X, Y, Z = np.meshgrid(g[0], g[1], g[2], indexing="ij")
        dense = sdf(np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1)).astype(np.float32)
        keep = prob.field.clone()
        prob.set_dense_field([dense])
        etri, _ = gp.gp_extract_surface(prob.ctx, 0, prob.field)
        m_exact = metrics.reconstruction_metrics(etri.cpu().numpy(), ref, sdf, grad, tau=0.005)
        prob.field.copy_(keep)
        gp.gp_extract_surface(prob.ctx, 0, prob.field)      # warm
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tri, key = gp.gp_extract_surface(prob.ctx, 0, prob.field)
        torch.cuda.synchronize()
        extract_ms = (time.perf_counter() - t0) * 1e3
        tri = tri.cpu().numpy()
        m = metrics.reconstruction_metrics(tri, ref, sdf, grad, tau=0.005)
        ttri, _ = gp.gp_extract_surface(prob.ctx, 0, prob.field, method=1)
        m_tet = metrics.reconstruction_metrics(ttri.cpu().numpy(), ref, sdf, grad, tau=0.005)
        print(json.dumps({"surface": name, "res": res, "m1": 3, "m2": 14, "alpha": alpha,
                          "normal_weight": 1.0 if normals is not None else 0.0, "iterations": iters,
                          "queries_per_iteration": n_queries, "run_s": run_s, "triangles": int(len(tri)),
                          "extract_ms": extract_ms, **m,
                          "closed_form_field": {"triangles": int(len(etri)),
                                                **{k: m_exact[k] for k in ("cd_l1", "nc", "fscore")}},
                          "marching_tetrahedra": {"triangles": int(len(ttri)),
                                                  **{k: m_tet[k] for k in ("cd_l1", "nc", "fscore")}}}),
              flush=True)
        del graph
        prob.close()
        del prob
        torch.cuda.empty_cache()


def _window(dom, pts, cells: int, centre=None):
    """A sub-grid of cells^3 cells of dom (same cell size and vertex lattice)
    around a point (centre; by default the densest region of the points), and
    the points inside it."""
    import numpy as np

    from paper_2308_13175_amd import synth

    R = np.asarray(dom.dims, np.int64)
    if np.all(R <= cells):
        return dom, pts
    lo = np.asarray(dom.lo, np.float64)
    h = np.asarray(dom.h, np.float64)
    w = np.minimum(R, cells)
    if centre is None:
        c = np.clip(np.floor((pts.astype(np.float64) - lo) / h), 0, R - 1).astype(np.int64)
        # the coarse block (of the window's size) holding the most points
        blk = c // w
        nb = (R + w - 1) // w
        ids, cnt = np.unique((blk[:, 0] * nb[1] + blk[:, 1]) * nb[2] + blk[:, 2], return_counts=True)
        b = ids[np.argmax(cnt)]
        b3 = np.array([b // (nb[1] * nb[2]), (b // nb[2]) % nb[1], b % nb[2]])
        c0 = np.minimum(b3 * w, R - w)
    else:
        cc = np.clip(np.floor((np.asarray(centre, np.float64) - lo) / h), 0, R - 1).astype(np.int64)
        c0 = np.clip(cc - w // 2, 0, R - w)
    wlo = lo + c0 * h
    whi = lo + (c0 + w) * h
    sub = synth.Domain(tuple(int(x) for x in w), tuple(float(x) for x in wlo), tuple(float(x) for x in whi))
    # in the window's own cell units, with a margin against rounding at its faces
    u = (pts.astype(np.float64) - wlo) / ((whi - wlo) / w)
    inside = np.all((u >= 1e-7) & (u <= w - 1e-7), axis=1)
    return sub, pts[inside]


def cpu_baseline(wl, v2_total: int, n_windows: int = 8, window_cells: int = 160, max_queries: int = 1_000_000):
    """The FP64 oracle on one host thread, on a bounded sample of the workload,
    in the metric's unit (forward + backward queries/s).

    Shape 0 of the workload, cut (when its grid is larger) to n_windows windows
    of window_cells^3 cells (same cell size): one around its densest points,
    the others around points drawn at random (seeded).  In each window the
    oracle's loss and gradient are timed on the window's share of the
    workload's queries (at most max_queries), and its query-independent part
    (TV over the window's band, gradient clear) once.  The per-query time
    (all windows' queries together) is scaled to the workload's queries per
    step, and the query-independent time to its v2_total TV vertices (counted
    on the library's band, which equals the oracle's).  Brute-force nearest
    points and Adam are timed too and reported beside it.
    """
    import numpy as np

    import oracle
    from paper_2308_13175_amd import synth

    s = wl.shapes[0]
    Q = wl.n_queries
    sigma = s.sigma if np.ndim(s.sigma) == 0 else float(np.median(s.sigma))
    whole = bool(np.all(np.asarray(s.domain.dims) <= window_cells))
    rng = np.random.default_rng(7)
    centres = [None] if whole else [None] + [s.points[i] for i in
                                             rng.choice(len(s.points), n_windows - 1, replace=False)]
    t_q_sum = t_fixed_sum = t_band_sum = 0.0
    n_q_sum = v2_sum = n_pts_sum = 0
    for wi, centre in enumerate(centres):
        sub, pts = _window(s.domain, s.points, window_cells, centre)
        n_q = max(1000, int(min(s.n_queries * len(pts) / max(len(s.points), 1), max_queries)))
        q = synth.host_queries(pts, n_q, sigma, seed=99 + wi)
        t0 = time.perf_counter()
        cf, vf = oracle.build_band(sub.dims, sub.lo, sub.hi, pts, wl.m1, wl.m2)
        t_band_sum += time.perf_counter() - t0
        # small-sphere initial field at the full domain's centre (its cost is what matters)
        dom = s.domain
        ctr = [0.5 * (dom.lo[a] + dom.hi[a]) for a in range(3)]
        vx, vy, vz = sub.vdims
        xs = sub.lo[0] + np.arange(vx) * sub.h[0] - ctr[0]
        ys = sub.lo[1] + np.arange(vy) * sub.h[1] - ctr[1]
        zs = sub.lo[2] + np.arange(vz) * sub.h[2] - ctr[2]
        D = (np.sqrt(xs[:, None, None] ** 2 + ys[None, :, None] ** 2 + zs[None, None, :] ** 2)
             - 2 * min(sub.h)).reshape(-1)
        # the query-independent part: no queries
        empty = np.zeros((0, 3), np.float32)
        t0 = time.perf_counter()
        oracle.loss_grad(sub.dims, sub.lo, sub.hi, cf, vf, D, empty, np.zeros(0, np.int32), pts)
        t_fixed = time.perf_counter() - t0
        nn_l = oracle.nn_exact(q, pts)
        t0 = time.perf_counter()
        oracle.loss_grad(sub.dims, sub.lo, sub.hi, cf, vf, D, q, nn_l, pts)
        t_q_sum += max(time.perf_counter() - t0 - t_fixed, 0.0)
        t_fixed_sum += t_fixed
        n_q_sum += n_q
        v2_sum += int(np.count_nonzero(vf & 2))
        n_pts_sum += len(pts)
    t_q = t_q_sum / max(n_q_sum, 1)
    t_fb = Q * t_q + t_fixed_sum * (v2_total / max(v2_sum, 1))
    # nearest points by brute force over all of shape 0's points, a few queries
    full_q = synth.host_queries(s.points, 64, s.sigma if np.ndim(s.sigma) == 0 else float(np.median(s.sigma)),
                                seed=98)
    k = 4
    t0 = time.perf_counter()
    oracle.nn_bruteforce(full_q[:k], s.points)
    t_nn = (time.perf_counter() - t0) / k
    G = np.zeros(len(D))
    m = np.zeros(len(D))
    v = np.zeros(len(D))
    t0 = time.perf_counter()
    oracle.adam(D, G, m, v, vf, 1, 0.01)
    t_adam = time.perf_counter() - t0
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {
        "value": Q / t_fb if t_fb > 0 else 0.0,
        "unit": "queries/s",
        "cores": 1,
        "host_cpu": model,
        "host_threads": os.cpu_count(),
        "kind": "oracle",
        "sample": ("FP64 oracle, 1 thread, shape 0 of %s in %d window(s) of %s cells (one around the densest "
                   "points, the others around random points; %d points in all, bands built in %.1f s): loss and "
                   "gradient on %d queries (%.3g s/query) plus the query-independent TV and gradient clear over "
                   "the windows' %d TV vertices (%.3g s), scaled to %d queries per step and %.3g TV vertices"
                   % (wl.name, len(centres), "x".join(str(x) for x in sub.dims), n_pts_sum, t_band_sum, n_q_sum,
                      t_q, v2_sum, t_fixed_sum, Q, float(v2_total))),
        "nn_bruteforce_s_per_query": t_nn,
        "nn_bruteforce_points": len(s.points),
        "adam_s_per_vertex": t_adam / max(len(D), 1),
    }


def timed_fwd_bwd(prob, steps: int):
    """steps fused forward + backward passes on the resident queries and
    nearest points, bracketed by device synchronisations; per-kernel HIP
    events (on the library's stream) over the same region.  Returns (wall
    seconds, {kernel: (launches, total ms)})."""
    import torch

    from paper_2308_13175_amd import gridpull as gp

    gp.gp_timing_enable(prob.ctx, True)
    gp.gp_timing_report(prob.ctx)          # a clean period
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        prob.forward_backward()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kern = gp.gp_timing_report(prob.ctx)
    gp.gp_timing_enable(prob.ctx, False)
    return elapsed, kern


def iteration_rate(prob, steps: int, warmup: int, graph: bool = True):
    """Whole iterations (sample, NN, forward + backward, Adam): as captured
    graph replays (or eager launches), then eager with per-kernel events."""
    import torch

    from paper_2308_13175_amd import gridpull as gp
    from paper_2308_13175_amd.problem import GraphedIteration

    out = {}
    if graph:
        g = GraphedIteration(prob)
        for _ in range(warmup):
            g.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            g.replay()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        prob.sync()
        del g
        out["graph"] = {"queries_per_s": prob.n_queries * steps / el, "ms_per_step": el * 1e3 / steps}
    gp.gp_timing_enable(prob.ctx, True)
    gp.gp_timing_report(prob.ctx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        prob.iteration(None)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    kern = gp.gp_timing_report(prob.ctx)
    gp.gp_timing_enable(prob.ctx, False)
    out["eager"] = {"queries_per_s": prob.n_queries * steps / el, "ms_per_step": el * 1e3 / steps}
    out["kernels_avg_ms"] = {k: round(ms / max(n, 1), 5) for k, (n, ms) in sorted(kern.items())}
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", type=int, default=5, choices=[1, 2, 3, 4, 5],
                    help="workload: 1 sphere-10k, 2 torus-200k, 3 union24-2M, 4 batched64, 5 room-20M (default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched-vs-per-shape record (configs 4 and 5)")
    ap.add_argument("--sweep", choices=["res", "m2", "m1"],
                    help="instead of the benchmark: whole runs on the paper's schedule, one JSON line per setting")
    ap.add_argument("--surface", action="store_true",
                    help="instead of the benchmark: whole runs, then the extracted mesh against the closed-form "
                         "surface (CD, NC, F-score), one JSON line per shape and grid")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default search and gradient-pass settings instead of tuning them first")
    ap.add_argument("--tuning-cache", default=None,
                    help="JSON cache of tuned settings per GPU architecture and size class (default: "
                         "~/.cache/gridpull/tuning.json); 'none' always tunes afresh and stores nothing")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 256 MiB device copy (scale for the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (--gpus %d requested)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2308_13175_amd import gridpull as gp
    from paper_2308_13175_amd import tuning

    torch.cuda.set_device(0)
    if args.sweep:
        schedule_sweep(args.sweep)
        return
    if args.surface:
        surface_runs()
        return
    made = make_workload(args.config)
    brick_rec = None
    brick = 8
    if not args.no_autotune:
        cache = tuning.DEFAULT_CACHE if args.tuning_cache is None else (
            None if args.tuning_cache == "none" else args.tuning_cache)
        brick_rec = tuning.choose_brick(made[1], made[0].m1, made[0].m2, made[2], cache_path=cache)
        brick = brick_rec["brick"]
        log("brick (%s): %s" % (brick_rec["source"], brick_rec))
    wl, prob, setup_ms = build_problem(args.config, brick, made)
    Q, J = prob.n_queries, prob.n_points
    log("band: %d slots, %d optimised vertices, bricks of %d^3, setup %.1f ms" % (prob.n_slots, prob.n_active,
                                                                                  brick, setup_ms))

    for _ in range(args.warmup):
        prob.iteration(None)
    tuned = None
    if not args.no_autotune:
        tuned = tuning.tune(prob, cache)
        log("tuning (%s, %s): %s" % (tuned["key"], tuned["source"], tuned))
    nn_params = gp.gp_get_nn_params(prob.ctx)
    grad_params = gp.gp_get_grad_params(prob.ctx)
    nn_grids = sorted({gp.gp_get_nn_grid(prob.ctx, s)[1] for s in range(len(wl.shapes))})
    log("NN search shape: %s, search grid levels %s; gradient pass: %s" % (nn_params, nn_grids, grad_params))
    it = iteration_rate(prob, max(5, args.steps // 2), args.warmup, graph=not args.no_graph)
    prob.sync()
    loss = prob.loss.cpu().numpy()
    log("loss: %s, valid %d" % (loss[0].tolist(), int(prob.n_valid.sum())))

    # the metric's step: forward + backward over the resident queries and nearest points
    for _ in range(args.warmup):
        prob.forward_backward()
    elapsed, kern = timed_fwd_bwd(prob, args.steps)
    prob.sync()
    fb_median = fwd_bwd_median_ms(prob)
    copy_gbps = copy_bandwidth()
    _, flags = prob.layout()
    V2 = int(((flags & 2) > 0).sum())
    V = prob.n_active
    avg = {k: (n, ms / max(n, 1)) for k, (n, ms) in kern.items()}
    ms_step = elapsed * 1e3 / args.steps
    fb_bytes = 16 * Q + 12 * min(Q, J) + 12 * V
    dom_k = "k_query_grad"
    by = kernel_bytes(dom_k, Q, J, V, V2, prob.n_slots, prob.sigma is not None)
    ach = by / (avg[dom_k][1] * 1e-3) / 1e9
    roof = {"bound": "hbm", "kernel": dom_k, "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": ach / HBM_PEAK_GBS, "traffic": measured_traffic(dom_k, args.config),
            "bytes_per_launch": by, "bytes_model": "16 Q + 12 min(Q, J) + 12 V",
            "avg_launch_ms": avg[dom_k][1]}
    kernels_hbm = {}
    for k in avg:
        b = kernel_bytes(k, Q, J, V, V2, prob.n_slots, prob.sigma is not None)
        if b is not None:
            kernels_hbm[k] = {"bytes": b, "GBps": b / (avg[k][1] * 1e-3) / 1e9,
                              "frac": b / (avg[k][1] * 1e-3) / 1e9 / HBM_PEAK_GBS}
    nn_ms = it["kernels_avg_ms"].get("k_nn")
    value = Q * args.steps / elapsed
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "shapes": len(wl.shapes), "points": J, "queries_per_step": Q, "brick": brick,
                   "grid": [list(s.domain.dims) for s in wl.shapes][:4], "m1": wl.m1, "m2": wl.m2,
                   "slots": prob.n_slots, "optimised_vertices": V, "tv_vertices": V2,
                   "step": "forward+backward (gp_pull_forward_backward) on resident queries and nearest points"},
        "roofline": roof,
        "fwd_bwd": {"queries_per_s": value, "ms": ms_step, "median_ms": fb_median,
                    "kernels_ms": {k: round(v[1], 5) for k, v in sorted(avg.items())},
                    "algorithmic_bytes": fb_bytes,
                    "algorithmic_GBps": fb_bytes / (ms_step * 1e-3) / 1e9,
                    "hbm_frac": fb_bytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS,
                    "copy_frac": fb_bytes / (ms_step * 1e-3) / 1e9 / copy_gbps},
        "iteration": {"step": "sample+nn+forward+backward+adam", **it},
        "nn": {"queries_per_s": Q / (nn_ms * 1e-3) if nn_ms else None, "ms": nn_ms,
               "search_shape": list(nn_params), "search_grid_levels": nn_grids},
        "tuning": {"brick": brick, "brick_source": brick_rec["source"] if brick_rec else "default",
                   "brick_ms": brick_rec.get("brick_ms") if brick_rec else None,
                   "nn": list(nn_params), "grad": list(grad_params),
                   "key": tuned["key"] if tuned else None, "source": tuned["source"] if tuned else "defaults",
                   "nn_ms": tuned.get("nn_ms") if tuned else None,
                   "grad_ms": tuned.get("grad_ms") if tuned else None},
        "copy_GBps": copy_gbps,
        "kernels_hbm": kernels_hbm,
        "setup_ms": setup_ms,
    }
    prob.close()
    del prob
    torch.cuda.empty_cache()
    if args.config in (4, 5) and not args.no_batched:
        out["batched_vs_per_shape"] = batched_record(args)
    if not args.no_cpu_baseline:
        t0 = time.perf_counter()
        out["cpu_baseline"] = cpu_baseline(wl, V2)
        log("cpu baseline took %.1f s" % (time.perf_counter() - t0))
    if args.copy_calibration:
        copy_calibration()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
