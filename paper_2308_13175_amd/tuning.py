"""Autotuning of a problem's launch settings, with a persistent cache.

Three groups of settings change only the speed, never the result:
- the band's brick size (4, 8 or 16 vertices per edge; it fixes the field
  layout, so it is chosen before the problem is built: `choose_brick` builds
  the problem with each size and times its forward + backward);
- the nearest-neighbour search grid and search shape (gp_autotune_nn);
- the gradient pass's LDS rows and slab limit, and the TV kernels' layouts
  (gp_autotune_grad).

`tune` times the last two on the problem's own inputs: the search on the
query samples of a few iterations (the sample moves the best shape, so each
shape the tuner picks on one sample is timed on all of them and the best mean
kept), then the gradient pass on the last sample.  The choices are stored in
a JSON file under a key made of the GPU architecture and the problem's size
class (queries per iteration and points, each rounded to a power of two, and
whether it is a batch), and a later problem of the same class takes them from
there without timing anything.
"""
from __future__ import annotations

import json
import math
import os
import tempfile
from typing import Dict, Optional

from . import gridpull as gp

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "gridpull", "tuning.json")


def size_class(n_queries: int, n_points: int, n_shapes: int) -> str:
    """Queries per iteration and points as the nearest powers of two, and single or batch
    (all known before the band is built, and the same for every brick size)."""
    q = int(round(math.log2(max(int(n_queries), 1))))
    p = int(round(math.log2(max(int(n_points), 1))))
    return "q2^%d-p2^%d-%s" % (q, p, "batch" if n_shapes > 1 else "single")


def class_key(specs, device: int = 0) -> str:
    """The cache key of a batch of shape specifications."""
    nq = sum(int(s.n_queries) for s in specs)
    npts = sum(len(s.points) for s in specs)
    return "%s|%s" % (arch_name(device), size_class(nq, npts, len(specs)))


def arch_name(device: int = 0) -> str:
    import torch

    name = getattr(torch.cuda.get_device_properties(device), "gcnArchName", "") or "unknown"
    return name.split(":")[0]


def load_cache(path: str) -> Dict[str, dict]:
    """The cache's entries ({} if the file does not exist)."""
    try:
        with open(path) as f:
            data = json.load(f)
    except FileNotFoundError:
        return {}
    if not isinstance(data, dict):
        raise ValueError("%s: not a tuning cache" % path)
    return data


def save_cache(path: str, data: Dict[str, dict]) -> None:
    """Write the cache atomically (a temporary file renamed over it)."""
    d = os.path.dirname(os.path.abspath(path))
    os.makedirs(d, exist_ok=True)
    fd, tmp = tempfile.mkstemp(dir=d, prefix=".tuning-")
    try:
        with os.fdopen(fd, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except BaseException:
        if os.path.exists(tmp):
            os.remove(tmp)
        raise


def apply(prob, entry: dict) -> None:
    """Put a cache entry's settings into the problem's context."""
    if "nn" in entry:
        gp.gp_set_nn_params(prob.ctx, *entry["nn"])
    if "grad" in entry:
        gp.gp_set_grad_params(prob.ctx, *entry["grad"])


def _fwd_bwd_ms(prob, reps: int) -> float:
    import torch

    prob.forward_backward()
    torch.cuda.synchronize()
    best = None
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        prob.forward_backward()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    return best


def choose_brick(specs, m1: int, m2: int, adam=None, weights=(1.0, 1.0, 0.005),
                 cache_path: Optional[str] = DEFAULT_CACHE, candidates=(4, 8, 16), reps: int = 5) -> dict:
    """The brick size for this batch: from the cache when its class is there,
    else each candidate's problem is built (small-sphere field, the queries of
    iteration 1 and their nearest points) and its forward + backward timed
    (the smallest of reps); the fastest is stored.  Returns {"key", "brick",
    "source", and when timed "brick_ms": {size: ms}}."""
    import torch

    from .problem import Problem

    key = class_key(specs)
    cache = load_cache(cache_path) if cache_path else {}
    if key in cache and "brick" in cache[key]:
        return {"key": key, "brick": int(cache[key]["brick"]), "source": "cache"}
    times = {}
    for b in candidates:
        prob = Problem(specs, m1=m1, m2=m2, weights=weights, adam=adam, brick=b)
        prob.init_sphere()
        prob.sample(0, 1)
        prob.nearest()
        times[b] = _fwd_bwd_ms(prob, reps)
        prob.close()
        del prob
        torch.cuda.empty_cache()
    best = min(times, key=times.get)
    if cache_path:
        cache = load_cache(cache_path)
        cache.setdefault(key, {})["brick"] = best
        save_cache(cache_path, cache)
    return {"key": key, "brick": best, "source": "tuned", "brick_ms": {str(b): t for b, t in times.items()}}


def _nn_mean_ms(prob, samples: int) -> float:
    import torch

    total = 0.0
    for it in range(1, samples + 1):
        prob.sample(0, it)
        prob.nearest()
        best = None
        for _ in range(2):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            prob.nearest()
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            best = ms if best is None else min(best, ms)
        total += best
    return total / samples


def tune_nn(prob, samples: int = 3, reps: int = 3) -> float:
    """The search autotuner on the query samples of `samples` iterations, then
    every setting it chose timed on all of them; keeps the best mean and
    returns it (ms)."""
    chosen = []
    for it in range(1, samples + 1):
        prob.sample(0, it)
        shape, _ = prob.autotune(reps=reps)
        if shape not in chosen:
            chosen.append(shape)
    best, best_ms = None, None
    for shape in chosen:
        gp.gp_set_nn_params(prob.ctx, *shape)
        ms = _nn_mean_ms(prob, samples)
        if best_ms is None or ms < best_ms:
            best, best_ms = shape, ms
    gp.gp_set_nn_params(prob.ctx, *best)
    return best_ms


def tune(prob, cache_path: Optional[str] = DEFAULT_CACHE, samples: int = 3, reps: int = 3) -> dict:
    """Settings for this problem: from the cache when its class is there,
    else timed (and stored when cache_path is given).  Leaves the problem
    holding the query sample of iteration `samples` and its nearest points.

    Returns {"key", "source" ("cache" or "tuned"), "nn", "grad", and, when
    timed, "nn_ms" and "grad_ms"}."""
    key = class_key(prob.specs, prob.device.index or 0)
    cache = load_cache(cache_path) if cache_path else {}
    if key in cache and "nn" in cache[key] and "grad" in cache[key]:
        entry = {k: cache[key][k] for k in ("nn", "grad")}
        try:
            apply(prob, entry)
        except gp.GridPullError:
            # settings this build of the library refuses (an older cache): tune again
            gp.gp_set_nn_params(prob.ctx, 8, 1)
            gp.gp_set_grad_params(prob.ctx)
        else:
            prob.sample(0, samples)
            prob.nearest()
            return {"key": key, "source": "cache", **entry}
    nn_ms = tune_nn(prob, samples, reps)
    prob.sample(0, samples)
    prob.nearest()
    grad, grad_ms = prob.autotune_grad(reps=reps)
    entry = {"nn": list(gp.gp_get_nn_params(prob.ctx)), "grad": list(grad)}
    if cache_path:
        cache = load_cache(cache_path)
        cache.setdefault(key, {}).update(entry)
        save_cache(cache_path, cache)
    return {"key": key, "source": "tuned", **entry, "nn_ms": nn_ms, "grad_ms": list(grad_ms)}
