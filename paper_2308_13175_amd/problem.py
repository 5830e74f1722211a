"""Optimisation driver over the C ABI: one context, its device buffers, and
the per-iteration sequence sample -> NN -> forward -> backward -> Adam step.

Also a torch.autograd.Function (PullLoss) whose backward is the library's
hand-written adjoint, and hipGraph capture of a whole iteration through
torch's graph API.  Everything numerical runs in libgridpull.so.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import gridpull as gp


@dataclasses.dataclass
class ShapeSpec:
    points: np.ndarray           # float32 [J, 3]
    dims: tuple
    lo: tuple
    hi: tuple
    n_queries: int
    sigma: object = 0.0          # scalar or float32 [J]


def spec_from_synth(shape) -> ShapeSpec:
    d = shape.domain
    return ShapeSpec(shape.points, d.dims, d.lo, d.hi, shape.n_queries, shape.sigma)


@dataclasses.dataclass
class AdamConfig:
    lr0: float = 1.0
    decay: float = 0.3
    decay_every: int = 400
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8


class Problem:
    """All shapes of one batch in one context (n_shapes = 1 for a single shape)."""

    def __init__(self, shapes: Sequence[ShapeSpec], m1: int = 3, m2: int = 3,
                 weights=(1.0, 1.0, 0.005), device: int = 0, adam: Optional[AdamConfig] = None, brick: int = 8):
        self.device = torch.device("cuda", device)
        self.brick = int(brick)
        self.specs = list(shapes)
        self.weights = tuple(float(x) for x in weights)
        self.adam = adam or AdamConfig()
        self.m1, self.m2 = int(m1), int(m2)
        pts = np.concatenate([np.asarray(s.points, dtype=np.float32).reshape(-1, 3) for s in self.specs])
        self.n_points = len(pts)
        dev = self.device
        self.px = torch.from_numpy(np.ascontiguousarray(pts[:, 0])).to(dev)
        self.py = torch.from_numpy(np.ascontiguousarray(pts[:, 1])).to(dev)
        self.pz = torch.from_numpy(np.ascontiguousarray(pts[:, 2])).to(dev)
        self.point_off = []
        self.query_off = []
        shp = []
        po = qo = 0
        for s in self.specs:
            J = len(s.points)
            shp.append(gp.make_shape(s.dims, s.lo, s.hi, po, J, qo, s.n_queries))
            self.point_off.append(po)
            self.query_off.append(qo)
            po += J
            qo += int(s.n_queries)
        self.n_queries = qo
        self.n_shapes = len(self.specs)
        # per-point sigma if any shape gives one
        if any(np.ndim(s.sigma) > 0 for s in self.specs):
            sig = np.concatenate([np.asarray(s.sigma, np.float32) if np.ndim(s.sigma) > 0
                                  else np.full(len(s.points), float(s.sigma), np.float32) for s in self.specs])
            self.sigma = torch.from_numpy(sig).to(dev)
            self.sigma_const = 0.0
        else:
            sc = {float(s.sigma) for s in self.specs}
            if len(sc) == 1:
                self.sigma = None
                self.sigma_const = sc.pop()
            else:
                sig = np.concatenate([np.full(len(s.points), float(s.sigma), np.float32) for s in self.specs])
                self.sigma = torch.from_numpy(sig).to(dev)
                self.sigma_const = 0.0
        with torch.cuda.device(dev):
            self.ctx = gp.gp_create(device)
            self.n_slots, self.n_active = gp.gp_build_band(self.ctx, shp, self.px, self.py, self.pz, m1, m2,
                                                           self.brick)
            self.slot_begin = gp.gp_shape_slots(self.ctx, self.n_shapes)
        n = max(self.n_slots, 1)
        self.field = torch.zeros(n, dtype=torch.float32, device=dev)
        self.grad = torch.zeros(n, dtype=torch.float32, device=dev)
        self.m = torch.zeros(n, dtype=torch.float32, device=dev)
        self.v = torch.zeros(n, dtype=torch.float32, device=dev)
        Q = max(self.n_queries, 1)
        self.qx = torch.zeros(Q, dtype=torch.float32, device=dev)
        self.qy = torch.zeros(Q, dtype=torch.float32, device=dev)
        self.qz = torch.zeros(Q, dtype=torch.float32, device=dev)
        self.nn = torch.zeros(Q, dtype=torch.int32, device=dev)
        self.src = torch.zeros(Q, dtype=torch.int32, device=dev)
        self.loss = torch.zeros(self.n_shapes, 5, dtype=torch.float64, device=dev)
        self.n_valid = torch.zeros(self.n_shapes, dtype=torch.int64, device=dev)
        self.dloss = torch.ones(self.n_shapes, dtype=torch.float64, device=dev)
        self.normals = None          # (nx, ny, nz, weight) once set_normals is called
        self.normal_term = torch.zeros(self.n_shapes, dtype=torch.float64, device=dev)

    # -- lifetime ----------------------------------------------------------
    def close(self):
        if getattr(self, "ctx", None) is not None:
            gp.gp_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- set-up helpers ----------------------------------------------------
    def init_sphere(self, centres=None, radii=None):
        """Geometric initialisation (Sec. 3): a sphere of radius two cells at the domain centre."""
        if centres is None:
            centres = [tuple(0.5 * (s.lo[a] + s.hi[a]) for a in range(3)) for s in self.specs]
        if radii is None:
            radii = [2.0 * min((s.hi[a] - s.lo[a]) / s.dims[a] for a in range(3)) for s in self.specs]
        gp.gp_init_sphere(self.ctx, centres, radii, self.field)
        self.m.zero_()
        self.v.zero_()
        self.grad.zero_()

    def set_dense_field(self, dense: Sequence[np.ndarray]):
        """Load per-shape dense x-major vertex arrays into the slots."""
        flat = np.concatenate([np.asarray(d, np.float32).reshape(-1) for d in dense])
        t = torch.from_numpy(flat).to(self.device)
        gp.gp_gather_vertices(self.ctx, t, self.field)

    def dense_field(self, fill: float = 0.0) -> List[np.ndarray]:
        sizes = [int(np.prod(np.asarray(s.dims, np.int64) + 1)) for s in self.specs]
        t = torch.full((sum(sizes),), float(fill), dtype=torch.float32, device=self.device)
        gp.gp_scatter_vertices(self.ctx, self.field, t)
        out = t.cpu().numpy()
        res, o = [], 0
        for n in sizes:
            res.append(out[o:o + n].copy())
            o += n
        return res

    def dense_grad(self) -> List[np.ndarray]:
        sizes = [int(np.prod(np.asarray(s.dims, np.int64) + 1)) for s in self.specs]
        t = torch.zeros(sum(sizes), dtype=torch.float32, device=self.device)
        gp.gp_scatter_vertices(self.ctx, self.grad, t)
        out = t.cpu().numpy()
        res, o = [], 0
        for n in sizes:
            res.append(out[o:o + n].copy())
            o += n
        return res

    def layout(self):
        vid = torch.empty(max(self.n_slots, 1), dtype=torch.int64, device=self.device)
        flags = torch.empty(max(self.n_slots, 1), dtype=torch.uint8, device=self.device)
        gp.gp_export_layout(self.ctx, vid, flags)
        return vid[: self.n_slots].cpu().numpy(), flags[: self.n_slots].cpu().numpy()

    def set_queries(self, q: np.ndarray):
        q = np.asarray(q, np.float32).reshape(-1, 3)
        assert len(q) == self.n_queries
        self.qx.copy_(torch.from_numpy(np.ascontiguousarray(q[:, 0])))
        self.qy.copy_(torch.from_numpy(np.ascontiguousarray(q[:, 1])))
        self.qz.copy_(torch.from_numpy(np.ascontiguousarray(q[:, 2])))

    def queries(self) -> np.ndarray:
        return torch.stack([self.qx, self.qy, self.qz], 1)[: self.n_queries].cpu().numpy()

    # -- the iteration -----------------------------------------------------
    def sample(self, seed: int, iteration: int):
        gp.gp_sample_queries(self.ctx, seed, iteration, self.sigma, self.sigma_const,
                             self.qx, self.qy, self.qz, self.src)

    def nearest(self):
        gp.gp_nn_query(self.ctx, self.qx[: self.n_queries], self.qy[: self.n_queries],
                       self.qz[: self.n_queries], self.nn)

    def autotune(self, reps: int = 2):
        """Pick the NN search grid and shape by timing them on the current queries (leaves nn filled).

        Returns ((group_span, first_shell, tile_parts, skip_empty, morton_sort, cell_points), best ms)."""
        return gp.gp_autotune_nn(self.ctx, self.qx[: self.n_queries], self.qy[: self.n_queries],
                                 self.qz[: self.n_queries], self.nn, reps)

    def autotune_grad(self, reps: int = 2):
        """Pick the gradient-pass and TV settings by timing them on the current
        queries, nearest points and field.

        Returns ((window_cap, window_max_passes, tv_forward_wave_from,
        tv_backward_wave_from), (query pass, TV forward, TV backward ms))."""
        return gp.gp_autotune_grad(self.ctx, self.qx[: self.n_queries], self.qy[: self.n_queries],
                                   self.qz[: self.n_queries], self.nn, self.field, self.weights, reps)

    def forward(self, field: Optional[torch.Tensor] = None):
        f = self.field if field is None else field
        gp.gp_pull_forward(self.ctx, self.qx[: self.n_queries], self.qy[: self.n_queries],
                           self.qz[: self.n_queries], self.nn, f, self.weights, self.loss, self.n_valid)
        return self.loss

    def forward_token(self) -> int:
        """Token of the last forward on this context (0: none usable)."""
        return gp.gp_forward_token(self.ctx)

    def backward(self, field: Optional[torch.Tensor] = None, grad: Optional[torch.Tensor] = None,
                 dloss: Optional[torch.Tensor] = None, token: Optional[int] = None):
        """Adjoint of the forward named by token (default: the last one)."""
        f = self.field if field is None else field
        g = self.grad if grad is None else grad
        d = self.dloss if dloss is None else dloss
        tok = self.forward_token() if token is None else token
        gp.gp_pull_backward(self.ctx, self.qx[: self.n_queries], self.qy[: self.n_queries],
                            self.qz[: self.n_queries], self.nn, f, self.weights, d, g, tok)
        return g

    def forward_backward(self, field: Optional[torch.Tensor] = None, grad: Optional[torch.Tensor] = None,
                         dloss: Optional[torch.Tensor] = None):
        """Loss and gradient in one pass over the queries (same results as forward + backward)."""
        f = self.field if field is None else field
        g = self.grad if grad is None else grad
        d = self.dloss if dloss is None else dloss
        gp.gp_pull_forward_backward(self.ctx, self.qx[: self.n_queries], self.qy[: self.n_queries],
                                    self.qz[: self.n_queries], self.nn, f, self.weights, d, self.loss,
                                    self.n_valid, g)
        return self.loss

    def step(self, t: Optional[int] = None, lr0: Optional[float] = None):
        """Adam step at iteration t; t=None uses the context's device-resident counter."""
        a = self.adam
        gp.gp_step(self.ctx, self.field, self.grad, self.m, self.v, 0 if t is None else int(t),
                   a.lr0 if lr0 is None else lr0, a.decay, a.decay_every, a.beta1, a.beta2, a.eps)

    def set_normals(self, normals: np.ndarray, weight: float):
        """Ground-truth unit normals of the points (indexed like them): every
        iteration then adds weight * the normal supervision term."""
        n = np.asarray(normals, np.float32).reshape(-1, 3)
        assert len(n) == self.n_points
        self.normals = tuple(torch.from_numpy(np.ascontiguousarray(n[:, a])).to(self.device) for a in range(3)) + (
            float(weight),)

    def iteration(self, t: Optional[int] = None, seed: int = 0):
        """One full optimisation iteration (sample, NN, forward, backward, Adam).

        t=None takes the iteration number from the device-resident counter, so
        the same launches can be captured once and replayed as a graph.
        """
        self.sample(seed, -1 if t is None else int(t))
        self.nearest()
        self.forward_backward()
        if self.normals is not None:
            nx, ny, nz, w = self.normals
            n = self.n_queries
            gp.gp_pull_normals(self.ctx, self.qx[:n], self.qy[:n], self.qz[:n], self.nn, self.field, nx, ny, nz, w,
                               self.dloss, self.normal_term, self.grad)
        self.step(t)

    def sync(self):
        gp.gp_sync(self.ctx)


class PullLoss(torch.autograd.Function):
    """Per-shape total loss L (Eq. 8) as a differentiable function of the field.

    forward runs gp_pull_forward, backward runs the hand-written adjoint
    gp_pull_backward with the incoming gradient as the per-shape scale.  The
    forward's token goes with the graph node: if another forward on the same
    problem, or a library call that rewrote its queries, nearest points or
    field, came in between, the backward raises (GP_ERR_STATE) instead of
    using that state.
    """

    @staticmethod
    def forward(ctx, field: torch.Tensor, problem: Problem):
        loss = problem.forward(field.detach())
        ctx.problem = problem
        ctx.token = problem.forward_token()
        ctx.save_for_backward(field)
        return loss[:, 0].clone()

    @staticmethod
    def backward(ctx, grad_total: torch.Tensor):
        (field,) = ctx.saved_tensors
        g = torch.zeros_like(field)
        ctx.problem.backward(field.detach(), g, grad_total.detach().to(torch.float64).contiguous(), ctx.token)
        return g, None


def pull_loss(field: torch.Tensor, problem: Problem) -> torch.Tensor:
    return PullLoss.apply(field, problem)


class GraphedIteration:
    """A whole iteration captured once as a hipGraph (torch's graph API) and replayed.

    The sampler's iteration index and the Adam step number come from the
    context's device-resident counter, so every replay is the next iteration.
    """

    def __init__(self, problem: Problem, seed: int = 0):
        self.problem = problem
        dev = problem.device
        s = torch.cuda.Stream(device=dev)
        s.wait_stream(torch.cuda.current_stream(dev))
        with torch.cuda.stream(s):
            problem.iteration(None, seed)      # warm-up outside the graph
        torch.cuda.current_stream(dev).wait_stream(s)
        torch.cuda.synchronize(dev)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            problem.iteration(None, seed)

    def replay(self):
        self.graph.replay()
