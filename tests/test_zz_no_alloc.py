"""gp_pull_forward_static, the forward that allocates nothing (its scratch is a
static device array), against gp_pull_forward on the same inputs: two calls
in a row, the second with a smaller input on another context of the same GPU
(so it finds the first call's contents in the array)."""
import numpy as np
import pytest

from paper_2308_13175_amd import synth
from helpers import log, make_problem, spec

pytestmark = pytest.mark.gpu


def _problem(specs):
    prob = make_problem(specs)
    prob.set_dense_field([synth.sphere_sdf_field(synth.Domain(s.dims, s.lo, s.hi), 0.5, noise=0.01, seed=1)
                          for s in specs])
    prob.sample(seed=5, iteration=1)
    prob.nearest()
    return prob


def test_static_forward_equals_forward_on_two_calls():
    import torch

    from paper_2308_13175_amd import gridpull as gp

    big = [spec(synth.sphere_points(10_000, 0.5, seed=1), synth.cube_domain(64), 50_000, 0.02),
           spec(synth.sphere_points(4_000, 0.45, seed=2), synth.cube_domain(48), 30_000, 0.03)]
    small = [spec(synth.sphere_points(3_000, 0.5, seed=3), synth.cube_domain(32), 9_000, 0.04)]
    for name, specs in (("two shapes, 80k queries", big), ("one shape, 9k queries", small)):
        log("case: static forward, %s" % name)
        prob = _problem(specs)
        n = prob.n_queries
        ref = prob.forward().clone()
        nv_ref = prob.n_valid.clone()
        token = prob.forward_token()
        assert token != 0
        loss = torch.full_like(ref, -1.0)
        nv = torch.full_like(nv_ref, -1)
        gp.gp_pull_forward_static(prob.ctx, prob.qx[:n], prob.qy[:n], prob.qz[:n], prob.nn, prob.field,
                                  prob.weights, loss, nv)
        prob.sync()
        assert torch.equal(nv, nv_ref)
        got, want = loss.cpu().numpy(), ref.cpu().numpy()
        assert np.all(np.abs(got - want) <= 1e-12 * np.abs(want)), (got, want)
        # the context's forward state is untouched: its backward still runs
        assert prob.forward_token() == token
        g0 = torch.zeros_like(prob.grad)
        prob.backward(grad=g0)
        prob.forward()
        g1 = torch.zeros_like(prob.grad)
        prob.backward(grad=g1)
        prob.sync()
        assert float((g0 - g1).abs().max()) <= 1e-5 * float(g1.abs().max())
        prob.close()
