"""The tuning module on the GPU: tune once, store, and a second problem of the
same size class takes the stored settings without timing; the results are
the oracle's either way."""
import numpy as np
import pytest

import oracle
from paper_2308_13175_amd import synth
from helpers import assert_grad_close, assert_terms_close, log, loss_terms, make_problem, spec

pytestmark = pytest.mark.gpu


def _problem():
    dom = synth.cube_domain(64)
    pts = synth.sphere_points(10_000, 0.5, seed=31)
    prob = make_problem([spec(pts, dom, 50_000, 0.02)])
    prob.set_dense_field([synth.sphere_sdf_field(dom, 0.5, noise=0.01, seed=32)])
    return prob, dom, pts


def test_tune_then_read_from_cache(tmp_path):
    from paper_2308_13175_amd import gridpull as gp
    from paper_2308_13175_amd import tuning

    path = str(tmp_path / "tuning.json")
    log("case: tuning, first problem (tuned and stored)")
    prob, dom, pts = _problem()
    first = tuning.tune(prob, path, samples=2, reps=1)
    assert first["source"] == "tuned" and first["key"].endswith("|q2^16-p2^13-single")
    assert tuning.load_cache(path)[first["key"]] == {"nn": first["nn"], "grad": first["grad"]}
    assert list(gp.gp_get_nn_params(prob.ctx)) == first["nn"]
    assert list(gp.gp_get_grad_params(prob.ctx)) == first["grad"]
    prob.close()

    log("case: tuning, second problem of the class (read from the cache)")
    prob, dom, pts = _problem()
    second = tuning.tune(prob, path, samples=2, reps=1)
    assert second["source"] == "cache" and second["key"] == first["key"]
    assert list(gp.gp_get_nn_params(prob.ctx)) == first["nn"]
    assert list(gp.gp_get_grad_params(prob.ctx)) == first["grad"]
    # the problem holds iteration 2's queries and their nearest points: check them and the step
    q = np.stack([prob.qx[: prob.n_queries].cpu().numpy(), prob.qy[: prob.n_queries].cpu().numpy(),
                  prob.qz[: prob.n_queries].cpu().numpy()], 1)
    assert np.array_equal(prob.nn[: prob.n_queries].cpu().numpy(), oracle.nn_bruteforce(q, pts))
    D = prob.dense_field()[0].astype(np.float64)
    cf, vf = oracle.build_band(dom.dims, dom.lo, dom.hi, pts, 3, 3)
    ref = oracle.loss_grad(dom.dims, dom.lo, dom.hi, cf, vf, D, q, prob.nn[: prob.n_queries].cpu().numpy(), pts)
    prob.grad.zero_()
    prob.forward_backward()
    prob.sync()
    got, nv = loss_terms(prob)
    assert int(nv[0]) == ref["n_valid"]
    assert_terms_close(got[0], ref)
    assert_grad_close(prob.dense_grad()[0], ref["dD"])
    prob.close()


def test_stale_cache_entry_is_tuned_again(tmp_path):
    """A cache entry holding settings this library refuses (written by a build
    with other window sizes) is not applied: the problem is tuned again and
    the entry replaced."""
    from paper_2308_13175_amd import gridpull as gp
    from paper_2308_13175_amd import tuning

    log("case: tuning, stale cache entry")
    path = str(tmp_path / "tuning.json")
    prob, dom, pts = _problem()
    key = tuning.class_key(prob.specs)
    tuning.save_cache(path, {key: {"nn": [8, 1, 1, 0, 1, 8], "grad": [4608, 16, 2048, 16384]}})
    out = tuning.tune(prob, path, samples=2, reps=1)
    assert out["source"] == "tuned" and out["key"] == key
    assert out["grad"][0] in (2048, 4096, 6144)
    assert tuning.load_cache(path)[key] == {"nn": out["nn"], "grad": out["grad"]}
    assert list(gp.gp_get_grad_params(prob.ctx)) == out["grad"]
    prob.close()
