"""The C ABI: symbols, loading, argument and state errors."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gridpull.h")
LIB = os.path.join(ROOT, "paper_2308_13175_amd", "libgridpull.so")


def _declared():
    text = open(HEADER).read()
    return re.findall(r"^(?:gp_status|void|const char\*|uint64_t)\s+(gp_\w+)\(", text, re.M)


def test_header_declares_the_abi():
    names = _declared()
    for n in ("gp_create", "gp_destroy", "gp_last_error", "gp_build_band", "gp_nn_query", "gp_pull_forward",
              "gp_pull_backward", "gp_step", "gp_sample_queries", "gp_sync"):
        assert n in names


def test_library_loads_and_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.fail("libgridpull.so is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(LIB)
    for n in _declared():
        assert hasattr(lib, n), n
    from paper_2308_13175_amd import gridpull

    assert set(gridpull.EXPORTS) == set(_declared())


def test_binding_refuses_a_missing_library(tmp_path):
    from paper_2308_13175_amd import gridpull

    saved = gridpull._lib
    gridpull._lib = None
    try:
        with pytest.raises(ImportError):
            gridpull.load_library(str(tmp_path / "absent.so"))
    finally:
        gridpull._lib = saved


def test_null_context_is_an_argument_error():
    lib = ctypes.CDLL(LIB)
    lib.gp_sync.restype = ctypes.c_int
    lib.gp_sync.argtypes = [ctypes.c_void_p]
    assert lib.gp_sync(None) == 1
    lib.gp_create.restype = ctypes.c_int
    lib.gp_create.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]
    assert lib.gp_create(None, 0, None) == 1


# ---------------------------------------------------------------------------
# error paths on the GPU
# ---------------------------------------------------------------------------

@pytest.mark.gpu
def test_state_and_argument_errors():
    import torch

    from paper_2308_13175_amd import gridpull as gp
    from paper_2308_13175_amd import synth

    ctx = gp.gp_create(0)
    try:
        q = torch.zeros(4, device="cuda")
        nn = torch.zeros(4, dtype=torch.int32, device="cuda")
        with pytest.raises(gp.GridPullError) as e:
            gp.gp_nn_query(ctx, q, q, q, nn)
        assert e.value.status == 6            # GP_ERR_STATE before gp_build_band
        dom = synth.cube_domain(8)
        pts = torch.tensor([[0.1, 0.2, 0.3], [0.5, -0.5, 0.25]], device="cuda")
        px, py, pz = [pts[:, a].contiguous() for a in range(3)]
        good = gp.make_shape(dom.dims, dom.lo, dom.hi, 0, 2, 0, 4)
        for brick in (0, 2, 6, 32):
            with pytest.raises(gp.GridPullError) as e:
                gp.gp_build_band(ctx, [good], px, py, pz, 3, 3, brick=brick)
            assert e.value.status == 1        # brick edge not 4, 8 or 16
        with pytest.raises(gp.GridPullError) as e:
            gp.gp_build_band(ctx, [gp.make_shape((0, 8, 8), dom.lo, dom.hi, 0, 2, 0, 4)], px, py, pz, 3, 3)
        assert e.value.status == 1
        with pytest.raises(gp.GridPullError) as e:
            gp.gp_build_band(ctx, [gp.make_shape(dom.dims, dom.lo, dom.hi, 0, 2, 0, 4)] * 2, px, py, pz, 3, 3)
        assert e.value.status == 1            # overlapping slices
        for m1, m2 in [(-1, 3), (3, 1025)]:
            with pytest.raises(gp.GridPullError) as e:
                gp.gp_build_band(ctx, [good], px, py, pz, m1, m2)
            assert e.value.status == 1        # band width out of range
        bad = torch.tensor([[0.1, 0.2, 0.3], [1.5, 0.0, 0.0]], device="cuda")
        with pytest.raises(gp.GridPullError) as e:
            gp.gp_build_band(ctx, [good], *[bad[:, a].contiguous() for a in range(3)], 3, 3)
        assert e.value.status == 2 and "point 1" in str(e.value)
        n_slots, n_act = gp.gp_build_band(ctx, [good], px, py, pz, 1, 1)
        assert n_slots > 0 and n_act > 0
        field = torch.zeros(n_slots, device="cuda")
        loss = torch.zeros(1, 5, dtype=torch.float64, device="cuda")
        nv = torch.zeros(1, dtype=torch.int64, device="cuda")
        dl = torch.ones(1, dtype=torch.float64, device="cuda")
        with pytest.raises(gp.GridPullError) as e:
            gp.gp_pull_backward(ctx, q, q, q, nn, field, (1, 1, 0.005), dl, field, 0)
        assert e.value.status == 6            # backward before forward
        assert gp.gp_forward_token(ctx) == 0
        # the token: only the last forward, on the arrays it read, unwritten since
        qq = torch.tensor([0.1, 0.5, 0.1, 0.5], device="cuda")
        gp.gp_nn_query(ctx, qq, qq, qq, nn)
        grad = torch.zeros_like(field)
        gp.gp_pull_forward(ctx, qq, qq, qq, nn, field, (1, 1, 0.005), loss, nv)
        t1 = gp.gp_forward_token(ctx)
        assert t1 != 0
        gp.gp_pull_backward(ctx, qq, qq, qq, nn, field, (1, 1, 0.005), dl, grad, t1)
        gp.gp_pull_forward(ctx, qq, qq, qq, nn, field, (1, 1, 0.005), loss, nv)
        t2 = gp.gp_forward_token(ctx)
        assert t2 not in (0, t1)
        for args, tok in (((qq, qq, qq, nn, field), t1),                 # an older forward
                          ((qq, qq, qq, nn, field.clone()), t2)):        # another field array
            with pytest.raises(gp.GridPullError) as e:
                gp.gp_pull_backward(ctx, *args, (1, 1, 0.005), dl, grad, tok)
            assert e.value.status == 6
        gp.gp_nn_query(ctx, qq, qq, qq, nn)                               # rewrites the forward's nn
        assert gp.gp_forward_token(ctx) == 0
        with pytest.raises(gp.GridPullError) as e:
            gp.gp_pull_backward(ctx, qq, qq, qq, nn, field, (1, 1, 0.005), dl, grad, t2)
        assert e.value.status == 6
        q3 = torch.zeros(3, device="cuda")
        with pytest.raises(gp.GridPullError) as e:
            gp.gp_pull_forward(ctx, q3, q3, q3, nn, field, (1, 1, 0.005), loss, nv)
        assert e.value.status == 1            # wrong query count
        # an out-of-range nearest index is reported by the next sync
        bad_nn = torch.tensor([7, 0, 0, 1], dtype=torch.int32, device="cuda")
        gp.gp_pull_forward(ctx, qq, qq, qq, bad_nn, field, (1, 1, 0.005), loss, nv)
        with pytest.raises(gp.GridPullError) as e:
            gp.gp_sync(ctx)
        assert e.value.status == 1
        gp.gp_sync(ctx)                        # the flag is cleared
        # a non-finite field value is reported as a numeric error
        gp.gp_nn_query(ctx, qq, qq, qq, nn)
        field.fill_(float("nan"))
        gp.gp_pull_forward(ctx, qq, qq, qq, nn, field, (1, 1, 0.005), loss, nv)
        with pytest.raises(gp.GridPullError) as e:
            gp.gp_sync(ctx)
        assert e.value.status == 7
    finally:
        gp.gp_destroy(ctx)
