"""The allocation-free entry point oscar_create_static, through the C ABI:
a context whose workspace is the library's static device array gives the
same results, bit for bit, as oscar_create with a caller-allocated
workspace, on two contexts in a row (the second on a smaller grid, after
the first is destroyed); a second live context on the device is refused,
and so is a grid too large for the array."""
import ctypes as C

import numpy as np
import pytest

from paper_2105_10576_amd import cases

pytestmark = pytest.mark.gpu

FIELDS = {"alpha": 0, "U": 1, "p": 2, "phi_cr": 9}


def _create_static(oscar, case, precision):
    import torch
    d, keep = oscar.make_desc(case, precision)
    ctx = C.c_void_p(None)
    stream = torch.cuda.current_stream()
    rc = oscar.lib().oscar_create_static(C.byref(d), C.c_void_p(stream.cuda_stream), C.byref(ctx))
    return rc, ctx


def _run(oscar, ctx, case, steps):
    L = oscar.lib()
    kf = C.c_int32(0)
    E = C.c_double(0.0)
    for _ in range(steps):
        assert L.oscar_viscous_step(ctx, case["dt_vd"]) == 0
        rc = L.oscar_capillary_relax(ctx, case["dt_vd"], case["n_sub"], case["max_iters"], case["tol"],
                                     C.byref(kf), C.byref(E))
        assert rc == 0
    out = {"k_f": kf.value}
    for name, fid in FIELDS.items():
        n = L.oscar_field_len(ctx, fid)
        a = np.empty(n)
        assert L.oscar_get_field(ctx, fid, a.ctypes.data_as(C.POINTER(C.c_double))) == 0
        out[name] = a
    return out


@pytest.mark.parametrize("precision,precond", [(0, 0), (1, 1)])
def test_static_workspace_matches_caller_workspace(precision, precond):
    from paper_2105_10576_amd import oscar
    L = oscar.lib()
    for nx, ny in ((96, 24), (48, 12)):      # the second context is smaller than the first
        c = cases.channel_bubble(nx=nx, ny=ny, n_sub=12, max_iters=4)
        c["precond"] = precond
        if precision == 1:
            c["pcg_rtol"] = 1e-8
        print("static workspace", nx, ny, precision, precond, flush=True)
        rc, ctx = _create_static(oscar, c, precision)
        assert rc == 0, L.oscar_last_error(None)
        rc2, ctx2 = _create_static(oscar, c, precision)
        assert rc2 == oscar.E_CAPACITY and not ctx2.value
        got = _run(oscar, ctx, c, 2)
        L.oscar_destroy(ctx)
        ref = oscar.Oscar(c, precision=precision)
        want = _run(oscar, ref.ctx, c, 2)
        ref.close()
        assert got["k_f"] == want["k_f"]
        for name in FIELDS:
            assert np.array_equal(got[name], want[name]), (nx, name)


def test_static_workspace_rejects_a_grid_too_large():
    from paper_2105_10576_amd import oscar
    c = cases.channel_bubble(nx=1024, ny=512, n_sub=12, max_iters=2)
    assert oscar.workspace_size(c, 0) > (64 << 20)
    rc, ctx = _create_static(oscar, c, 0)
    assert rc == oscar.E_WORKSPACE and not ctx.value
    c = cases.channel_bubble(nx=64, ny=16, n_sub=12, max_iters=2)
    rc, ctx = _create_static(oscar, c, 0)    # the array is free again after the refusal
    assert rc == 0
    oscar.lib().oscar_destroy(ctx)
