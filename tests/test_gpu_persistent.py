"""The persistent pressure solve (one launch per solve: its workgroups take
the tiles of every CG iteration, multigrid cycle and refinement step from a
work queue in device memory) against the grid-wide launches, host-driven in
chunks.  The tiles run the same bodies on the same blocks and the
reductions keep their block order, so the two modes must agree bit for bit:
contexts in both precisions with both preconditioners (the multigrid tail
from LDS and from global memory), a 3D grid, the stand-alone solve, and the
serving engine with a mix of requests."""
import numpy as np
import pytest

from paper_2105_10576_amd import cases

pytestmark = pytest.mark.gpu

FIELDS = ("alpha", "p", "U")


def _steps(oscar, c, precision, mode, steps):
    g = oscar.Oscar(c, precision=precision, solve_mode=mode)
    out = []
    for _ in range(steps):
        rc1, rc2, kf, E = g.step()
        st = g.stats()
        out.append((kf, E, st["pcg_iters_call"], st["refine_steps_call"], {f: g.get(f) for f in FIELDS}))
    g.close()
    return out


def _same(a, b):
    for step, (x, y) in enumerate(zip(a, b)):
        assert x[0] == y[0], ("k_f", step)
        assert np.array_equal(x[1], y[1]), ("E", step)
        assert x[2] == y[2], ("CG iterations", step)
        assert x[3] == y[3], ("refinement steps", step)
        for f in FIELDS:
            assert np.array_equal(x[4][f], y[4][f]), (f, step)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("precond", [0, 1])
def test_context_persistent_equals_launches(precision, precond):
    """Channel bubble 128 x 32, three steps.  The multigrid tail block is
    39 KB in mixed precision (run from LDS) and 78 KB in FP64 (from global
    memory)."""
    from paper_2105_10576_amd import oscar
    c = cases.channel_bubble()
    c["precond"] = precond
    if precision == 1:
        c["pcg_rtol"] = 1e-10
    a = _steps(oscar, c, precision, oscar.SOLVE_LAUNCHES, 3)
    b = _steps(oscar, c, precision, oscar.SOLVE_PERSISTENT, 3)
    _same(a, b)


def test_context_persistent_equals_launches_3d():
    """3D constricted channel 64 x 32 x 32, mixed precision, multigrid (two
    sweeps on the grid-wide coarse levels): one step."""
    from paper_2105_10576_amd import oscar
    c = cases.constricted_channel(nx=64, ny=32, nz=32, max_iters=3)
    c["precond"] = 1
    c["pcg_rtol"] = 1e-8
    a = _steps(oscar, c, 1, oscar.SOLVE_LAUNCHES, 1)
    b = _steps(oscar, c, 1, oscar.SOLVE_PERSISTENT, 1)
    _same(a, b)


@pytest.mark.parametrize("precision", [0, 1])
def test_standalone_solve_persistent_equals_launches(precision):
    from paper_2105_10576_amd import oscar
    c = cases.micromodel(nx=480, ny=256, seed=7, r_lo=5, r_hi=9, inlet_cols=8, buffer=16, max_iters=2, ca=1e-4)
    c["precond"] = 1
    res = {}
    for mode in (oscar.SOLVE_LAUNCHES, oscar.SOLVE_PERSISTENT):
        g = oscar.Oscar(c, precision=precision, solve_mode=mode)
        g.viscous_step(c["dt_vd"])
        rc, it, r = g.pressure_solve(1, c["dt_vd"] / c["n_sub"], 1e-9, 500)
        res[mode] = (it, r, g.get("p_cr"))
        g.close()
    a, b = res[oscar.SOLVE_LAUNCHES], res[oscar.SOLVE_PERSISTENT]
    assert a[0] == b[0] and a[1] == b[1]
    assert np.array_equal(a[2], b[2])


def _engine_run(oscar, reqs, precision, mode):
    heap = sum(oscar.workspace_size(c, precision) for c in reqs) + (1 << 20)
    e = oscar.Engine(8, heap, precision=precision, solve_mode=mode)
    slots = {e.admit(reqs[0]): 0, e.admit(reqs[1]): 1}
    e.run(2)
    slots[e.admit(reqs[2])] = 2
    e.run(1)
    slots[e.admit(reqs[3])] = 3
    got = {}
    for _ in range(10000):
        done, act = e.poll()
        for s in done:
            got[slots[s]] = e.fetch(s)
            e.release(s)
        if len(got) == len(reqs):
            break
        e.run(1)
    e.close()
    assert len(got) == len(reqs)
    return got


@pytest.mark.parametrize("precision", [0, 1])
def test_engine_persistent_equals_launches(precision):
    """A mix of Jacobi and multigrid requests of different sizes and
    corrector counts, admitted while others run."""
    from paper_2105_10576_amd import oscar
    reqs = [
        cases.channel_bubble(nx=64, ny=16, n_sub=12, max_iters=6),
        cases.channel_bubble(nx=96, ny=32, n_sub=None, max_iters=5, ca=1e-3),
        cases.micromodel(nx=160, ny=64, seed=11, r_lo=4, r_hi=8, inlet_cols=8, buffer=16, max_iters=4, ca=1e-4),
        cases.channel_bubble(nx=50, ny=14, n_sub=12, max_iters=3),
    ]
    reqs[1]["precond"] = 1
    reqs[2]["precond"] = 1
    reqs[3]["n_corr"] = 2
    if precision == 1:
        for c in reqs:
            c["pcg_rtol"] = 1e-8
    a = _engine_run(oscar, reqs, precision, oscar.SOLVE_LAUNCHES)
    b = _engine_run(oscar, reqs, precision, oscar.SOLVE_PERSISTENT)
    for i in range(len(reqs)):
        assert a[i]["k_f"] == b[i]["k_f"] and a[i]["status"] == b[i]["status"], i
        for f in FIELDS:
            assert np.array_equal(a[i][f], b[i][f]), (i, f)


@pytest.mark.parametrize("precision", [0, 1])
def test_brick_kernel_equals_single_cell_kernel(precision):
    """On a 3D grid of at least 4M cells the grid-wide path runs the fine
    pre-smoothing on LDS-staged bricks, while the persistent solve's tiles
    run the single-cell body: the two must agree bit for bit in both
    precisions (256 x 128 x 128 constricted channel, one step of one
    sub-step)."""
    from paper_2105_10576_amd import oscar
    c = cases.constricted_channel(nx=256, ny=128, nz=128, max_iters=1)
    c["precond"] = 1
    c["pcg_rtol"] = 1e-8 if precision == 1 else 1e-10
    a = _steps(oscar, c, precision, oscar.SOLVE_LAUNCHES, 1)
    b = _steps(oscar, c, precision, oscar.SOLVE_PERSISTENT, 1)
    _same(a, b)


@pytest.mark.parametrize("precision", [0, 1])
def test_split_coarse_sweeps_equal_fused_kernels(precision):
    """A grid-wide level of at least 128k cells with two sweeps per side runs
    each sweep as a launch of its own (the stored sweep read on the radius-1
    star), while the persistent solve's tiles run the fused kernels, which
    evaluate it again at the neighbours: the two must agree bit for bit in
    both precisions (128 x 128 x 64 constricted channel, whose level 1 has
    131072 cells; one step of one sub-step)."""
    from paper_2105_10576_amd import oscar
    c = cases.constricted_channel(nx=128, ny=128, nz=64, max_iters=1)
    c["precond"] = 1
    c["pcg_rtol"] = 1e-8 if precision == 1 else 1e-10
    a = _steps(oscar, c, precision, oscar.SOLVE_LAUNCHES, 1)
    b = _steps(oscar, c, precision, oscar.SOLVE_PERSISTENT, 1)
    _same(a, b)
