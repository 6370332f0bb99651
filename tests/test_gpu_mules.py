"""Parity of the iterative limiter (mules_iter > 1: passes after the first
limit the unused antidiffusive flux against the first pass's local bounds)
between the HIP path, through the C ABI, and the FP64 CPU oracle.  The FP64
limiter passes are written in the oracle's operation order, so one transport
is bitwise equal; whole steps follow the tolerances of the single-pass
path."""
import numpy as np
import pytest

from oracle.pyoracle import Oracle
from paper_2105_10576_amd import cases

pytestmark = pytest.mark.gpu


def _oscar():
    from paper_2105_10576_amd import oscar
    return oscar


def rel_linf(x, ref):
    den = np.abs(ref).max()
    return float(np.abs(x - ref).max() / (den if den > 0 else 1.0))


def _rough_box(shape, seed):
    nx, ny, nz, dim = shape
    solid = ((3, 2, 0), (4, 2, 0)) if dim == 2 else ((1, 1, 1), (2, 3, 4))
    c = cases.tiny_box(nx=nx, ny=ny, nz=nz, dim=dim, seed=seed, solid_cells=solid, theta=70.0)
    rng = np.random.Generator(np.random.PCG64(seed + 100))
    a = rng.random(nx * ny * nz)
    a[: a.size // 2] = np.round(a[: a.size // 2])   # sharp half, smooth half
    c["alpha0"] = a
    c["sigma"] = 0.0   # transport only: no capillary time-step limit
    return c


@pytest.mark.parametrize("passes", [2, 3, 8])
@pytest.mark.parametrize("shape", [(37, 19, 1, 2), (13, 9, 7, 3)])
def test_limiting_passes_bitwise(shape, passes):
    """One transport of a rough alpha field (half sharp 0/1, half random) by a
    random flux field at a Courant number of 0.8, several blocks and a
    ragged tail: alpha after `passes` limiting passes is bitwise equal to
    the oracle's, and differs from the single-pass result (the later passes
    did apply flux)."""
    o = _oscar()
    c = _rough_box(shape, seed=5)
    f = cases.random_fields(c, seed=31)
    probe = Oracle(c)
    probe.set("phi_cr", f["phi"])
    probe.capillary_relax(1e-7, 1, 1, 0.0)
    dt = 1e-7 * 0.8 / probe.stats()["max_courant"]
    out = {}
    for m in (1, passes):
        cm = dict(c, mules_iter=m)
        g, r = o.Oscar(cm, precision=o.FP64), Oracle(cm)
        for side in (g, r):
            side.set("phi_cr", f["phi"])
            side.capillary_relax(dt, 1, 1, 0.0)
        ag, ar = g.get("alpha"), r.get("alpha")
        print(shape, m, "max |gpu - oracle|", np.abs(ag - ar).max(), flush=True)
        assert np.array_equal(ag, ar), (m, np.abs(ag - ar).max())
        assert g.stats()["max_courant"] == pytest.approx(0.8, rel=1e-12)
        out[m] = ag
    assert not np.array_equal(out[1], out[passes])


def test_channel_bubble_three_passes_fp64():
    """Three OSCAR steps of the scaled channel bubble with three limiting
    passes: FP64 GPU within 1e-9 relative of the oracle on alpha, p and U,
    the same completed sub-steps, and phase mass conserved to 1e-12."""
    o = _oscar()
    c = cases.channel_bubble(nx=64, ny=16, n_sub=12, max_iters=12)
    c["mules_iter"] = 3
    g, r = o.Oscar(c, precision=o.FP64), Oracle(c)
    for step in range(3):
        kg, ko = g.step()[2], r.step()[2]
        assert kg == ko, step
    for fld in ("alpha", "p", "U"):
        assert rel_linf(g.get(fld), r.get(fld)) <= 1e-9, fld
    so = r.stats()
    assert abs(g.stats()["mass_phase1"] - so["mass"]) <= 1e-12 * so["mass"]
    assert g.stats()["mass_defect"] <= 1e-12 * so["mass"]


def test_channel_bubble_three_passes_mixed():
    """The mixed path (FP32 transport and limiter passes) with three passes:
    p and U within 1e-5 relative of the FP64 oracle after the first two
    steps, within the regression envelope of the single-pass mixed path
    (1e-3) after the third (the FP32 storage of alpha limits the curvature
    to about six significant digits, which the bubble's start-up amplifies),
    and the interface within 0.01 cells along every row."""
    o = _oscar()
    c = cases.channel_bubble(nx=64, ny=16, n_sub=12, max_iters=12)
    c["pcg_rtol"] = 1e-10
    c["mules_iter"] = 3
    g, r = o.Oscar(c, precision=o.MIXED), Oracle(c)
    for step, tol in ((1, 1e-5), (2, 1e-5), (3, 1e-3)):
        g.step()
        r.step()
        for fld in ("p", "U"):
            assert rel_linf(g.get(fld), r.get(fld)) <= tol, (step, fld)
    nx, ny = c["nx"], c["ny"]
    for ag, ao in zip(g.get("alpha").reshape(ny, nx), r.get("alpha").reshape(ny, nx)):
        sg = np.nonzero((ag[:-1] - 0.5) * (ag[1:] - 0.5) < 0)[0]
        so = np.nonzero((ao[:-1] - 0.5) * (ao[1:] - 0.5) < 0)[0]
        assert len(sg) == len(so)
        xg = sg + (0.5 - ag[sg]) / (ag[sg + 1] - ag[sg])
        xo = so + (0.5 - ao[so]) / (ao[so + 1] - ao[so])
        if len(xg):
            assert np.abs(xg - xo).max() <= 0.01


@pytest.mark.parametrize("precision", [0, 1])
def test_engine_slots_with_different_pass_counts(precision):
    """Requests with 1, 2, 3 and 4 limiting passes (2D and 3D, Jacobi and
    multigrid) share one engine: a launch runs as many passes as its
    largest request asks for and every slot stops at its own count, so each
    result equals the request run alone, bitwise."""
    o = _oscar()
    reqs = [cases.channel_bubble(nx=64, ny=16, n_sub=12, max_iters=6),
            cases.channel_bubble(nx=50, ny=14, n_sub=12, max_iters=3),
            cases.constricted_channel(nx=32, ny=16, nz=16, max_iters=3),
            cases.channel_bubble(nx=96, ny=32, n_sub=None, max_iters=4, ca=1e-3)]
    for c, m in zip(reqs, (3, 1, 2, 4)):
        c["mules_iter"] = m
    reqs[2]["pcg_rtol"] = 1e-8
    reqs[3]["precond"] = o.PC_MG
    if precision == 1:
        for c in reqs:
            c["pcg_rtol"] = 1e-8
    alone = []
    for c in reqs:
        e = o.Engine(2, 4 * o.workspace_size(c, precision), precision=precision)
        s = e.admit(c)
        assert s is not None
        for _ in range(10000):
            if e.poll()[0]:
                break
            e.run(1)
        alone.append(e.fetch(s))
        e.release(s)
        e.close()
    heap = sum(o.workspace_size(c, precision) for c in reqs) + (1 << 20)
    e = o.Engine(8, heap, precision=precision)
    slots = {e.admit(c): i for i, c in enumerate(reqs)}
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
    for i, a in enumerate(alone):
        assert got[i]["k_f"] == a["k_f"], i
        for f in ("alpha", "p", "U"):
            assert np.array_equal(got[i][f], a[f]), (i, f)
