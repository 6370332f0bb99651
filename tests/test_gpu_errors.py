"""Error and warning paths of the C ABI on the GPU, and checkpoint/restore:
non-finite input and state, the Brackbill limit, the iteration cap, and a
run restored from the fields of an earlier step."""
import numpy as np
import pytest

from paper_2105_10576_amd import cases

pytestmark = pytest.mark.gpu


def _small(**over):
    c = cases.channel_bubble(nx=64, ny=16, n_sub=12, max_iters=4)
    c.update(over)
    return c


def test_set_field_rejects_non_finite_values():
    """A NaN or an infinity in a field handed to oscar_set_field is refused
    with OSCAR_E_NONFINITE and the field keeps its value."""
    from paper_2105_10576_amd import oscar
    c = _small()
    g = oscar.Oscar(c, precision=0)
    before = g.get("U_vd")
    for bad in (np.nan, np.inf):
        u = before.copy()
        u[7] = bad
        with pytest.raises(oscar.OscarError) as ex:
            g.set("U_vd", u)
        assert ex.value.code == oscar.E_NONFINITE
        assert np.array_equal(g.get("U_vd"), before)


@pytest.mark.parametrize("precision", [0, 1])
def test_overflowing_state_reports_non_finite(precision):
    """A velocity field of 1e300 (FP64) or 1e38 (FP32) overflows the momentum
    assembly: the step ends with OSCAR_E_NONFINITE (the iteration cap bounds
    the solves of the non-finite system) and the context can still be read
    and destroyed."""
    from paper_2105_10576_amd import oscar
    c = _small(pcg_max_it=20)
    g = oscar.Oscar(c, precision=precision)
    big = 1e300 if precision == 0 else 1e38
    g.set("U_vd", np.full(2 * c["nx"] * c["ny"], big))
    print("overflow, precision", precision, flush=True)
    rc = g.viscous_step(c["dt_vd"], check=False)
    assert rc == oscar.E_NONFINITE
    assert g.get("alpha").shape == (c["nx"] * c["ny"],)
    g.close()


def test_substep_at_the_brackbill_limit_is_rejected():
    """dt_vd / n_sub must lie below the Brackbill limit sqrt(rho_bar h^3 /
    (2 pi sigma)) (Section 2.2): at the limit, and above it, the relaxation
    returns OSCAR_E_UNSTABLE before any work; just below it runs."""
    from paper_2105_10576_amd import oscar
    c = _small()
    g = oscar.Oscar(c, precision=0)
    dtb = oscar.dt_brackbill(c["rho1"], c["rho2"], c["h"], c["sigma"])
    a0 = g.get("alpha")
    for dt_vd, n in ((dtb * 4, 4), (dtb * 8, 4)):
        rc, kf, E = g.capillary_relax(dt_vd, n, 1, 0.0, check=False)
        assert rc == oscar.E_UNSTABLE
        assert np.array_equal(g.get("alpha"), a0)
    rc, kf, E = g.capillary_relax(dtb * 3.99, 4, 1, 0.0, check=False)
    assert rc == oscar.OK and kf == 1


@pytest.mark.parametrize("precond", [0, 1])
def test_iteration_cap_warns(precond):
    """A pressure solve that reaches pcg_max_it before its tolerance returns
    the warning OSCAR_W_PCG_MAXIT (outputs valid) and counts the hit."""
    from paper_2105_10576_amd import oscar
    c = _small(pcg_max_it=2, precond=precond)
    g = oscar.Oscar(c, precision=0)
    rc = g.viscous_step(c["dt_vd"])
    assert rc == oscar.W_PCG_MAXIT
    st = g.stats()
    assert st["pcg_maxit_hits"] >= 1 and st["last_pcg_iters"] <= 2
    assert np.isfinite(g.get("U_vd")).all()


STATE = ("alpha", "U_vd", "U_cr", "p_vd", "p_cr", "phi_vd", "phi_vd_prev", "phi_cr")


@pytest.mark.parametrize("precision,precond", [(0, 0), (1, 1)])
def test_checkpoint_restore_is_bitwise(precision, precond):
    """Fields read after step 1 and written into a fresh context continue
    the run exactly: steps 2 and 3 from the checkpoint equal steps 2 and 3
    of the uninterrupted run bit for bit (every other array is recomputed
    from these at the start of a step)."""
    from paper_2105_10576_amd import oscar
    c = _small(precond=precond)
    if precision == 1:
        c["pcg_rtol"] = 1e-8
    a = oscar.Oscar(c, precision=precision)
    a.step()
    ck = {k: a.get(k) for k in STATE}
    for _ in range(2):
        a.step()
    b = oscar.Oscar(c, precision=precision)
    for k, v in ck.items():
        b.set(k, v)
    for _ in range(2):
        b.step()
    for k in ("alpha", "p", "U", "phi_cr"):
        assert np.array_equal(a.get(k), b.get(k)), k
