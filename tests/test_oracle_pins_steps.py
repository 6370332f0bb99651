"""Further pins of the oracle: the transport's high-order face value and
its bounds, the regularised interface normal, mass conservation of the
corrected fluxes, and the relaxation loop's stop and sum rules.  Each test
states the fact it checks and the mistakes that fail it."""

import numpy as np
import pytest

from oracle.pyoracle import Oracle
from paper_2105_10576_amd import cases


def _line_case(n, h, a, bc, u_in=0.0, sigma=0.0, theta=90.0, ph1=cases.WATER, ph2=cases.OIL):
    return cases._case("line", 2, n, 1, 1, h, ph1, ph2, sigma, theta, bc, u_in,
                       np.zeros(n, np.uint8), a, 1e-6, 1, 1, 1e-6)


def _x_flux(nx, ny, h, u):
    phi = np.zeros((nx + 1) * ny + nx * (ny + 1))
    phi[: (nx + 1) * ny] = u * h
    return phi


# ---------------------------------------------------------------------------
# transport: the van Leer face value is second order in space
# ---------------------------------------------------------------------------

def _transport_rate_error(n, sign, co=0.1):
    """One explicit transport step of a smooth monotone profile of tiny
    amplitude.  At Courant 0.1 the antidiffusive flux of every cell is far
    inside its local bounds, so the limiter passes the high-order flux
    whole, and (alpha - alpha_new) / (Co h) is the discrete flux divergence
    (alpha_f+ - alpha_f-)/h.  The amplitude (1e-12) keeps the interface
    normal |grad alpha| / (|grad alpha| + delta) near 1e-5, so the
    compression flux is negligible.  Returns the max error against
    d(alpha)/dx relative to its maximum."""
    L, u = 1e-3, 1e-3
    h = L / n
    x = (np.arange(n) + 0.5) * h
    A, w = 1e-12, L / 8
    a = A * (1.0 + 0.5 * np.tanh((x - 0.5 * L) / w))
    bc = [cases.BC_INLET, cases.BC_OUTLET, cases.BC_WALL, cases.BC_WALL, 0, 0]
    if sign < 0:
        bc[0], bc[1] = cases.BC_OUTLET, cases.BC_INLET
    o = Oracle(_line_case(n, h, a, bc))
    o.set("phi_cr", _x_flux(n, 1, h, sign * u))
    rc, kf, E = o.capillary_relax(co * h / u, 1, 1, 0.0)
    assert rc == 0
    rate = (a - o.get("alpha")) / (co * h) / sign
    exact = A * 0.5 / w / np.cosh((x - 0.5 * L) / w) ** 2
    sl = slice(2, n - 2)
    return np.abs(rate[sl] - exact[sl]).max() / exact.max()


@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_van_leer_flux_divergence_is_second_order(sign):
    """The van Leer face value (product form) reconstructs a smooth monotone
    profile to second order: the flux divergence error falls 4x per grid
    halving.  Plain upwind, or half the van Leer increment, are first order
    (ratio 2, errors 10x and 5x larger at 128 cells).  Both flow directions
    (the far-upwind cell UU is looked up on each side)."""
    errs = [_transport_rate_error(n, sign) for n in (32, 64, 128)]
    for a, b in zip(errs, errs[1:]):
        assert 3.7 < a / b < 4.3, errs
    assert errs[-1] < 1e-3, errs


def test_limiter_bounds_are_clipped_to_the_unit_interval():
    """The local bounds of the limiter are clipped to [0, 1].  A state that
    already exceeds 1 (a step from 1.02 down to 1.0, e.g. after round-off)
    carried at Courant 0.5: no antidiffusive flux may raise a cell above
    its low-order (upwind) value, since the upper bound is 1 and Q+ = 0.
    Without the clip the bound would be 1.02 and the front cell would be
    steepened above its upwind value."""
    n, h, u, co = 24, 1e-5, 1e-3, 0.5
    a = np.where(np.arange(n) < 8, 1.02, 1.0)
    bc = [cases.BC_INLET, cases.BC_OUTLET, cases.BC_WALL, cases.BC_WALL, 0, 0]
    o = Oracle(_line_case(n, h, a, bc))
    o.set("phi_cr", _x_flux(n, 1, h, u))
    rc, kf, E = o.capillary_relax(co * h / u, 1, 1, 0.0)
    new = o.get("alpha")
    upwind = a.copy()
    upwind[1:] = a[1:] - co * (a[1:] - a[:-1])      # zero-gradient inflow keeps cell 0
    assert (new <= upwind + 1e-15).all(), new - upwind
    assert new.sum() == pytest.approx(a.sum() - co * (a[-1] - a[0]), abs=1e-12)


# ---------------------------------------------------------------------------
# interface normal: the regularisation delta = 1e-8 / h
# ---------------------------------------------------------------------------

def test_regularised_normal_at_gradient_equal_to_delta():
    """On a linear ramp of slope exactly delta = 1e-8/h (alpha rises by 1e-8
    per cell) the Gauss gradient is exact away from the ends, and the face
    normal G / (|G| + delta) is 1/2.  Catches a gradient off by a factor
    (e.g. divided by 2h instead of h: normal 1/3) and a different delta."""
    n, h = 16, 1e-5
    a = 0.3 + 1e-8 * np.arange(n)
    bc = [cases.BC_WALL, cases.BC_OUTLET, cases.BC_WALL, cases.BC_WALL, 0, 0]
    o = Oracle(_line_case(n, h, a, bc, sigma=0.0))
    o.pressure_solve(1, 1e-9, 1e-6, 1)
    nx_faces = o.get("nhatf")[: n + 1]
    assert np.abs(nx_faces[2:n - 1] - 0.5).max() < 1e-6, nx_faces


def test_normal_on_open_boundary_faces_is_the_boundary_cells_own():
    """Inlet and outlet faces take the regularised gradient of their
    boundary cell.  On the same ramp of slope delta per cell, that cell's
    Gauss gradient, with the zero-gradient face value on the open face, is
    half the slope, so the face normal is (delta/2) / (delta/2 + delta) =
    1/3 at both ends.  Catches a zeroed normal on open faces (0), the
    neighbouring cell's gradient (1/2) and the mean of the two gradients
    (3/7)."""
    n, h = 16, 1e-5
    a = 0.3 + 1e-8 * np.arange(n)
    bc = [cases.BC_INLET, cases.BC_OUTLET, cases.BC_WALL, cases.BC_WALL, 0, 0]
    o = Oracle(_line_case(n, h, a, bc, sigma=0.0))
    o.pressure_solve(1, 1e-9, 1e-6, 1)
    nx_faces = o.get("nhatf")[: n + 1]
    assert abs(nx_faces[0] - 1.0 / 3.0) < 1e-6, nx_faces[:2]
    assert abs(nx_faces[n] - 1.0 / 3.0) < 1e-6, nx_faces[-2:]
    assert np.abs(nx_faces[2:n - 1] - 0.5).max() < 1e-6


# ---------------------------------------------------------------------------
# mass: the corrected face fluxes are divergence-free
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("shape", [(8, 6, 1, 2), (5, 4, 3, 3)])
def test_corrected_fluxes_are_divergence_free(shape):
    """After a PISO corrector the face fluxes phi = phi_HbyA - rAU_f S dp/h
    satisfy the discrete mass equation (Eq. md / Eq. mc) in every fluid cell
    to the pressure solver's tolerance: sum_f s_f phi_f = 0, inlet, outlet
    and wall faces included.  Catches a flux correction that disagrees with
    the pressure matrix (e.g. the outlet correction with the wrong sign, or
    a wrong outlet distance h instead of h/2)."""
    nx, ny, nz, dim = shape
    solid = ((3, 2, 0),) if dim == 2 else ((2, 1, 1),)
    c = cases.tiny_box(nx=nx, ny=ny, nz=nz, dim=dim, seed=3, solid_cells=solid)
    c["pcg_rtol"] = 1e-14
    o = Oracle(c)
    f = cases.random_fields(c, seed=5)
    o.set("U_vd", f["U"])
    o.set("phi_vd", f["phi"] * 0.0)
    dt = 1e-7
    assert o.viscous_step(dt) == 0
    o.set("U_cr", f["U"])
    rc, kf, E = o.capillary_relax(dt, 1, 1, 0.0)
    assert rc == 0
    mask = c["mask"].astype(bool)
    nc = nx * ny * nz
    nfx, nfy = (nx + 1) * ny * nz, nx * (ny + 1) * nz
    for name in ("phi_vd", "phi_cr"):
        phi = o.get(name)
        px = phi[:nfx].reshape(nz, ny, nx + 1)
        py = phi[nfx:nfx + nfy].reshape(nz, ny + 1, nx)
        div = (px[:, :, 1:] - px[:, :, :-1]) + (py[:, 1:, :] - py[:, :-1, :])
        if dim == 3:
            pz = phi[nfx + nfy:].reshape(nz + 1, ny, nx)
            div = div + (pz[1:] - pz[:-1])
        div = div.reshape(nc)[~mask]
        scale = np.abs(phi).max()
        assert scale > 0
        assert np.abs(div).max() <= 1e-11 * scale, (name, np.abs(div).max() / scale)


# ---------------------------------------------------------------------------
# relaxation loop: stop rule and the velocity sum (Section 3.2)
# ---------------------------------------------------------------------------

def test_relaxation_sum_is_divided_by_N_not_by_k_f():
    """When the loop stops early (k_f < N) the global velocity is
    U_vd + (1/N) sum of the k_f capillary velocities: the sum runs over the
    sub-steps performed, the divisor is the number N the viscous step was
    split into (Section 3.2)."""
    c = cases.channel_bubble(nx=64, ny=16, n_sub=12, max_iters=4)
    o = Oracle(c)
    rc1, rc2, kf, E = o.step(tol=0.0)
    assert kf == 4 < c["n_sub"]
    assert np.abs(o.get("U_sum")).max() > 0
    assert np.array_equal(o.get("U"), o.get("U_vd") + o.get("U_sum") / c["n_sub"])


def test_stopping_substep_is_accumulated():
    """With a tolerance every residual meets (E_k <= 1 always, by the
    triangle inequality; tol = 2) the loop stops after its first sub-step,
    k_f = 1, and that sub-step's velocity is in the sum: U_sum = u_cr^1,
    U = U_vd + u_cr^1 / N."""
    c = cases.channel_bubble(nx=64, ny=16, n_sub=12)
    o = Oracle(c)
    assert o.viscous_step(c["dt_vd"]) == 0
    rc, kf, E = o.capillary_relax(c["dt_vd"], c["n_sub"], c["n_sub"], 2.0)
    assert rc == 0 and kf == 1 and 0.0 < E[0] <= 1.0
    ucr = o.get("U_cr")
    assert np.abs(ucr).max() > 0
    assert np.array_equal(o.get("U_sum"), ucr)
    assert np.array_equal(o.get("U"), o.get("U_vd") + ucr / c["n_sub"])


def test_stop_rule_is_strict():
    """The loop stops after the sub-step whose E_k is below the tolerance
    (strictly).  A flat interface at rest has E_k = 0 in every sub-step: with
    tol = 0 the loop never stops early (k_f = max_iters), with tol = 1e-12
    it stops at once (k_f = 1)."""
    nx, ny = 16, 8
    a = np.zeros((ny, nx))
    a[:, : nx // 2] = 1.0
    c = cases._case("flat", 2, nx, ny, 1, 1e-5, cases.AIR, cases.WATER, 0.07, 90.0,
                    [cases.BC_WALL, cases.BC_OUTLET, cases.BC_WALL, cases.BC_WALL, 0, 0], 0.0,
                    np.zeros(nx * ny, np.uint8), a, 1e-6, 1, 1, 1e-6)
    dtb = cases.brackbill_limit(1.0, 1000.0, 1e-5, 0.07)
    rc, kf, E = Oracle(c).capillary_relax(dtb * 3, 6, 5, 0.0)
    assert rc == 0 and kf == 5 and not E.any()
    rc, kf, E = Oracle(c).capillary_relax(dtb * 3, 6, 5, 1e-12)
    assert rc == 0 and kf == 1


# ---------------------------------------------------------------------------
# solid voxels are walls: a channel bounded by the box or by solid rows
# ---------------------------------------------------------------------------

def test_solid_rows_behave_as_box_walls():
    """The same channel bubble bounded by wall faces of the box (64 x 16) or
    by a row of solid voxels on each side inside a 64 x 18 box: a face
    between a fluid and a solid cell is a wall face like a box wall, in
    every operator (transport stencil, wall adhesion, wall friction, pressure
    equation), so two OSCAR steps give the same fluid-cell values.  The
    fluid cells are visited in the same order, so the agreement is exact.
    Catches a stencil that reads a solid cell's value where it would take a
    boundary value (e.g. the far-upwind cell of the van Leer face value)."""
    a = cases.channel_bubble(nx=64, ny=16, n_sub=12, max_iters=3)
    nx, ny = a["nx"], a["ny"]
    b = dict(a)
    mask = np.zeros((ny + 2, nx), np.uint8)
    mask[0, :] = mask[-1, :] = 1
    alpha = np.zeros((ny + 2, nx))
    alpha[1:-1, :] = a["alpha0"].reshape(ny, nx)
    b.update(ny=ny + 2, mask=mask.reshape(-1), alpha0=alpha.reshape(-1))
    oa, ob = Oracle(a), Oracle(b)
    for _ in range(2):
        ra, rb = oa.step(), ob.step()
        assert ra[:3] == rb[:3]
        assert np.array_equal(ra[3], rb[3])
    for name, comps in (("alpha", 1), ("p", 1), ("U", 2), ("kappa", 1)):
        va = oa.get(name).reshape(comps, ny, nx)
        vb = ob.get(name).reshape(comps, ny + 2, nx)[:, 1:-1, :]
        assert np.array_equal(va, vb), name


def test_courant_number_above_one_is_rejected():
    """The explicit transport is stable only up to Courant 1 (Section 2.2):
    a step at Co = 1.2 reports OSCAR's 'unstable' status (-4), one at
    Co = 0.9 does not."""
    n, h, u = 16, 1e-5, 1e-3
    a = np.where(np.arange(n) < 4, 1.0, 0.0)
    bc = [cases.BC_INLET, cases.BC_OUTLET, cases.BC_WALL, cases.BC_WALL, 0, 0]
    for co, expect in ((0.9, 0), (1.2, -4)):
        o = Oracle(_line_case(n, h, a, bc))
        o.set("phi_cr", _x_flux(n, 1, h, u))
        rc, kf, E = o.capillary_relax(co * h / u, 1, 1, 0.0)
        assert rc == expect, (co, rc)
        assert o.stats()["max_courant"] == pytest.approx(co, rel=1e-12)
