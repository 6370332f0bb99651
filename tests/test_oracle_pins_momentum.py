"""Pins of the oracle's momentum operator and of the relaxation residual E_k
against facts that do not come from the oracle itself.

* Linear-upwind convection (Section 4: momentum convection by linear upwind,
  applied as an explicit deferred correction on the old velocity): on a
  smooth field carried by a uniform flux the discrete convection term is a
  second-order approximation of d(u)/ds; the plain upwind part alone is only
  first order.
* The transpose viscous term (Eq. NSE1d / NSEc: div(mu (grad u + grad u^T))):
  a manufactured velocity whose x component is zero, in a fluid whose
  viscosity varies across the grid, has an x component of the viscous
  operator that comes from the transpose term alone.
* E_k (Section 3.2): two tiny grids where the normalised residual is a
  rational number worked out by hand (tests/golden/ek_hand_cases.json).

The operator values are read from the oracle's assembled momentum equation:
with the old and the current velocity equal, A u - H = (V / rAU) (u - H/A)
is the sum of the convection and diffusion terms of the cell (the time
derivative cancels), which the tests compare with the exact derivatives of
the manufactured fields at the cell centres.  Cells within two of the box
boundary are left out (their stencils see the boundary values)."""
import json
import math
import os

import numpy as np
import pytest

from oracle.pyoracle import Oracle
from paper_2105_10576_amd import cases

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _box(dim, shape, h, fl1, fl2, bc, alpha):
    nx, ny, nz = shape
    return cases._case("pin", dim, nx, ny, nz, h, fl1, fl2, 0.0, 90.0, bc, 0.0,
                       np.zeros(nx * ny * nz, np.uint8), alpha, 1e-6, 1, 1, 1e-6)


def _face_counts(c):
    nx, ny, nz, d = c["nx"], c["ny"], c["nz"], c["dim"]
    nf = [(nx + 1) * ny * nz, nx * (ny + 1) * nz, nx * ny * (nz + 1) if d == 3 else 0]
    return nf


# ---------------------------------------------------------------------------
# linear-upwind convection: second order with the deferred correction
# ---------------------------------------------------------------------------

def _convection_error(n, dim, e, sign):
    """Max error of the discrete convection term, relative to max|du/ds|,
    for u_c = sin(k s) (c = e) and cos(k s) (c != e) carried along
    direction e by a uniform volumetric flux of sign `sign`."""
    L, rho, u0 = 1e-3, 1000.0, 0.1
    h = L / n
    shape = [1, 1, 1]
    shape[e] = n
    if dim == 2 and e == 2:
        raise ValueError
    # the walls of the one-cell-wide directions add mu S / (h/2) to A: keep mu
    # small enough that this zero-order friction is far below (kh)^2 / 12
    fl = dict(rho=rho, mu=1e-14)
    bc = [cases.BC_WALL] * 6
    bc[2 * e], bc[2 * e + 1] = cases.BC_INLET, cases.BC_OUTLET
    c = _box(dim, tuple(shape), h, fl, fl, bc, np.zeros(n))
    o = Oracle(c)
    S = h ** (dim - 1)
    V = h ** dim
    nf = _face_counts(c)
    phi = np.zeros(sum(nf))
    off = sum(nf[:e])
    phi[off:off + nf[e]] = sign * u0 * S
    o.set("phi_cr", phi)
    s = (np.arange(n) + 0.5) * h
    k = 2 * math.pi / L
    U = np.zeros((dim, n))
    for comp in range(dim):
        U[comp] = np.sin(k * s) if comp == e else np.cos(k * s)
    o.set("U_cr", U.reshape(-1))
    dt = h / u0                       # Courant 1: time and convection terms of similar size
    o.pressure_solve(1, dt, 1e-6, 1)  # assembles A, H from u^o = u; the solve itself is not used
    HbyA = o.get("HbyA").reshape(dim, n)
    rAU = o.get("rAU")
    # A u - H = sum_f s_f F_f u_f (+ a 1e-14 viscous part), F = rho * flux
    conv = (V / rAU) * (U - HbyA) / (rho * sign * u0 * V)
    exact = np.zeros((dim, n))
    for comp in range(dim):
        exact[comp] = k * np.cos(k * s) if comp == e else -k * np.sin(k * s)
    sl = slice(2, n - 2)
    return np.abs(conv[:, sl] - exact[:, sl]).max() / k


@pytest.mark.parametrize("dim,e", [(2, 0), (2, 1), (3, 2)])
@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_linear_upwind_convection_is_second_order(dim, e, sign):
    """The convection term of a smooth field at h, h/2, h/4 falls 4x per
    halving, to 1/12 (kh)^2 of max|du/ds| (the truncation error of linear
    upwind).  Without the deferred correction, with it doubled or with its
    sign flipped the scheme is first order (error ~ kh/2, kh/2 or kh) and
    the ratio drops to 2.  Both flux signs and each direction are checked,
    so a mistake in one branch or one index is caught too."""
    errs = [_convection_error(n, dim, e, sign) for n in (32, 64, 128)]
    for a, b in zip(errs, errs[1:]):
        assert 3.6 < a / b < 4.4, errs
    kh = 2 * math.pi / 128
    assert errs[-1] == pytest.approx(kh * kh / 12, rel=0.05), errs


# ---------------------------------------------------------------------------
# transpose viscous term: variable viscosity, manufactured velocity
# ---------------------------------------------------------------------------

def _viscous_error(n):
    """u = (0, sin(k x) cos(k y)) in a fluid with alpha = (1 + sin(k y)) / 2
    and mu = alpha mu1 + (1 - alpha) mu2, so mu' = dmu/dy.  The exact
    div(mu (grad u + grad u^T)) is
      x: d/dy(mu du_y/dx)                 = k cos(kx) (mu' cos(ky) - mu k sin(ky))
         (the transpose term alone, since u_x = 0)
      y: div(mu grad u_y) + d/dy(mu du_y/dy) = -k sin(kx) (3 mu k cos(ky) + 2 mu' sin(ky))
    Returns the max errors of both components relative to max|exact|."""
    L, rho, mu1, mu2 = 1e-3, 1000.0, 3e-3, 1e-3
    h = L / n
    k = 2 * math.pi / L
    x = (np.arange(n) + 0.5) * h
    X, Y = np.meshgrid(x, x, indexing="xy")      # [j, i]
    alpha = 0.5 * (1 + np.sin(k * Y))
    bc = [cases.BC_WALL, cases.BC_OUTLET, cases.BC_WALL, cases.BC_WALL, 0, 0]
    c = _box(2, (n, n, 1), h, dict(rho=rho, mu=mu1), dict(rho=rho, mu=mu2), bc, alpha.reshape(-1))
    o = Oracle(c)
    U = np.zeros((2, n, n))
    U[1] = np.sin(k * X) * np.cos(k * Y)
    o.set("U_cr", U.reshape(-1))
    V = h * h
    o.pressure_solve(1, 1.0, 1e-6, 1)
    HbyA = o.get("HbyA").reshape(2, n, n)
    rAU = o.get("rAU").reshape(n, n)
    visc = -(V / rAU) * (U - HbyA) / V            # = div(mu (grad u + grad u^T)) per unit volume
    mu = alpha * mu1 + (1 - alpha) * mu2
    dmu = (mu1 - mu2) * 0.5 * k * np.cos(k * Y)
    ex_x = k * np.cos(k * X) * (dmu * np.cos(k * Y) - mu * k * np.sin(k * Y))
    ex_y = -k * np.sin(k * X) * (3 * mu * k * np.cos(k * Y) + 2 * dmu * np.sin(k * Y))
    sl = (slice(2, n - 2), slice(2, n - 2))
    return (np.abs(visc[0][sl] - ex_x[sl]).max() / np.abs(ex_x).max(),
            np.abs(visc[1][sl] - ex_y[sl]).max() / np.abs(ex_y).max())


def test_transpose_viscous_term_variable_viscosity():
    """The x component of the viscous operator, which only the transpose
    term supplies here, matches its exact value to second order (errors
    falling ~4x from 32^2 to 64^2 cells, below 1 % at 64^2); so does the y
    component, which holds both terms.  Dropping the transpose term leaves x
    at zero (error 1), flipping its sign gives error 2, doubling it error 1,
    swapping the gradient's indices (du_c/dx_e instead of du_e/dx_c) makes it
    vanish again, and a face gradient taken from one cell instead of the mean
    of the two loses the mu d2u/dxdy part."""
    ex32, ey32 = _viscous_error(32)
    ex64, ey64 = _viscous_error(64)
    assert ex64 < 0.01 and ey64 < 0.01, (ex64, ey64)
    assert 3.0 < ex32 / ex64 < 5.0, (ex32, ex64)
    assert 3.0 < ey32 / ey64 < 5.0, (ey32, ey64)


# ---------------------------------------------------------------------------
# boundary terms: uniform flow through an open duct is a fixed point
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dim", [2, 3])
def test_uniform_flow_is_a_fixed_point(dim):
    """Uniform flow u_in along x from an inlet to an outlet, the side faces
    open (p = 0, zero-gradient u), is an exact steady solution of the
    momentum and mass equations: every convective and viscous flux
    difference vanishes, the inlet brings in exactly the momentum the
    outlet carries out.  One viscous step from that state must return it
    unchanged (u = u_in, p = 0, fluxes u_in S) to round-off.  Catches a
    missing inflow momentum F u_b or inlet viscous term mu S/(h/2) u_b, a
    zero inlet velocity in the viscous step's assembly, and a missing
    outflow term at the outlet."""
    nx, ny, nz = (16, 4, 1) if dim == 2 else (8, 4, 4)
    h, u, rho, mu = 1e-5, 0.01, 1000.0, 1e-3
    bc = [cases.BC_INLET, cases.BC_OUTLET] + [cases.BC_OUTLET] * 4
    fl = dict(rho=rho, mu=mu)
    c = cases._case("duct", dim, nx, ny, nz, h, fl, fl, 0.0, 90.0, bc, u,
                    np.zeros(nx * ny * nz, np.uint8), np.zeros(nx * ny * nz), 1e-6, 1, 1, 1e-6)
    o = Oracle(c)
    nc = nx * ny * nz
    S = h ** (dim - 1)
    nf = _face_counts(c)
    phi = np.zeros(sum(nf))
    phi[:nf[0]] = u * S
    U = np.zeros((dim, nc))
    U[0] = u
    o.set("phi_vd", phi)
    o.set("U_vd", U.reshape(-1))
    assert o.viscous_step(0.25 * h / u) == 0
    Un = o.get("U_vd").reshape(dim, nc)
    assert np.abs(Un[0] - u).max() <= 1e-12 * u
    assert np.abs(Un[1:]).max() <= 1e-12 * u
    assert np.abs(o.get("p_vd")).max() <= 1e-12 * rho * u * u
    assert np.abs(o.get("phi_vd") - phi).max() <= 1e-12 * u * S


# ---------------------------------------------------------------------------
# density time levels of d(rho u)/dt and the convecting flux
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("step", ["viscous", "capillary"])
def test_momentum_of_a_cell_whose_density_changes(step):
    """Alpha is moved by its transport flux (phi_vd in the viscous step,
    phi_cr in a capillary sub-step) while the momentum is convected by
    phi_vd + phi_cr, which the test sets to zero.  Without convection and
    with negligible viscosity the predicted velocity of every cell is
    (rho(alpha_old) u_old) / rho(alpha_new): the cell keeps its momentum
    while its density changes (d(rho u)/dt with rho before and after the
    transport, Eq. NSE1d / NSEc).  Catches rho_new used in both time
    levels, and a convecting flux other than phi_vd + phi_cr."""
    nx, ny, h, u = 16, 4, 1e-5, 0.01
    x = np.arange(nx) + 0.5
    a0 = np.tile(0.5 * (1 - np.tanh((x - 6.0) / 1.5)), (ny, 1)).reshape(-1)
    bc = [cases.BC_INLET, cases.BC_OUTLET, cases.BC_WALL, cases.BC_WALL, 0, 0]
    ph1, ph2 = dict(rho=1000.0, mu=1e-18), dict(rho=100.0, mu=1e-18)
    c = cases._case("dens", 2, nx, ny, 1, h, ph1, ph2, 0.0, 90.0, bc, u,
                    np.zeros(nx * ny, np.uint8), a0, 1e-6, 1, 1, 1e-6)
    o = Oracle(c)
    nf = _face_counts(c)
    fwd = np.zeros(sum(nf))
    fwd[:nf[0]] = u * h
    U = np.zeros((2, nx * ny))
    U[0] = u
    dt = 0.5 * h / u
    if step == "viscous":
        o.set("phi_vd", fwd)
        o.set("phi_cr", -fwd)
        o.set("U_vd", U.reshape(-1))
        assert o.viscous_step(dt) == 0
    else:
        o.set("phi_cr", fwd)
        o.set("phi_vd_prev", -fwd)
        o.set("U_cr", U.reshape(-1))
        rc, kf, E = o.capillary_relax(dt, 1, 1, 0.0)
        assert rc == 0
    a1 = o.get("alpha")
    assert np.abs(a1 - a0).max() > 0.05          # the densities did change
    rho = lambda a: a * 1000.0 + (1 - a) * 100.0
    HbyA = o.get("HbyA").reshape(2, -1)
    assert np.allclose(HbyA[0], rho(a0) * u / rho(a1), rtol=1e-10, atol=0)
    assert np.abs(HbyA[1]).max() <= 1e-10 * u


# ---------------------------------------------------------------------------
# E_k worked by hand on a tiny grid with a solid cell and p != 0
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("case", json.load(open(os.path.join(GOLD, "ek_hand_cases.json")))["cases"],
                         ids=lambda c: c["name"])
def test_normalised_residual_hand_cases(case):
    """E_k of the first corrector equals the value worked out by hand from
    the definition (the fixture gives the matrix, the right-hand side and
    the sums).  Catches a mean taken over all cells instead of the fluid
    ones, a missing |b - M pbar| term, pbar = 0, an L2 instead of an L1 sum
    and a residual taken after the solve instead of before it."""
    nx, ny, h, dt, rho = 3, 2, 1e-5, 1e-6, 1000.0
    mask = np.zeros(nx * ny, np.uint8)
    mask[3] = 1
    fl = dict(rho=rho, mu=1e-12)
    bc = [cases.BC_WALL, cases.BC_OUTLET, cases.BC_WALL, cases.BC_WALL, 0, 0]
    c = cases._case("ek", 2, nx, ny, 1, h, fl, fl, 0.0, 90.0, bc, 0.0, mask, np.zeros(nx * ny),
                    dt, 1, 1, 0.0)
    o = Oracle(c)
    scale = 1.0 if case["p_scale"] == "unit" else rho * h / (2 * dt)
    p = np.zeros(nx * ny)
    for cell, v in case["p"].items():
        p[int(cell)] = v * (scale if int(cell) != 3 else 1.0)
    U = np.zeros(2 * nx * ny)
    for cell, v in case["u_x"].items():
        U[int(cell)] = v
    o.set("p_cr", p)
    o.set("U_cr", U)
    rc, kf, E = o.capillary_relax(dt, 1, 1, 0.0)
    assert rc == 0 and kf == 1
    assert E[0] == pytest.approx(case["E"], rel=1e-9)
