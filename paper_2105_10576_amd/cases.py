"""Seeded synthetic inputs for the OSCAR capillary-relaxation path.

This module only builds inputs: voxel masks, initial phase fractions,
fluid properties, boundary types and the time-step recipe of each workload.
It holds none of the method's arithmetic and is the only module that both
the GPU library's callers and the CPU oracle's tests import.

The workloads stand in for the paper's three benchmarks (arXiv 2105.10576,
Section 5): a bubble in a straight 2D channel, CO2 injection into a 3D
constricted channel, drainage of a 2D micromodel; plus a batched mix of 2D
requests and a large 3D sphere pack.  Geometry of the paper's micromodel
(an external generator and a snappyHexMesh mesh) is not available; seeded
disc and sphere packings of the stated porosity replace it.

Time-step recipe (paper, Sections 2.2 and 5.1-5.3): the inlet speed follows
from Ca = mu U / sigma with the viscosity of the injected phase, the
viscous step is a fraction of dt_CFL = h / U, and the number of capillary
sub-steps N is the smallest integer with dt_vd / N below the Brackbill limit
sqrt(rho_bar h^3 / (2 pi sigma)), rho_bar the mean of the two densities.
"""
from __future__ import annotations

import math

import numpy as np

BC_WALL, BC_INLET, BC_OUTLET = 0, 1, 2

WATER = dict(rho=1000.0, mu=1.0e-3)
AIR = dict(rho=1.0, mu=1.8e-5)
CO2 = dict(rho=700.0, mu=5.0e-5)
BRINE = dict(rho=1000.0, mu=5.0e-4)
OIL = dict(rho=800.0, mu=5.0e-3)


# ---------------------------------------------------------------------------
# time-step recipe
# ---------------------------------------------------------------------------

def inlet_speed(ca: float, mu_injected: float, sigma: float) -> float:
    """U from Ca = mu U / sigma."""
    return ca * sigma / mu_injected


def brackbill_limit(rho1: float, rho2: float, h: float, sigma: float) -> float:
    rbar = 0.5 * (rho1 + rho2)
    return math.sqrt(rbar * h ** 3 / (2.0 * math.pi * sigma))


def smallest_substeps(dt_vd: float, dt_b: float) -> int:
    """Smallest integer N with dt_vd / N < dt_B."""
    n = max(1, int(math.ceil(dt_vd / dt_b)))
    while not dt_vd / n < dt_b:
        n += 1
    while n > 1 and dt_vd / (n - 1) < dt_b:
        n -= 1
    return n


# ---------------------------------------------------------------------------
# geometry helpers
# ---------------------------------------------------------------------------

def keep_outlet_connected(mask: np.ndarray, bc, dim: int) -> np.ndarray:
    """Turn solid every fluid component that touches no outlet face.

    A fluid pocket without an outlet has a singular pressure equation; the
    library rejects such masks, so the generators remove them first.
    mask is indexed [k, j, i] (x fastest in memory), 1 = solid."""
    from scipy import ndimage

    fluid = mask == 0
    lab, n = ndimage.label(fluid)
    keep = np.zeros(n + 1, dtype=bool)
    sides = []
    # (bc index, slice selecting the cells adjacent to that box face)
    sides.append((0, (slice(None), slice(None), 0)))
    sides.append((1, (slice(None), slice(None), -1)))
    sides.append((2, (slice(None), 0, slice(None))))
    sides.append((3, (slice(None), -1, slice(None))))
    if dim == 3:
        sides.append((4, (0, slice(None), slice(None))))
        sides.append((5, (-1, slice(None), slice(None))))
    for b, sl in sides:
        if bc[b] == BC_OUTLET:
            keep[np.unique(lab[sl])] = True
    keep[0] = False
    out = mask.copy()
    out[fluid & ~keep[lab]] = 1
    return out


def _capsule_alpha(nx, ny, x0, x1, yc, rad, sub=16):
    """Phase fraction of a 2D capsule (points within rad of the segment
    (x0,yc)-(x1,yc)), in cell units, by sub x sub point sampling per cell."""
    off = (np.arange(sub) + 0.5) / sub
    xs = (np.arange(nx)[:, None] + off[None, :]).reshape(-1)
    ys = (np.arange(ny)[:, None] + off[None, :]).reshape(-1)
    X, Y = np.meshgrid(xs, ys, indexing="xy")          # [ny*sub, nx*sub]
    cx = np.clip(X, x0, x1)
    inside = (X - cx) ** 2 + (Y - yc) ** 2 <= rad * rad
    return inside.reshape(ny, sub, nx, sub).mean(axis=(1, 3))


def _disc_pack(rng, nx, ny, x_lo, x_hi, r_lo, r_hi, gap, target_solid, max_tries=200000, batch=512):
    """Random sequential addition of non-overlapping discs with a minimum gap,
    in cell units, inside x in [x_lo, x_hi) and at least `gap` from y walls,
    until the solid fraction of the zone reaches target_solid.  Candidates
    are drawn in batches (radius, then centre); each is accepted in draw
    order if it keeps the gap to every disc accepted before it."""
    cx = np.zeros(0)
    cy = np.zeros(0)
    cr = np.zeros(0)
    zone = (x_hi - x_lo) * ny
    area = 0.0
    tries = 0
    while area / zone < target_solid and tries < max_tries:
        r = rng.uniform(r_lo, r_hi, size=batch)
        x = x_lo + r + rng.uniform(size=batch) * np.maximum(x_hi - x_lo - 2 * r, 0.0)
        y = r + gap + rng.uniform(size=batch) * np.maximum(ny - 2 * (r + gap), 0.0)
        tries += batch
        if cx.size:
            d2 = (x[:, None] - cx[None, :]) ** 2 + (y[:, None] - cy[None, :]) ** 2
            ok = np.all(d2 >= (r[:, None] + cr[None, :] + gap) ** 2, axis=1)
        else:
            ok = np.ones(batch, dtype=bool)
        n_before = cx.size
        for t in np.nonzero(ok)[0]:
            if area / zone >= target_solid:
                break
            # against discs accepted earlier in this batch
            if cx.size > n_before:
                dd = (x[t] - cx[n_before:]) ** 2 + (y[t] - cy[n_before:]) ** 2
                if np.any(dd < (r[t] + cr[n_before:] + gap) ** 2):
                    continue
            cx = np.append(cx, x[t])
            cy = np.append(cy, y[t])
            cr = np.append(cr, r[t])
            area += math.pi * r[t] * r[t]
    X, Y = np.meshgrid(np.arange(nx) + 0.5, np.arange(ny) + 0.5, indexing="xy")
    solid = np.zeros((ny, nx), dtype=bool)
    for x0, y0, r0 in zip(cx, cy, cr):
        i0, i1 = max(0, int(x0 - r0) - 1), min(nx, int(x0 + r0) + 2)
        j0, j1 = max(0, int(y0 - r0) - 1), min(ny, int(y0 + r0) + 2)
        sub = (X[j0:j1, i0:i1] - x0) ** 2 + (Y[j0:j1, i0:i1] - y0) ** 2 <= r0 * r0
        solid[j0:j1, i0:i1] |= sub
    return solid


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------

def _case(name, dim, nx, ny, nz, h, ph1, ph2, sigma, theta, bc, u_in, mask, alpha0,
          dt_vd, n_sub, max_iters, tol, **extra):
    c = dict(name=name, dim=dim, nx=nx, ny=ny, nz=nz, h=h,
             rho1=ph1["rho"], mu1=ph1["mu"], rho2=ph2["rho"], mu2=ph2["mu"],
             sigma=sigma, theta_deg=theta, bc=list(bc), u_inlet=u_in,
             mask=np.ascontiguousarray(mask.reshape(-1), dtype=np.uint8),
             alpha0=np.ascontiguousarray(alpha0.reshape(-1), dtype=np.float64),
             dt_vd=dt_vd, n_sub=n_sub, max_iters=max_iters, tol=tol,
             n_corr=3, pcg_rtol=1e-12, pcg_max_it=20000)
    c.update(extra)
    return c


def channel_bubble(nx=128, ny=32, h=1e-6, ca=1e-2, cfl=0.25, n_sub=20, max_iters=None, tol=1e-4):
    """Air bubble in a straight 2D channel (paper Section 5.1, scaled): water
    injected at x-, outlet at x+, no-slip walls at y+-; capsule of air with
    length 0.47 nx, width 0.875 ny, centred at x = 0.31 nx; theta = 180 deg
    through the air (0 deg through the water)."""
    rad = 0.4375 * ny
    length = 0.46875 * nx
    xc = 0.3125 * nx
    x0, x1 = xc - 0.5 * length + rad, xc + 0.5 * length - rad
    alpha = _capsule_alpha(nx, ny, x0, x1, 0.5 * ny, rad)
    mask = np.zeros((ny, nx), dtype=np.uint8)
    sigma = 0.07
    u = inlet_speed(ca, WATER["mu"], sigma)
    dt_vd = cfl * h / u
    if n_sub is None:
        n_sub = smallest_substeps(dt_vd, brackbill_limit(AIR["rho"], WATER["rho"], h, sigma))
    return _case("channel_bubble_%dx%d" % (nx, ny), 2, nx, ny, 1, h, AIR, WATER, sigma, 180.0,
                 [BC_INLET, BC_OUTLET, BC_WALL, BC_WALL, BC_WALL, BC_WALL], u, mask, alpha,
                 dt_vd, n_sub, n_sub if max_iters is None else max_iters, tol, ca=ca)


def constricted_channel(nx=128, ny=64, nz=64, h=5e-6, ca=1e-4, cfl=0.1, slug=0.3, throat=0.4,
                        max_iters=None, tol=1e-4):
    """CO2 slug entering a 3D channel with a cosine throat of radius
    throat*R at mid-length (paper Section 5.2 analogue)."""
    R = 0.5 * ny
    x = np.arange(nx) + 0.5
    y = np.arange(ny) + 0.5
    z = np.arange(nz) + 0.5
    r = R * (1.0 - (1.0 - throat) * 0.5 * (1.0 + np.cos(2.0 * math.pi * (x - 0.5 * nx) / nx)))
    Z, Y, X = np.meshgrid(z, y, np.arange(nx), indexing="ij")
    rr = (Y - 0.5 * ny) ** 2 + (Z - 0.5 * nz) ** 2
    mask = (rr > r[X] ** 2).astype(np.uint8)
    xs = slug * nx
    col = np.clip(xs - np.arange(nx), 0.0, 1.0)            # fraction of each column below xs
    alpha = np.broadcast_to(col[None, None, :], (nz, ny, nx)).astype(np.float64).copy()
    alpha[mask == 1] = 0.0
    bc = [BC_INLET, BC_OUTLET, BC_WALL, BC_WALL, BC_WALL, BC_WALL]
    mask = keep_outlet_connected(mask, bc, 3)
    sigma = 0.03
    u = inlet_speed(ca, CO2["mu"], sigma)
    dt_vd = cfl * h / u
    n_sub = smallest_substeps(dt_vd, brackbill_limit(CO2["rho"], BRINE["rho"], h, sigma))
    return _case("constricted_channel_%dx%dx%d" % (nx, ny, nz), 3, nx, ny, nz, h, CO2, BRINE, sigma,
                 180.0, bc, u, mask, alpha, dt_vd, n_sub, n_sub if max_iters is None else max_iters,
                 tol, ca=ca)


def micromodel(nx=1024, ny=512, h=30e-6, ca=1e-5, cfl=0.1, seed=3, r_lo=8.0, r_hi=20.0, gap=2.0,
               porosity=0.6, inlet_cols=16, buffer=32, max_iters=20, tol=1e-4, theta=150.0):
    """2D oil-wet micromodel drainage (paper Section 5.3 analogue): discs of
    radius U[r_lo, r_hi] cells by seeded dart throwing, water injected at x-."""
    rng = np.random.Generator(np.random.PCG64(seed))
    solid = _disc_pack(rng, nx, ny, buffer, nx - buffer, r_lo, r_hi, gap, 1.0 - porosity)
    mask = solid.astype(np.uint8)
    bc = [BC_INLET, BC_OUTLET, BC_WALL, BC_WALL, BC_WALL, BC_WALL]
    mask = keep_outlet_connected(mask[None], bc, 2)[0]
    alpha = np.zeros((ny, nx))
    alpha[:, :inlet_cols] = 1.0
    alpha[mask == 1] = 0.0
    sigma = 0.03
    u = inlet_speed(ca, WATER["mu"], sigma)
    dt_vd = cfl * h / u
    n_sub = smallest_substeps(dt_vd, brackbill_limit(WATER["rho"], OIL["rho"], h, sigma))
    return _case("micromodel_%dx%d" % (nx, ny), 2, nx, ny, 1, h, WATER, OIL, sigma, theta, bc, u,
                 mask, alpha, dt_vd, n_sub, min(max_iters, n_sub), tol, ca=ca, seed=seed)


def sphere_pack(n=256, h=5e-6, ca=1e-5, cfl=0.1, seed=5, r_lo=6.0, r_hi=14.0, porosity=0.35,
                buffer=8, max_iters=20, tol=0.0, theta=140.0):
    """3D drainage of a seeded overlapping-sphere pack of the given porosity
    between inlet and outlet buffers of `buffer` voxels."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nx = ny = nz = n
    solid = np.zeros((nz, ny, nx), dtype=bool)
    x_lo, x_hi = buffer, nx - buffer
    zone = (x_hi - x_lo) * ny * nz
    count = 0
    while True:
        batch = 64
        for _ in range(batch):
            r = rng.uniform(r_lo, r_hi)
            c = rng.uniform([x_lo, 0.0, 0.0], [x_hi, ny, nz])
            i0, i1 = max(x_lo, int(c[0] - r) - 1), min(x_hi, int(c[0] + r) + 2)
            j0, j1 = max(0, int(c[1] - r) - 1), min(ny, int(c[1] + r) + 2)
            k0, k1 = max(0, int(c[2] - r) - 1), min(nz, int(c[2] + r) + 2)
            zz, yy, xx = np.meshgrid(np.arange(k0, k1) + 0.5, np.arange(j0, j1) + 0.5,
                                     np.arange(i0, i1) + 0.5, indexing="ij")
            solid[k0:k1, j0:j1, i0:i1] |= (xx - c[0]) ** 2 + (yy - c[1]) ** 2 + (zz - c[2]) ** 2 <= r * r
            count += 1
        if 1.0 - solid[:, :, x_lo:x_hi].sum() / zone <= porosity:
            break
    mask = solid.astype(np.uint8)
    bc = [BC_INLET, BC_OUTLET, BC_WALL, BC_WALL, BC_WALL, BC_WALL]
    mask = keep_outlet_connected(mask, bc, 3)
    alpha = np.zeros((nz, ny, nx))
    alpha[:, :, :buffer] = 1.0
    alpha[mask == 1] = 0.0
    sigma = 0.03
    u = inlet_speed(ca, WATER["mu"], sigma)
    dt_vd = cfl * h / u
    n_sub = smallest_substeps(dt_vd, brackbill_limit(WATER["rho"], OIL["rho"], h, sigma))
    return _case("sphere_pack_%d" % n, 3, nx, ny, nz, h, WATER, OIL, sigma, theta, bc, u, mask, alpha,
                 dt_vd, n_sub, min(max_iters, n_sub), tol, ca=ca, seed=seed, spheres=count)


def serving_requests(n=64, seed=4):
    """The batched-serving mix: n requests, each a 2D channel bubble or a 2D
    micromodel, grid Nx = 128 + 32 round(12 s), Ny = 32 + 32 round(7 s) with
    s ~ U[0,1], Ca log-uniform in [1e-6, 1e-3], exponential inter-arrival
    gaps of unit mean (scaled by the caller)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    reqs = []
    for r in range(n):
        s = rng.uniform()
        nx = 128 + 32 * int(round(12 * s))
        ny = 32 + 32 * int(round(7 * s))
        ca = 10.0 ** rng.uniform(-6.0, -3.0)
        kind = "channel" if rng.uniform() < 0.5 else "micromodel"
        gap = rng.exponential(1.0)
        if kind == "channel":
            c = channel_bubble(nx=nx, ny=ny, h=1e-6, ca=ca, cfl=0.1, n_sub=None, tol=1e-4)
            c["max_iters"] = min(200, c["n_sub"])
        else:
            rs = ny / 512.0 * 20.0
            c = micromodel(nx=nx, ny=ny, h=30e-6, ca=ca, cfl=0.1, seed=1000 + r,
                           r_lo=max(4.0, 0.4 * rs), r_hi=max(6.0, rs), gap=2.0,
                           inlet_cols=8, buffer=16, max_iters=200, tol=1e-4)
        c["request"] = r
        c["kind"] = kind
        c["arrival_gap"] = gap
        reqs.append(c)
    return reqs


def tiny_box(nx=8, ny=6, nz=1, dim=2, seed=0, solid_cells=((3, 2, 0),), bc=None, theta=60.0,
             sigma=0.05, h=1e-5):
    """A small random state for direct-solve and kernel parity checks."""
    rng = np.random.Generator(np.random.PCG64(seed))
    mask = np.zeros((nz, ny, nx), dtype=np.uint8)
    for (i, j, k) in solid_cells:
        mask[k, j, i] = 1
    if bc is None:
        bc = [BC_INLET, BC_OUTLET, BC_WALL, BC_WALL, BC_WALL, BC_WALL]
    alpha = rng.uniform(0.0, 1.0, size=(nz, ny, nx))
    alpha[mask == 1] = 0.0
    c = _case("tiny_%dx%dx%d" % (nx, ny, nz), dim, nx, ny, nz, h, WATER, OIL, sigma, theta, bc, 1e-3,
              mask, alpha, 1e-4, 4, 4, 1e-4)
    return c


def random_fields(case, seed=1, u_scale=1e-3, p_scale=1.0):
    """Random velocity, pressure and face-flux fields with the case's layout,
    for injected-state checks (solid cells and faces next to solids are
    zeroed by the caller's own face masks when needed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    d, nx, ny, nz = case["dim"], case["nx"], case["ny"], case["nz"]
    nc = nx * ny * nz
    nf = (nx + 1) * ny * nz + nx * (ny + 1) * nz + (nx * ny * (nz + 1) if d == 3 else 0)
    solid = case["mask"].astype(bool)
    U = rng.uniform(-u_scale, u_scale, size=(d, nc))
    U[:, solid] = 0.0
    p = rng.uniform(-p_scale, p_scale, size=nc)
    p[solid] = 0.0
    phi = rng.uniform(-u_scale, u_scale, size=nf) * case["h"] ** (d - 1)
    return dict(U=U.reshape(-1), p=p, phi=phi)


def fp32_ulp_perturbed(alpha, seed=0):
    """alpha with every partial cell (0 < alpha < 1) moved by one FP32 unit
    in the last place, up or down at random (seeded): an input perturbation
    of the size of FP32 storage, for sensitivity yardsticks."""
    rng = np.random.Generator(np.random.PCG64(seed))
    a32 = alpha.astype(np.float32)
    up = np.nextafter(a32, np.float32(2.0))
    dn = np.nextafter(a32, np.float32(-1.0))
    pick = rng.uniform(size=alpha.shape) < 0.5
    out = np.where(pick, up, dn).astype(np.float64)
    part = (alpha > 0.0) & (alpha < 1.0)
    return np.where(part, out, alpha)


CONFIGS = {
    "c1": channel_bubble,
    "c2": constricted_channel,
    "c3": micromodel,
    "c5": sphere_pack,
}
