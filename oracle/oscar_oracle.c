/*
 * OSCAR FP64 CPU oracle -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg load
 * this library.  It shares no code with the GPU library.
 *
 * Paper: J. Maes, H. P. Menke, "GeoChemFoam: Operator Splitting based
 * time-stepping for efficient Volume-Of-Fluid simulation of
 * capillary-dominated two-phase flow", arXiv 2105.10576.
 *
 * Everything is double precision, sequential, one loop per step of the
 * method, in the order the paper gives them.  The discretisation of the
 * operators the paper names but does not spell out (van Leer with interface
 * compression and a bounded explicit flux limiter for alpha, linear upwind
 * convection, the Gauss-linear gradients, the PISO pressure equation, the
 * Jacobi-preconditioned conjugate gradient) follows the published methods
 * named in the function comments; every reading of a silent or garbled
 * passage is listed in the design notes of the repository.
 *
 * Build: gcc -O2 -std=c99 -ffp-contract=off -fPIC -shared (no fused
 * multiply-add, so every expression rounds once per operation).
 *
 * Pins: the tests under tests/test_oracle_*.py check this file against
 * closed forms, conservation laws, a dense direct solve, the static-drop
 * Laplace jump, Poiseuille flow and symmetry (see each test's docstring).
 */
#include "oscar_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define F_NONE 0
#define F_INT 1
#define F_WALL 2
#define F_INLET 3
#define F_OUTLET 4

#define ORC_OK 0
#define ORC_W_PCG_MAXIT 1
#define ORC_E_ARG (-1)
#define ORC_E_UNSTABLE (-4)
#define ORC_E_NONFINITE (-5)

struct orc {
  orc_params prm;
  int d;                 /* dimension */
  int mules_iter;        /* limiting passes of the alpha transport */
  long nx, ny, nz, nc;   /* cells */
  long nf[3];            /* faces per direction */
  long nftot;
  double V, S, Sh, S2h, hh, delta, cos_t, sin_t;
  uint8_t *solid;
  long n_fluid;
  double *alpha, *alpha_old;
  double *U_vd, *U_cr, *U_sum, *U;  /* d*nc, component-major */
  double *p_vd, *p_cr, *p;
  double *phi_vd, *phi_vd_prev, *phi_cr;   /* nftot */
  double *kappa, *nhatf;                   /* nc, nftot */
  /* work arrays */
  double *grad;      /* d*nc gradient of alpha */
  double *gradU;     /* d*d*nc, gradU[(c*d+e)*nc + P] = dU_c/dx_e */
  double *Fmass;     /* nftot momentum mass flux */
  double *phic;      /* nftot convecting volumetric flux */
  double *aP, *rAU, *b;   /* nc, nc, d*nc */
  double *HbyA;      /* d*nc */
  double *phiH;      /* nftot */
  double *rhs, *invD, *r, *z, *dvec, *q, *tmp, *tmp2;   /* nc */
  double *FL, *Aflux, *Rp, *Rm;   /* nftot, nftot, nc, nc */
  double *lam;                    /* nftot: face limiter of the last pass */
  orc_stats_t st;
};

/* ------------------------------------------------------------------------ */
/* Grid and boundary classification                                          */
/* ------------------------------------------------------------------------ */

static long cidx(const orc_t *o, long i, long j, long k) { return i + o->nx * (j + o->ny * k); }

/* face of direction e whose high-side cell is (i,j,k); coordinate along e in [0, n_e] */
static long fidx(const orc_t *o, int e, long i, long j, long k) {
  if (e == 0) return i + (o->nx + 1) * (j + o->ny * k);
  if (e == 1) return o->nf[0] + i + o->nx * (j + (o->ny + 1) * k);
  return o->nf[0] + o->nf[1] + i + o->nx * (j + o->ny * k);
}

static int in_box(const orc_t *o, long i, long j, long k) {
  return i >= 0 && i < o->nx && j >= 0 && j < o->ny && k >= 0 && k < o->nz;
}

static int bc_type(int bc) {
  if (bc == ORC_BC_INLET) return F_INLET;
  if (bc == ORC_BC_OUTLET) return F_OUTLET;
  return F_WALL;
}

/* The face f (0..5 = x-, x+, y-, y+, z-, z+) of fluid cell (i,j,k):
 * type, neighbour cell (INT only), face array index, direction, and the
 * sign s = +1 when the face's +e orientation points out of the cell. */
typedef struct { int type; long nb; long fi; int e; double s; } cface;

static cface cell_face(const orc_t *o, long i, long j, long k, int f) {
  cface c;
  int e = f >> 1, hi = f & 1;
  long ii = i, jj = j, kk = k;
  c.e = e;
  c.s = hi ? 1.0 : -1.0;
  c.nb = -1;
  if (e >= o->d) { c.type = F_NONE; c.fi = -1; return c; }
  if (e == 0) ii += hi ? 1 : -1;
  if (e == 1) jj += hi ? 1 : -1;
  if (e == 2) kk += hi ? 1 : -1;
  c.fi = hi ? fidx(o, e, ii, jj, kk) : fidx(o, e, i, j, k);
  if (!in_box(o, ii, jj, kk)) { c.type = bc_type(o->prm.bc[f]); return c; }
  long n = cidx(o, ii, jj, kk);
  if (o->solid[n]) { c.type = F_WALL; return c; }
  c.type = F_INT;
  c.nb = n;
  return c;
}

/* Face-centred view of the face of direction e whose high-side cell is (i,j,k):
 * lo/hi cells (-1 outside the box), its type, and which side is the fluid one
 * for WALL/INLET/OUTLET faces (s_fluid = orientation sign seen from the fluid cell). */
typedef struct { int type; long lo, hi, P; double s_fluid; } fface;

static fface face_view(const orc_t *o, int e, long i, long j, long k) {
  fface v;
  long li = i - (e == 0), lj = j - (e == 1), lk = k - (e == 2);
  int loin = in_box(o, li, lj, lk), hiin = in_box(o, i, j, k);
  v.lo = loin ? cidx(o, li, lj, lk) : -1;
  v.hi = hiin ? cidx(o, i, j, k) : -1;
  v.P = -1;
  v.s_fluid = 0.0;
  v.type = F_NONE;
  int lof = loin && !o->solid[v.lo];
  int hif = hiin && !o->solid[v.hi];
  if (lof && hif) { v.type = F_INT; return v; }
  if (!lof && !hif) return v;
  if (lof) { v.P = v.lo; v.s_fluid = 1.0; } else { v.P = v.hi; v.s_fluid = -1.0; }
  if (loin && hiin) { v.type = F_WALL; return v; }
  /* box boundary: low boundary of direction e is side 2e, high is 2e+1 */
  v.type = bc_type(o->prm.bc[2 * e + (lof ? 1 : 0)]);
  return v;
}

/* iterate over every face of direction e: calls body with (fi, view) */
#define FOR_FACES(o, e, fi, v)                                                  \
  for (long _k = 0; _k < (o)->nz + ((e) == 2); ++_k)                            \
    for (long _j = 0; _j < (o)->ny + ((e) == 1); ++_j)                          \
      for (long _i = 0; _i < (o)->nx + ((e) == 0); ++_i)                        \
        for (int _once = 1; _once; _once = 0)                                   \
          for (long fi = fidx((o), (e), _i, _j, _k); _once; _once = 0)          \
            for (fface v = face_view((o), (e), _i, _j, _k); _once; _once = 0)

#define FOR_CELLS(o, P, i, j, k)                                                \
  for (long k = 0; k < (o)->nz; ++k)                                            \
    for (long j = 0; j < (o)->ny; ++j)                                          \
      for (long i = 0; i < (o)->nx; ++i)                                        \
        for (long P = cidx((o), i, j, k), _c1 = 1; _c1; _c1 = 0)

/* ------------------------------------------------------------------------ */
/* Mixture properties (Section 2.1).  The printed viscosity line repeats the */
/* density symbols; the viscosity mixture uses mu_1, mu_2.                   */
/* ------------------------------------------------------------------------ */

static double rho_of(const orc_t *o, double a) { return a * o->prm.rho1 + (1.0 - a) * o->prm.rho2; }
static double mu_of(const orc_t *o, double a) { return a * o->prm.mu1 + (1.0 - a) * o->prm.mu2; }

/* ------------------------------------------------------------------------ */
/* Interface normal and curvature (Section 2.1: f = sigma*kappa*grad(alpha), */
/* n = grad(alpha)/|grad(alpha)|; kappa taken as -div(n) so that a drop of   */
/* phase 1 has positive curvature), wall adhesion n.n_wall = cos(theta)      */
/* (boundary conditions of Eq. VOFd / VOFc) in the construction of Brackbill */
/* et al. (1992).                                                            */
/* ------------------------------------------------------------------------ */

/* Gauss-linear cell gradient of alpha; face value = mean of the two cells on
 * interior faces, the cell value on every other face (zero gradient). */
static void alpha_gradient(orc_t *o, const double *a) {
  for (int e = 0; e < o->d; ++e) memset(o->grad + e * o->nc, 0, sizeof(double) * o->nc);
  FOR_CELLS(o, P, i, j, k) {
    if (o->solid[P]) continue;
    for (int e = 0; e < o->d; ++e) {
      cface lo = cell_face(o, i, j, k, 2 * e), hi = cell_face(o, i, j, k, 2 * e + 1);
      double alo = lo.type == F_INT ? 0.5 * (a[P] + a[lo.nb]) : a[P];
      double ahi = hi.type == F_INT ? 0.5 * (a[P] + a[hi.nb]) : a[P];
      o->grad[e * o->nc + P] = (ahi - alo) / o->prm.h;
    }
  }
}

static double vnorm(const double *v, int d) {
  double s = v[0] * v[0] + v[1] * v[1];
  if (d == 3) s = s + v[2] * v[2];
  return sqrt(s);
}

/* e-component of the unit interface normal on every face, from alpha a. */
static void face_normals(orc_t *o, const double *a) {
  alpha_gradient(o, a);
  memset(o->nhatf, 0, sizeof(double) * o->nftot);
  for (int e = 0; e < o->d; ++e) {
    FOR_FACES(o, e, fi, v) {
      double G[3] = {0, 0, 0};
      if (v.type == F_INT) {
        for (int c = 0; c < o->d; ++c)
          G[c] = 0.5 * (o->grad[c * o->nc + v.lo] + o->grad[c * o->nc + v.hi]);
        o->nhatf[fi] = G[e] / (vnorm(G, o->d) + o->delta);
      } else if (v.type == F_INLET || v.type == F_OUTLET) {
        for (int c = 0; c < o->d; ++c) G[c] = o->grad[c * o->nc + v.P];
        o->nhatf[fi] = G[e] / (vnorm(G, o->d) + o->delta);
      } else if (v.type == F_WALL) {
        /* Wall adhesion: the wall condition n.n_w = cos(theta) fixes the
         * wall-normal component of the unit interface normal at the wall
         * face (the tangential part of the Brackbill construction has no
         * component along the face normal).  It is scaled by the same
         * regularisation |g|/(|g| + delta) as the interior normals, so it
         * fades out continuously away from an interface. */
        double g[3] = {0, 0, 0};
        for (int c = 0; c < o->d; ++c) g[c] = o->grad[c * o->nc + v.P];
        double mg = vnorm(g, o->d);
        double nw = v.s_fluid;   /* n_w . e: from the fluid into the wall */
        o->nhatf[fi] = (mg / (mg + o->delta)) * (o->cos_t * nw);
      }
    }
  }
}

/* kappa_P = -(1/V) sum_f s_f nhat_f . S_f = -(1/h) sum_e (n_{e+} - n_{e-}) */
static void curvature(orc_t *o) {
  face_normals(o, o->alpha);
  memset(o->kappa, 0, sizeof(double) * o->nc);
  FOR_CELLS(o, P, i, j, k) {
    if (o->solid[P]) continue;
    double acc = 0.0;
    for (int e = 0; e < o->d; ++e) {
      cface lo = cell_face(o, i, j, k, 2 * e), hi = cell_face(o, i, j, k, 2 * e + 1);
      acc = acc + (o->nhatf[hi.fi] - o->nhatf[lo.fi]);
    }
    o->kappa[P] = -acc / o->prm.h;
  }
}

/* Surface-tension face term sigma*kappa_f*snGrad(alpha) on interior faces
 * (continuum surface force, balanced-force face form). */
static double st_face(const orc_t *o, long lo, long hi) {
  return (o->prm.sigma * (0.5 * (o->kappa[lo] + o->kappa[hi]))) * ((o->alpha[hi] - o->alpha[lo]) / o->prm.h);
}

/* ------------------------------------------------------------------------ */
/* Explicit alpha transport (Eq. alphaExp, Eq. VOFd, Eq. VOFc): upwind flux   */
/* plus a van Leer (1974) high-order flux with interface compression,        */
/* blended by a Zalesak (1979) flux-corrected-transport limiter that keeps   */
/* alpha inside local [0,1]-clipped bounds.  With mules_iter = M > 1 the     */
/* limiting is iterated (iterative flux correction: Schaer & Smolarkiewicz   */
/* 1996; Kuzmin & Moeller 2005): pass m limits the antidiffusive flux that   */
/* the passes before it left unused, (1 - lambda) A, against the same local  */
/* bounds, starting from the state the previous pass produced.               */
/* ------------------------------------------------------------------------ */

/* one further limiting pass: cur holds the state after the previous pass,
 * o->Aflux the antidiffusive flux still unused, o->lam the previous face
 * limiter; the new state goes to nxt */
static void limit_again(orc_t *o, double dtV, double Vdt, const double *cur, double *nxt) {
  const double *ab = o->alpha_old;   /* the bounds are those of the first pass */
  for (long fi = 0; fi < o->nftot; ++fi) o->Aflux[fi] = (1.0 - o->lam[fi]) * o->Aflux[fi];
  FOR_CELLS(o, P, i, j, k) {
    o->Rp[P] = 0.0;
    o->Rm[P] = 0.0;
    if (o->solid[P]) continue;
    double Pp = 0.0, Pm = 0.0, amax = ab[P], amin = ab[P];
    for (int f = 0; f < 2 * o->d; ++f) {
      cface c = cell_face(o, i, j, k, f);
      if (c.type != F_INT) continue;   /* only interior faces carry antidiffusive flux */
      double sA = c.s * o->Aflux[c.fi];
      Pp = Pp + (sA < 0.0 ? -sA : 0.0);
      Pm = Pm + (sA > 0.0 ? sA : 0.0);
      if (ab[c.nb] > amax) amax = ab[c.nb];
      if (ab[c.nb] < amin) amin = ab[c.nb];
    }
    if (amax > 1.0) amax = 1.0;
    if (amin < 0.0) amin = 0.0;
    double Qp = Vdt * (amax - cur[P] > 0.0 ? amax - cur[P] : 0.0);
    double Qm = Vdt * (cur[P] - amin > 0.0 ? cur[P] - amin : 0.0);
    o->Rp[P] = Pp > 0.0 ? (Qp / Pp < 1.0 ? Qp / Pp : 1.0) : 0.0;
    o->Rm[P] = Pm > 0.0 ? (Qm / Pm < 1.0 ? Qm / Pm : 1.0) : 0.0;
  }
  FOR_CELLS(o, P, i, j, k) {
    if (o->solid[P]) continue;
    double acc = 0.0;
    for (int f = 0; f < 2 * o->d; ++f) {
      cface c = cell_face(o, i, j, k, f);
      if (c.type != F_INT) continue;
      long lo = c.s > 0.0 ? P : c.nb, hi = c.s > 0.0 ? c.nb : P;
      double Af = o->Aflux[c.fi];
      double x1 = Af >= 0.0 ? o->Rm[lo] : o->Rp[lo];
      double x2 = Af >= 0.0 ? o->Rp[hi] : o->Rm[hi];
      double lam = x1 < x2 ? x1 : x2;
      o->lam[c.fi] = lam;
      acc = acc + c.s * (lam * Af);
    }
    nxt[P] = cur[P] - dtV * acc;
  }
}

static int advect(orc_t *o, const double *phi, double dt) {
  const double dtV = dt / o->V, Vdt = o->V / dt;
  double *a = o->alpha;
  memcpy(o->alpha_old, a, sizeof(double) * o->nc);
  /* compression needs the interface normal of the alpha being transported */
  face_normals(o, a);

  /* Courant number: outgoing volumetric flux of each cell times dt/V */
  double comax = 0.0;
  FOR_CELLS(o, P, i, j, k) {
    if (o->solid[P]) continue;
    double acc = 0.0;
    for (int f = 0; f < 2 * o->d; ++f) {
      cface c = cell_face(o, i, j, k, f);
      if (c.type == F_NONE) continue;
      double sp = c.s * phi[c.fi];
      if (sp > 0.0) acc = acc + sp;
    }
    double co = acc * dtV;
    if (co > comax) comax = co;
  }
  o->st.max_courant = comax;

  /* face fluxes: low-order F_L and antidiffusive A = F_H - F_L */
  for (int e = 0; e < o->d; ++e) {
    FOR_FACES(o, e, fi, v) {
      double FLv = 0.0, Av = 0.0, ph = phi[fi];
      if (v.type == F_INT) {
        long C = ph >= 0.0 ? v.lo : v.hi;
        long D = ph >= 0.0 ? v.hi : v.lo;
        /* cell beyond C on the line through D, C */
        long ci = C % o->nx, cj = (C / o->nx) % o->ny, ck = C / (o->nx * o->ny);
        int step = ph >= 0.0 ? -1 : 1;
        long ui = ci + (e == 0 ? step : 0), uj = cj + (e == 1 ? step : 0), uk = ck + (e == 2 ? step : 0);
        double aUU = a[C];
        if (in_box(o, ui, uj, uk) && !o->solid[cidx(o, ui, uj, uk)]) aUU = a[cidx(o, ui, uj, uk)];
        double dD = a[D] - a[C], dU = a[C] - aUU;
        double avl = a[C] + (dU * dD > 0.0 ? (dU * dD) / (dU + dD) : 0.0);
        double abar = 0.5 * (a[v.lo] + a[v.hi]);
        double phir = fabs(ph) * o->nhatf[fi];          /* compression coefficient 1 */
        double Fc = (phir * abar) * (1.0 - abar);
        double FH = ph * avl + Fc;
        FLv = ph * a[C];
        Av = FH - FLv;
      } else if (v.type == F_INLET || v.type == F_OUTLET) {
        FLv = ph * a[v.P];   /* zero-gradient alpha on open boundaries */
      }
      o->FL[fi] = FLv;
      o->Aflux[fi] = Av;
    }
  }

  /* Zalesak limiter: P+, P-, Q+, Q-, R+, R- per cell */
  FOR_CELLS(o, P, i, j, k) {
    o->Rp[P] = 0.0;
    o->Rm[P] = 0.0;
    if (o->solid[P]) continue;
    double sumL = 0.0, Pp = 0.0, Pm = 0.0, amax = a[P], amin = a[P];
    for (int f = 0; f < 2 * o->d; ++f) {
      cface c = cell_face(o, i, j, k, f);
      if (c.type == F_NONE) continue;
      sumL = sumL + c.s * o->FL[c.fi];
      double sA = c.s * o->Aflux[c.fi];
      Pp = Pp + (sA < 0.0 ? -sA : 0.0);
      Pm = Pm + (sA > 0.0 ? sA : 0.0);
      if (c.type == F_INT) {
        if (a[c.nb] > amax) amax = a[c.nb];
        if (a[c.nb] < amin) amin = a[c.nb];
      }
    }
    double aL = a[P] - dtV * sumL;
    if (amax > 1.0) amax = 1.0;
    if (amin < 0.0) amin = 0.0;
    double Qp = Vdt * (amax - aL > 0.0 ? amax - aL : 0.0);
    double Qm = Vdt * (aL - amin > 0.0 ? aL - amin : 0.0);
    o->Rp[P] = Pp > 0.0 ? (Qp / Pp < 1.0 ? Qp / Pp : 1.0) : 0.0;
    o->Rm[P] = Pm > 0.0 ? (Qm / Pm < 1.0 ? Qm / Pm : 1.0) : 0.0;
  }

  /* limited update */
  double bflux = 0.0, m0 = 0.0, m1 = 0.0;
  FOR_CELLS(o, P, i, j, k) {
    if (o->solid[P]) continue;
    double acc = 0.0;
    for (int f = 0; f < 2 * o->d; ++f) {
      cface c = cell_face(o, i, j, k, f);
      if (c.type == F_NONE) continue;
      double lam = 0.0;
      if (c.type == F_INT) {
        long lo = c.s > 0.0 ? P : c.nb, hi = c.s > 0.0 ? c.nb : P;
        double Af = o->Aflux[c.fi];
        double x1 = Af >= 0.0 ? o->Rm[lo] : o->Rp[lo];
        double x2 = Af >= 0.0 ? o->Rp[hi] : o->Rm[hi];
        lam = x1 < x2 ? x1 : x2;
      } else {
        bflux = bflux + c.s * o->FL[c.fi];
      }
      o->lam[c.fi] = lam;
      acc = acc + c.s * (o->FL[c.fi] + lam * o->Aflux[c.fi]);
    }
    o->tmp[P] = a[P] - dtV * acc;
  }
  for (int m = 2; m <= o->mules_iter; ++m) {
    limit_again(o, dtV, Vdt, o->tmp, o->tmp2);
    FOR_CELLS(o, P, i, j, k) if (!o->solid[P]) o->tmp[P] = o->tmp2[P];
  }
  FOR_CELLS(o, P, i, j, k) {
    if (o->solid[P]) continue;
    m0 = m0 + a[P];
    a[P] = o->tmp[P];
    m1 = m1 + a[P];
  }
  m0 = m0 * o->V;
  m1 = m1 * o->V;
  double defect = fabs(m1 - m0 + dt * bflux);
  if (defect > o->st.mass_defect) o->st.mass_defect = defect;
  o->st.mass = m1;
  return comax > 1.0 ? ORC_E_UNSTABLE : ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Momentum matrix (Eq. NSE1d / Eq. NSEc): implicit Euler in rho*u, upwind   */
/* convection with the linear-upwind explicit correction, implicit           */
/* mu*grad(u) diffusion and the explicit transpose term mu*(grad u)^T.       */
/* A = diagonal a_P, H = b - sum a_N u_N.                                    */
/* ------------------------------------------------------------------------ */

/* inlet boundary velocity component c of an inlet face of direction e seen
 * from its fluid cell with orientation sign s: inward speed ub */
static double inlet_u(int c, int e, double s, double ub) { return c == e ? -s * ub : 0.0; }

/* Gauss-linear gradient of a vector field: gU[(c*d+e)*nc+P] = dU_c/dx_e */
static void velocity_gradient(orc_t *o, const double *Uo, double ub) {
  const int d = o->d;
  memset(o->gradU, 0, sizeof(double) * d * d * o->nc);
  FOR_CELLS(o, P, i, j, k) {
    if (o->solid[P]) continue;
    for (int e = 0; e < d; ++e) {
      cface lo = cell_face(o, i, j, k, 2 * e), hi = cell_face(o, i, j, k, 2 * e + 1);
      for (int c = 0; c < d; ++c) {
        const double *Uc = Uo + c * o->nc;
        double f[2];
        cface fc[2] = {lo, hi};
        for (int s = 0; s < 2; ++s) {
          cface cf = fc[s];
          if (cf.type == F_INT) f[s] = 0.5 * (Uc[P] + Uc[cf.nb]);
          else if (cf.type == F_WALL) f[s] = 0.0;
          else if (cf.type == F_INLET) f[s] = inlet_u(c, e, cf.s, ub);
          else f[s] = Uc[P];   /* outlet: zero gradient */
        }
        o->gradU[(c * d + e) * o->nc + P] = (f[1] - f[0]) / o->prm.h;
      }
    }
  }
}

static void assemble(orc_t *o, const double *phic, const double *Uo, double ub, double dt) {
  const int d = o->d;
  const long nc = o->nc;
  const double Vdt = o->V / dt;
  const double *an = o->alpha, *ao = o->alpha_old;
  velocity_gradient(o, Uo, ub);
  /* momentum mass flux on faces: rho of the face-mean alpha (interior), of the
   * boundary cell (inlet/outlet), times the convecting volumetric flux */
  for (int e = 0; e < d; ++e) {
    FOR_FACES(o, e, fi, v) {
      double F = 0.0;
      if (v.type == F_INT) F = rho_of(o, 0.5 * (an[v.lo] + an[v.hi])) * phic[fi];
      else if (v.type == F_INLET || v.type == F_OUTLET) F = rho_of(o, an[v.P]) * phic[fi];
      o->Fmass[fi] = F;
    }
  }
  FOR_CELLS(o, P, i, j, k) {
    o->aP[P] = 0.0;
    o->rAU[P] = 0.0;
    for (int c = 0; c < d; ++c) o->b[c * nc + P] = 0.0;
    if (o->solid[P]) continue;
    double rho_o = rho_of(o, ao[P]), rho_n = rho_of(o, an[P]), mu_n = mu_of(o, an[P]);
    double aP = rho_n * Vdt;
    double b[3];
    for (int c = 0; c < d; ++c) b[c] = (rho_o * Uo[c * nc + P]) * Vdt;
    for (int f = 0; f < 2 * d; ++f) {
      cface cf = cell_face(o, i, j, k, f);
      int e = cf.e;
      double s = cf.s;
      if (cf.type == F_INT) {
        double F = o->Fmass[cf.fi], sF = s * F;
        double muf = mu_of(o, 0.5 * (an[P] + an[cf.nb]));
        double D = muf * o->Sh;
        aP = aP + (sF > 0.0 ? sF : 0.0);
        aP = aP + D;
        long lo = s > 0.0 ? P : cf.nb, hi = s > 0.0 ? cf.nb : P;
        for (int c = 0; c < d; ++c) {
          /* linear upwind: U_f = U_C + (x_f - x_C).grad(U_c)_C, explicit part */
          double lu = F >= 0.0 ? o->hh * o->gradU[(c * d + e) * nc + lo]
                               : -(o->hh * o->gradU[(c * d + e) * nc + hi]);
          b[c] = b[c] - s * (F * lu);
          /* transpose viscous term: mu_f (dU_e/dx_c)_f S */
          double tv = (muf * o->S) * (0.5 * (o->gradU[(e * d + c) * nc + P] + o->gradU[(e * d + c) * nc + cf.nb]));
          b[c] = b[c] + s * tv;
        }
      } else if (cf.type == F_WALL) {
        aP = aP + mu_n * o->S2h;
      } else if (cf.type == F_INLET) {
        double F = o->Fmass[cf.fi];
        aP = aP + mu_n * o->S2h;
        for (int c = 0; c < d; ++c) {
          double ubc = inlet_u(c, e, s, ub);
          b[c] = b[c] + (mu_n * o->S2h) * ubc;
          b[c] = b[c] - s * (F * ubc);
        }
      } else if (cf.type == F_OUTLET) {
        aP = aP + s * o->Fmass[cf.fi];
      }
    }
    o->aP[P] = aP;
    o->rAU[P] = o->V / aP;   /* inverse of the diagonal per unit volume */
    for (int c = 0; c < d; ++c) o->b[c * nc + P] = b[c];
  }
}

/* ------------------------------------------------------------------------ */
/* PISO corrector (Issa 1985; Section 2.2): u* = H/A (+ the surface-tension  */
/* face term), div(A^-1 grad p) = div(u*), u = u* - A^-1 grad p.             */
/* ------------------------------------------------------------------------ */

static void predictor(orc_t *o, const double *U) {
  const int d = o->d;
  const long nc = o->nc;
  const double *an = o->alpha;
  FOR_CELLS(o, P, i, j, k) {
    for (int c = 0; c < d; ++c) o->HbyA[c * nc + P] = 0.0;
    if (o->solid[P]) continue;
    double H[3];
    for (int c = 0; c < d; ++c) H[c] = o->b[c * nc + P];
    for (int f = 0; f < 2 * d; ++f) {
      cface cf = cell_face(o, i, j, k, f);
      if (cf.type != F_INT) continue;
      double sF = cf.s * o->Fmass[cf.fi];
      double D = mu_of(o, 0.5 * (an[P] + an[cf.nb])) * o->Sh;
      double aN = (sF < 0.0 ? sF : 0.0) - D;
      for (int c = 0; c < d; ++c) H[c] = H[c] - aN * U[c * nc + cf.nb];
    }
    for (int c = 0; c < d; ++c) o->HbyA[c * nc + P] = H[c] / o->aP[P];
  }
}

static void predicted_flux(orc_t *o, double ub, int with_st) {
  const int d = o->d;
  const long nc = o->nc;
  memset(o->phiH, 0, sizeof(double) * o->nftot);
  for (int e = 0; e < d; ++e) {
    FOR_FACES(o, e, fi, v) {
      double ph = 0.0;
      if (v.type == F_INT) {
        ph = (0.5 * (o->HbyA[e * nc + v.lo] + o->HbyA[e * nc + v.hi])) * o->S;
        if (with_st) {
          double rAUf = 0.5 * (o->rAU[v.lo] + o->rAU[v.hi]);
          ph = ph + (rAUf * st_face(o, v.lo, v.hi)) * o->S;
        }
      } else if (v.type == F_INLET) {
        ph = -v.s_fluid * (ub * o->S);
      } else if (v.type == F_OUTLET) {
        ph = o->HbyA[e * nc + v.P] * o->S;
      }
      o->phiH[fi] = ph;
    }
  }
}

/* pressure matrix coefficient of face f of cell P (0 when the face has none) */
static double pcoef(const orc_t *o, long P, const cface *cf) {
  if (cf->type == F_INT) return (0.5 * (o->rAU[P] + o->rAU[cf->nb])) * o->Sh;
  if (cf->type == F_OUTLET) return o->rAU[P] * o->S2h;
  return 0.0;
}

/* y = M x, M the matrix of div(rAU grad p) with p = 0 on outlet faces,
 * sign chosen so that M is symmetric positive definite */
static void matvec(const orc_t *o, const double *x, double *y) {
  FOR_CELLS(o, P, i, j, k) {
    y[P] = 0.0;
    if (o->solid[P]) continue;
    double acc = 0.0;
    for (int f = 0; f < 2 * o->d; ++f) {
      cface cf = cell_face(o, i, j, k, f);
      if (cf.type == F_INT) acc = acc + pcoef(o, P, &cf) * (x[P] - x[cf.nb]);
      else if (cf.type == F_OUTLET) acc = acc + pcoef(o, P, &cf) * x[P];
    }
    y[P] = acc;
  }
}

static void pressure_system(orc_t *o) {
  FOR_CELLS(o, P, i, j, k) {
    o->rhs[P] = 0.0;
    o->invD[P] = 0.0;
    if (o->solid[P]) continue;
    double acc = 0.0, dg = 0.0;
    for (int f = 0; f < 2 * o->d; ++f) {
      cface cf = cell_face(o, i, j, k, f);
      if (cf.type == F_NONE) continue;
      acc = acc + cf.s * o->phiH[cf.fi];
      if (cf.type == F_INT || cf.type == F_OUTLET) dg = dg + pcoef(o, P, &cf);
    }
    o->rhs[P] = -acc;
    o->invD[P] = 1.0 / dg;
  }
}

/* Normalised initial residual of the pressure equation (the "normalised
 * norm" of the relaxation stop rule): sum|b - Mp| / (sum(|Mp - M pbar| +
 * |b - M pbar|) + 1e-20), pbar = mean of p over the fluid cells. */
static double normalised_residual(orc_t *o, const double *p) {
  double psum = 0.0;
  FOR_CELLS(o, P, i, j, k) if (!o->solid[P]) psum = psum + p[P];
  double pbar = psum / (double)o->n_fluid;
  FOR_CELLS(o, P, i, j, k) o->tmp2[P] = o->solid[P] ? 0.0 : pbar;
  matvec(o, p, o->q);
  matvec(o, o->tmp2, o->tmp);
  double num = 0.0, den = 0.0;
  FOR_CELLS(o, P, i, j, k) {
    if (o->solid[P]) continue;
    num = num + fabs(o->rhs[P] - o->q[P]);
    den = den + (fabs(o->q[P] - o->tmp[P]) + fabs(o->rhs[P] - o->tmp[P]));
  }
  return num / (den + 1e-20);
}

static double dot(const orc_t *o, const double *x, const double *y) {
  double s = 0.0;
  for (long P = 0; P < o->nc; ++P)
    if (!o->solid[P]) s = s + x[P] * y[P];
  return s;
}

/* Jacobi-preconditioned conjugate gradient (Hestenes & Stiefel), warm start
 * from x; stops when ||b - Mx||_2 <= rtol ||b||_2. */
static int pcg(orc_t *o, double *x, double rtol, int max_it, int *iters, double *rel) {
  const long nc = o->nc;
  double bn = sqrt(dot(o, o->rhs, o->rhs));
  *iters = 0;
  if (bn == 0.0) {
    for (long P = 0; P < nc; ++P) x[P] = 0.0;
    *rel = 0.0;
    return ORC_OK;
  }
  matvec(o, x, o->q);
  for (long P = 0; P < nc; ++P) o->r[P] = o->solid[P] ? 0.0 : o->rhs[P] - o->q[P];
  double rn = sqrt(dot(o, o->r, o->r));
  if (rn <= rtol * bn) { *rel = rn / bn; return ORC_OK; }
  for (long P = 0; P < nc; ++P) o->z[P] = o->r[P] * o->invD[P];
  double rz = dot(o, o->r, o->z);
  memcpy(o->dvec, o->z, sizeof(double) * nc);
  for (int it = 1; it <= max_it; ++it) {
    matvec(o, o->dvec, o->q);
    double dq = dot(o, o->dvec, o->q);
    double al = rz / dq;
    for (long P = 0; P < nc; ++P) {
      if (o->solid[P]) continue;
      x[P] = x[P] + al * o->dvec[P];
      o->r[P] = o->r[P] - al * o->q[P];
    }
    rn = sqrt(dot(o, o->r, o->r));
    *iters = it;
    if (rn <= rtol * bn) { *rel = rn / bn; return ORC_OK; }
    for (long P = 0; P < nc; ++P) o->z[P] = o->r[P] * o->invD[P];
    double rz1 = dot(o, o->r, o->z);
    double be = rz1 / rz;
    rz = rz1;
    for (long P = 0; P < nc; ++P) o->dvec[P] = o->z[P] + be * o->dvec[P];
  }
  *rel = rn / bn;
  return ORC_W_PCG_MAXIT;
}

/* true relative residual ||b - Mx|| / ||b|| */
static double true_residual(orc_t *o, const double *x) {
  double bn = sqrt(dot(o, o->rhs, o->rhs));
  matvec(o, x, o->q);
  double s = 0.0;
  for (long P = 0; P < o->nc; ++P) {
    if (o->solid[P]) continue;
    double r = o->rhs[P] - o->q[P];
    s = s + r * r;
  }
  return bn == 0.0 ? 0.0 : sqrt(s) / bn;
}

static void correct(orc_t *o, double *U, double *phi, const double *p, int with_st) {
  const int d = o->d;
  const long nc = o->nc;
  for (int e = 0; e < d; ++e) {
    FOR_FACES(o, e, fi, v) {
      double ph = o->phiH[fi];
      if (v.type == F_INT) {
        double c = (0.5 * (o->rAU[v.lo] + o->rAU[v.hi])) * o->Sh;
        ph = ph - c * (p[v.hi] - p[v.lo]);
      } else if (v.type == F_OUTLET) {
        double c = o->rAU[v.P] * o->S2h;
        ph = ph + v.s_fluid * (c * p[v.P]);
      }
      phi[fi] = ph;
    }
  }
  /* cell velocity from the face accelerations (f - grad p) in +e orientation */
  FOR_CELLS(o, P, i, j, k) {
    if (o->solid[P]) { for (int c = 0; c < d; ++c) U[c * nc + P] = 0.0; continue; }
    for (int c = 0; c < d; ++c) {
      double q[2];
      for (int side = 0; side < 2; ++side) {
        cface cf = cell_face(o, i, j, k, 2 * c + side);
        double qq = 0.0;
        if (cf.type == F_INT) {
          long lo = side ? P : cf.nb, hi = side ? cf.nb : P;
          double ff = with_st ? st_face(o, lo, hi) : 0.0;
          qq = ff - (p[hi] - p[lo]) / o->prm.h;
        } else if (cf.type == F_OUTLET) {
          double pplus = side ? 0.0 : p[P], pminus = side ? p[P] : 0.0;
          qq = -(pplus - pminus) / o->hh;
        }
        q[side] = qq;
      }
      U[c * nc + P] = o->HbyA[c * nc + P] + o->rAU[P] * (0.5 * (q[0] + q[1]));
    }
  }
}

/* one PISO corrector; E (if not NULL) receives the normalised initial residual */
static int piso_corrector(orc_t *o, double *U, double *phi, double *p, double ub, int with_st, double *E) {
  predictor(o, U);
  predicted_flux(o, ub, with_st);
  pressure_system(o);
  if (E) *E = normalised_residual(o, p);
  int it;
  double rel;
  int rc = pcg(o, p, o->prm.pcg_rtol, o->prm.pcg_max_it, &it, &rel);
  o->st.last_pcg_iters = it;
  o->st.pcg_iters_step += it;
  o->st.last_res = rel;
  if (rc == ORC_W_PCG_MAXIT) o->st.pcg_maxit_hit++;
  correct(o, U, phi, p, with_st);
  return rc;
}

static int all_finite(const orc_t *o) {
  for (long P = 0; P < o->nc; ++P) {
    if (!isfinite(o->alpha[P]) || !isfinite(o->p_vd[P]) || !isfinite(o->p_cr[P])) return 0;
    for (int c = 0; c < o->d; ++c)
      if (!isfinite(o->U_vd[c * o->nc + P]) || !isfinite(o->U_cr[c * o->nc + P])) return 0;
  }
  return 1;
}

/* ------------------------------------------------------------------------ */
/* Viscous-drag step (Section 3.1): alpha* from u_vd^n (Eq. VOFd), then the  */
/* momentum/mass system (Eq. NSE1d, Eq. md) by PISO with the inlet velocity, */
/* convected by u_vd^n + u_cr^n, no surface tension.                         */
/* ------------------------------------------------------------------------ */

int32_t orc_viscous_step(orc_t *o, double dt) {
  if (!(dt > 0.0)) return ORC_E_ARG;
  int rc = ORC_OK, warn = ORC_OK;
  o->st.pcg_iters_step = 0;
  memcpy(o->phi_vd_prev, o->phi_vd, sizeof(double) * o->nftot);
  if (advect(o, o->phi_vd_prev, dt) != ORC_OK) rc = ORC_E_UNSTABLE;
  for (long f = 0; f < o->nftot; ++f) o->phic[f] = o->phi_vd_prev[f] + o->phi_cr[f];
  assemble(o, o->phic, o->U_vd, o->prm.u_inlet, dt);
  for (int j = 0; j < o->prm.n_corr; ++j)
    if (piso_corrector(o, o->U_vd, o->phi_vd, o->p_vd, o->prm.u_inlet, 0, NULL) != ORC_OK) warn = ORC_W_PCG_MAXIT;
  if (!all_finite(o)) return ORC_E_NONFINITE;
  return rc != ORC_OK ? rc : warn;
}

/* ------------------------------------------------------------------------ */
/* Capillary relaxation (Section 3.2): N sub-steps of dt/N below the         */
/* Brackbill limit; each advances alpha** with u_cr (Eq. VOFc), recomputes   */
/* the surface tension from it, and solves Eq. NSEc / Eq. mc by PISO; E_k is */
/* the normalised initial residual of the first corrector; stop after the   */
/* sub-step whose E_k < tol or after max_iters sub-steps; then               */
/* U = U_vd + (1/N) sum_k u_cr^k and p = p_vd + p_cr.                         */
/* ------------------------------------------------------------------------ */

double orc_dt_brackbill(double rho1, double rho2, double h, double sigma) {
  const double pi = 3.14159265358979323846;
  double rbar = 0.5 * (rho1 + rho2);
  return sqrt(rbar * h * h * h / (2.0 * pi * sigma));
}
double orc_dt_cfl(double h, double u) { return h / u; }
double orc_velocity_from_ca(double ca, double mu, double sigma) { return ca * sigma / mu; }

int32_t orc_capillary_relax(orc_t *o, double dt_vd, int32_t n_sub, int32_t max_iters, double tol,
                            int32_t *k_f, double *E_hist) {
  if (!(dt_vd > 0.0) || n_sub < 1 || max_iters < 1 || max_iters > n_sub) return ORC_E_ARG;
  const int d = o->d;
  const long nc = o->nc;
  double dt = dt_vd / (double)n_sub;
  if (o->prm.sigma > 0.0 && !(dt < orc_dt_brackbill(o->prm.rho1, o->prm.rho2, o->prm.h, o->prm.sigma)))
    return ORC_E_UNSTABLE;
  int rc = ORC_OK, warn = ORC_OK;
  o->st.pcg_iters_step = 0;
  for (long x = 0; x < d * nc; ++x) o->U_sum[x] = 0.0;
  int k, kf = max_iters;
  for (k = 0; k < max_iters; ++k) {
    if (advect(o, o->phi_cr, dt) != ORC_OK) rc = ORC_E_UNSTABLE;
    curvature(o);
    for (long f = 0; f < o->nftot; ++f) o->phic[f] = o->phi_vd_prev[f] + o->phi_cr[f];
    assemble(o, o->phic, o->U_cr, 0.0, dt);
    double E = 0.0;
    for (int j = 0; j < o->prm.n_corr; ++j)
      if (piso_corrector(o, o->U_cr, o->phi_cr, o->p_cr, 0.0, 1, j == 0 ? &E : NULL) != ORC_OK)
        warn = ORC_W_PCG_MAXIT;
    if (E_hist) E_hist[k] = E;
    o->st.last_E = E;
    for (long x = 0; x < d * nc; ++x) o->U_sum[x] = o->U_sum[x] + o->U_cr[x];
    if (E < tol) { kf = k + 1; break; }
  }
  for (long x = 0; x < d * nc; ++x) o->U[x] = o->U_vd[x] + o->U_sum[x] / (double)n_sub;
  for (long x = 0; x < nc; ++x) o->p[x] = o->p_vd[x] + o->p_cr[x];
  o->st.k_f = kf;
  if (k_f) *k_f = kf;
  if (!all_finite(o)) return ORC_E_NONFINITE;
  return rc != ORC_OK ? rc : warn;
}

/* Assemble the pressure equation of a viscous (which = 0) or capillary
 * (which = 1) step from the current state without moving alpha, and solve it
 * for p_vd or p_cr.  Velocities and fluxes are left untouched. */
int32_t orc_pressure_solve(orc_t *o, int32_t which, double dt, double rtol, int32_t max_it,
                           int32_t *iters, double *rel_res) {
  if (!(dt > 0.0) || (which != 0 && which != 1)) return ORC_E_ARG;
  memcpy(o->alpha_old, o->alpha, sizeof(double) * o->nc);
  double *U = which ? o->U_cr : o->U_vd, *p = which ? o->p_cr : o->p_vd;
  double ub = which ? 0.0 : o->prm.u_inlet;
  /* a viscous step convects with u_vd^n: keep it as the previous flux */
  if (!which) memcpy(o->phi_vd_prev, o->phi_vd, sizeof(double) * o->nftot);
  const double *phiv = o->phi_vd_prev;
  if (which) curvature(o);
  for (long f = 0; f < o->nftot; ++f) o->phic[f] = phiv[f] + o->phi_cr[f];
  assemble(o, o->phic, U, ub, dt);
  predictor(o, U);
  predicted_flux(o, ub, which);
  pressure_system(o);
  int it;
  double rel;
  int rc = pcg(o, p, rtol, max_it, &it, &rel);
  if (iters) *iters = it;
  if (rel_res) *rel_res = true_residual(o, p);
  return rc;
}

/* Dense Gaussian elimination with partial pivoting of the last assembled
 * pressure system (M, rhs) over the fluid cells. */
int32_t orc_dense_solve(orc_t *o, double *p_out) {
  long n = o->n_fluid;
  if (n > 4000) return ORC_E_ARG;
  long *id = (long *)malloc(sizeof(long) * o->nc);
  long *cell = (long *)malloc(sizeof(long) * n);
  double *A = (double *)calloc((size_t)n * n, sizeof(double));
  double *bb = (double *)malloc(sizeof(double) * n);
  long m = 0;
  for (long P = 0; P < o->nc; ++P) { id[P] = o->solid[P] ? -1 : m; if (!o->solid[P]) cell[m++] = P; }
  FOR_CELLS(o, P, i, j, k) {
    if (o->solid[P]) continue;
    long r = id[P];
    bb[r] = o->rhs[P];
    for (int f = 0; f < 2 * o->d; ++f) {
      cface cf = cell_face(o, i, j, k, f);
      double c = pcoef(o, P, &cf);
      if (cf.type == F_INT) { A[r * n + r] += c; A[r * n + id[cf.nb]] -= c; }
      else if (cf.type == F_OUTLET) A[r * n + r] += c;
    }
  }
  for (long c = 0; c < n; ++c) {
    long piv = c;
    for (long r = c + 1; r < n; ++r) if (fabs(A[r * n + c]) > fabs(A[piv * n + c])) piv = r;
    if (piv != c) {
      for (long x = 0; x < n; ++x) { double t = A[c * n + x]; A[c * n + x] = A[piv * n + x]; A[piv * n + x] = t; }
      double t = bb[c]; bb[c] = bb[piv]; bb[piv] = t;
    }
    for (long r = c + 1; r < n; ++r) {
      double fct = A[r * n + c] / A[c * n + c];
      if (fct == 0.0) continue;
      for (long x = c; x < n; ++x) A[r * n + x] -= fct * A[c * n + x];
      bb[r] -= fct * bb[c];
    }
  }
  for (long c = n - 1; c >= 0; --c) {
    double s = bb[c];
    for (long x = c + 1; x < n; ++x) s -= A[c * n + x] * bb[x];
    bb[c] = s / A[c * n + c];
  }
  for (long P = 0; P < o->nc; ++P) p_out[P] = 0.0;
  for (long r = 0; r < n; ++r) p_out[cell[r]] = bb[r];
  free(id); free(cell); free(A); free(bb);
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Construction, fields, statistics                                          */
/* ------------------------------------------------------------------------ */

static double *zalloc(long n) { return (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double)); }

orc_t *orc_create(const orc_params *prm, const uint8_t *mask, const double *alpha0) {
  if (!prm || !mask || !alpha0) return NULL;
  if (prm->dim != 2 && prm->dim != 3) return NULL;
  if (prm->nx < 1 || prm->ny < 1 || prm->nz < 1 || (prm->dim == 2 && prm->nz != 1)) return NULL;
  if (!(prm->h > 0.0) || !(prm->rho1 > 0.0) || !(prm->rho2 > 0.0) || !(prm->mu1 > 0.0) || !(prm->mu2 > 0.0) ||
      prm->sigma < 0.0 || prm->n_corr < 1 || prm->mules_iter < 0 || prm->mules_iter > 8)
    return NULL;
  orc_t *o = (orc_t *)calloc(1, sizeof(orc_t));
  o->prm = *prm;
  o->d = prm->dim;
  o->mules_iter = prm->mules_iter > 0 ? prm->mules_iter : 1;
  o->nx = prm->nx; o->ny = prm->ny; o->nz = prm->nz;
  o->nc = o->nx * o->ny * o->nz;
  o->nf[0] = (o->nx + 1) * o->ny * o->nz;
  o->nf[1] = o->nx * (o->ny + 1) * o->nz;
  o->nf[2] = o->d == 3 ? o->nx * o->ny * (o->nz + 1) : 0;
  o->nftot = o->nf[0] + o->nf[1] + o->nf[2];
  double h = prm->h;
  o->V = o->d == 3 ? h * h * h : h * h;
  o->S = o->d == 3 ? h * h : h;
  o->Sh = o->S / h;
  o->hh = 0.5 * h;
  o->S2h = o->S / o->hh;
  o->delta = 1e-8 / h;
  /* cos and sin of theta, written so that 90 degrees gives exactly 0 and 1 */
  const double pi = 3.14159265358979323846;
  double comp = (90.0 - prm->theta_deg) * (pi / 180.0);
  o->cos_t = sin(comp);
  o->sin_t = cos(comp);
  long nc = o->nc, d = o->d, nf = o->nftot;
  o->solid = (uint8_t *)malloc((size_t)nc);
  memcpy(o->solid, mask, (size_t)nc);
  o->alpha = zalloc(nc); o->alpha_old = zalloc(nc);
  o->U_vd = zalloc(d * nc); o->U_cr = zalloc(d * nc); o->U_sum = zalloc(d * nc); o->U = zalloc(d * nc);
  o->p_vd = zalloc(nc); o->p_cr = zalloc(nc); o->p = zalloc(nc);
  o->phi_vd = zalloc(nf); o->phi_vd_prev = zalloc(nf); o->phi_cr = zalloc(nf);
  o->kappa = zalloc(nc); o->nhatf = zalloc(nf);
  o->grad = zalloc(d * nc); o->gradU = zalloc(d * d * nc);
  o->Fmass = zalloc(nf); o->phic = zalloc(nf);
  o->aP = zalloc(nc); o->rAU = zalloc(nc); o->b = zalloc(d * nc);
  o->HbyA = zalloc(d * nc); o->phiH = zalloc(nf);
  o->rhs = zalloc(nc); o->invD = zalloc(nc); o->r = zalloc(nc); o->z = zalloc(nc);
  o->dvec = zalloc(nc); o->q = zalloc(nc); o->tmp = zalloc(nc); o->tmp2 = zalloc(nc);
  o->FL = zalloc(nf); o->Aflux = zalloc(nf); o->Rp = zalloc(nc); o->Rm = zalloc(nc);
  o->lam = zalloc(nf);
  long nfl = 0;
  double m = 0.0;
  for (long P = 0; P < nc; ++P) {
    if (o->solid[P]) continue;
    nfl++;
    o->alpha[P] = alpha0[P];
    m = m + alpha0[P];
  }
  o->n_fluid = nfl;
  o->st.n_fluid = (int32_t)nfl;
  o->st.mass = m * o->V;
  return o;
}

void orc_destroy(orc_t *o) {
  if (!o) return;
  void *ptrs[] = {o->solid, o->alpha, o->alpha_old, o->U_vd, o->U_cr, o->U_sum, o->U, o->p_vd, o->p_cr,
                  o->p, o->phi_vd, o->phi_vd_prev, o->phi_cr, o->kappa, o->nhatf, o->grad, o->gradU,
                  o->Fmass, o->phic, o->aP, o->rAU, o->b, o->HbyA, o->phiH, o->rhs, o->invD, o->r,
                  o->z, o->dvec, o->q, o->tmp, o->tmp2, o->FL, o->Aflux, o->Rp, o->Rm, o->lam};
  for (size_t x = 0; x < sizeof(ptrs) / sizeof(ptrs[0]); ++x) free(ptrs[x]);
  free(o);
}

static double *field_ptr(const orc_t *o, int32_t id, long *len) {
  long nc = o->nc, dn = o->d * o->nc, nf = o->nftot;
  switch (id) {
    case ORC_ALPHA: *len = nc; return o->alpha;
    case ORC_U: *len = dn; return o->U;
    case ORC_P: *len = nc; return o->p;
    case ORC_U_VD: *len = dn; return o->U_vd;
    case ORC_P_VD: *len = nc; return o->p_vd;
    case ORC_U_CR: *len = dn; return o->U_cr;
    case ORC_P_CR: *len = nc; return o->p_cr;
    case ORC_PHI_VD: *len = nf; return o->phi_vd;
    case ORC_PHI_VD_PREV: *len = nf; return o->phi_vd_prev;
    case ORC_PHI_CR: *len = nf; return o->phi_cr;
    case ORC_KAPPA: *len = nc; return o->kappa;
    case ORC_RAU: *len = nc; return o->rAU;
    case ORC_RHS: *len = nc; return o->rhs;
    case ORC_U_SUM: *len = dn; return o->U_sum;
    case ORC_HBYA: *len = dn; return o->HbyA;
    case ORC_NHATF: *len = nf; return o->nhatf;
    default: *len = -1; return NULL;
  }
}

int64_t orc_field_len(const orc_t *o, int32_t id) {
  long len;
  field_ptr(o, id, &len);
  return len;
}

int32_t orc_get_field(const orc_t *o, int32_t id, double *dst) {
  long len;
  double *src = field_ptr(o, id, &len);
  if (!src || !dst) return ORC_E_ARG;
  memcpy(dst, src, sizeof(double) * len);
  return ORC_OK;
}

int32_t orc_set_field(orc_t *o, int32_t id, const double *src) {
  long len;
  double *dst = field_ptr(o, id, &len);
  if (!dst || !src) return ORC_E_ARG;
  memcpy(dst, src, sizeof(double) * len);
  if (id == ORC_ALPHA) {
    double m = 0.0;
    for (long P = 0; P < o->nc; ++P) if (!o->solid[P]) m = m + o->alpha[P];
    o->st.mass = m * o->V;
  }
  return ORC_OK;
}

void orc_get_stats(const orc_t *o, orc_stats_t *s) { *s = o->st; }
