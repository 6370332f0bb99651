/*
 * OSCAR FP64 CPU oracle -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.
 *
 * A plain, slow, sequential double-precision implementation of the OSCAR
 * time-stepping (Maes & Menke, "GeoChemFoam: Operator Splitting based
 * time-stepping for efficient Volume-Of-Fluid simulation of
 * capillary-dominated two-phase flow", arXiv 2105.10576) on a uniform
 * Cartesian voxel grid with a solid mask.  It exists only so that the tests,
 * the smoke check and the benchmark's CPU-baseline leg can check and time the
 * GPU library against an independent implementation.  It shares no code,
 * header, table or constant with the GPU library and the GPU library never
 * calls it.
 *
 * Layout conventions (also used by the arrays passed in and out):
 *   cells  idx = i + nx*(j + ny*k), x fastest; nz = 1 when dim = 2
 *   vector cell fields: component c at [c*ncell + idx], c < dim
 *   face fields: x-faces (nx+1)*ny*nz, then y-faces nx*(ny+1)*nz, then
 *     (3D) z-faces nx*ny*(nz+1); x-face (i,j,k) sits between cells i-1 and i
 *     and is indexed i + (nx+1)*(j + ny*k), likewise for y and z.
 *   face fluxes are oriented along +x, +y, +z.
 */
#ifndef OSCAR_ORACLE_H
#define OSCAR_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_BC_WALL = 0, ORC_BC_INLET = 1, ORC_BC_OUTLET = 2 };

enum {
  ORC_ALPHA = 0, ORC_U = 1, ORC_P = 2, ORC_U_VD = 3, ORC_P_VD = 4,
  ORC_U_CR = 5, ORC_P_CR = 6, ORC_PHI_VD = 7, ORC_PHI_VD_PREV = 8,
  ORC_PHI_CR = 9, ORC_KAPPA = 10, ORC_RAU = 11, ORC_RHS = 12,
  ORC_U_SUM = 13, ORC_HBYA = 14, ORC_NHATF = 15, ORC_NFIELDS = 16
};

typedef struct {
  int32_t dim, nx, ny, nz;
  double h;
  double rho1, mu1, rho2, mu2;  /* phase 1 is alpha = 1 */
  double sigma;
  double theta_deg;             /* contact angle measured through phase 1 */
  int32_t bc[6];                /* x-, x+, y-, y+, z-, z+ */
  double u_inlet;               /* inward normal inlet speed of the viscous step */
  int32_t n_corr;               /* PISO correctors */
  double pcg_rtol;
  int32_t pcg_max_it;
  int32_t mules_iter;           /* limiting passes of the alpha transport, 1..8 (0 = 1) */
} orc_params;

typedef struct {
  double mass;          /* V * sum(alpha) over fluid cells after the last update */
  double max_courant;   /* of the last advection */
  double mass_defect;   /* max |m_after - m_before + dt*B| over all advections */
  double last_E;        /* last normalised residual E_k */
  double last_res;      /* last PCG relative residual (2-norm) */
  int32_t last_pcg_iters;  /* PCG iterations of the last pressure solve */
  int32_t pcg_iters_step;  /* PCG iterations summed over the last step */
  int32_t n_fluid;
  int32_t pcg_maxit_hit;   /* number of solves that hit the iteration cap */
  int32_t k_f;
} orc_stats_t;

typedef struct orc orc_t;

orc_t  *orc_create(const orc_params *prm, const uint8_t *mask, const double *alpha0);
void    orc_destroy(orc_t *o);
int64_t orc_field_len(const orc_t *o, int32_t id);
int32_t orc_get_field(const orc_t *o, int32_t id, double *dst);
int32_t orc_set_field(orc_t *o, int32_t id, const double *src);
int32_t orc_viscous_step(orc_t *o, double dt_vd);
int32_t orc_capillary_relax(orc_t *o, double dt_vd, int32_t n_sub, int32_t max_iters,
                            double tol, int32_t *k_f, double *E_hist);
int32_t orc_pressure_solve(orc_t *o, int32_t which, double dt, double rtol, int32_t max_it,
                           int32_t *iters, double *rel_res);
int32_t orc_dense_solve(orc_t *o, double *p_out);
void    orc_get_stats(const orc_t *o, orc_stats_t *s);
/* closed forms of the paper's stability section */
double  orc_dt_brackbill(double rho1, double rho2, double h, double sigma);
double  orc_dt_cfl(double h, double u);
double  orc_velocity_from_ca(double ca, double mu, double sigma);

#ifdef __cplusplus
}
#endif
#endif
