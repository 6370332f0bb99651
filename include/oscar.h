/*
 * oscar.h -- C ABI of the OSCAR capillary-relaxation library for AMD MI355X
 * (gfx950).
 *
 * OSCAR (Operator Splitting with Capillary Relaxation; J. Maes and
 * H. P. Menke, arXiv 2105.10576) advances an algebraic Volume-Of-Fluid
 * two-phase flow in two operator-split parts (Section 3):
 *   - a viscous-drag step (Section 3.1, Eq. VOFd, NSE1d, md) of length
 *     dt_vd < dt_CFL that transports alpha with u_vd and solves the
 *     momentum/mass system with the inlet velocity and no surface tension;
 *   - N capillary-relaxation sub-steps (Section 3.2, Eq. VOFc, NSEc, mc) of
 *     length dt_vd/N below the Brackbill limit that transport alpha with u_cr
 *     and solve the system with the surface-tension force, stopping early
 *     once the normalised initial pressure residual E_k drops below a
 *     tolerance; the global fields are U = U_vd + (1/N) sum_k u_cr^k and
 *     p = p_vd + p_cr (additive split, Section 3).
 * The problem lives on a uniform Cartesian voxel grid with a solid mask.
 *
 * Conventions
 *   - Every function returns an int32_t status: 0 = OK, > 0 = warning (the
 *     outputs are valid), < 0 = error (see OSCAR_* below).
 *   - Cells are stored x-fastest: idx = i + nx*(j + ny*k); nz = 1 in 2D.
 *   - Vector fields are component-major: component c at [c*ncell + idx].
 *   - Face fields (volumetric fluxes in m^3/s, oriented +x/+y/+z): x-faces
 *     first ((nx+1)*ny*nz, face i between cells i-1 and i, indexed
 *     i + (nx+1)*(j + ny*k)), then y-faces (nx*(ny+1)*nz), then z-faces in 3D.
 *   - Phase 1 is alpha = 1.  Mask value 1 = solid, 0 = fluid.
 *   - Ownership: the caller owns every host array (read or written only
 *     during the call), the device workspace (no field memory is allocated
 *     by the library) and the HIP stream; all device work is ordered on that
 *     stream, and calls that return host values synchronise it.
 *   - One host thread per context at a time.
 *   - After an error the context remains valid for oscar_destroy and
 *     oscar_get_field; fields may be partially advanced.
 */
#ifndef OSCAR_H
#define OSCAR_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define OSCAR_OK 0
#define OSCAR_W_PCG_MAXIT 1        /* a pressure solve hit its iteration cap */
#define OSCAR_W_REFINE_STALL 2     /* mixed precision: FP64 refinement stopped improving above pcg_rtol */
#define OSCAR_E_ARG (-1)           /* bad argument or descriptor */
#define OSCAR_E_WORKSPACE (-2)     /* workspace too small or misaligned */
#define OSCAR_E_MASK (-3)          /* a fluid region cannot reach an outlet */
#define OSCAR_E_UNSTABLE (-4)      /* dt_vd/n_sub >= Brackbill limit, or Courant > 1 */
#define OSCAR_E_NONFINITE (-5)     /* a NaN/Inf appeared in the velocity */
#define OSCAR_E_HIP (-6)           /* a HIP runtime call failed */
#define OSCAR_E_CAPACITY (-7)      /* serving engine: no free slot or memory */

/* boundary type of each box side */
#define OSCAR_BC_WALL 0            /* no-slip, no-flux, contact angle */
#define OSCAR_BC_INLET 1           /* fixed inward velocity u_inlet (viscous step), zero gradient alpha and p */
#define OSCAR_BC_OUTLET 2          /* p = 0, zero-gradient velocity and alpha */

/* arithmetic of the path */
#define OSCAR_FP64 0               /* every field and solve in double precision */
#define OSCAR_MIXED 1              /* FP32 fields, stencils and CG; FP64 pressure, refinement residual, dots, mass sums */

/* preconditioner of the pressure conjugate gradient (oscar_desc.precond) */
#define OSCAR_PC_JACOBI 0          /* diagonal scaling */
#define OSCAR_PC_MG 1              /* one geometric multigrid V-cycle: 2^dim-cell aggregation, Jacobi
                                      smoothing (two sweeps per side on the grid-wide coarse levels in 3D,
                                      one in 2D, unless oscar_desc.mg_sweeps2 says otherwise); coarse
                                      operators rebuilt from 1/a_P at every viscous step and every 4th
                                      capillary sub-step (a preconditioner only: each solve still meets
                                      pcg_rtol on the current operator) */

/* field identifiers for oscar_get_field / oscar_set_field */
#define OSCAR_FIELD_ALPHA 0        /* cells */
#define OSCAR_FIELD_U 1            /* global velocity U_vd + (1/N) sum u_cr (dim*cells) */
#define OSCAR_FIELD_P 2            /* global pressure p_vd + p_cr (cells) */
#define OSCAR_FIELD_U_VD 3
#define OSCAR_FIELD_P_VD 4
#define OSCAR_FIELD_U_CR 5
#define OSCAR_FIELD_P_CR 6
#define OSCAR_FIELD_PHI_VD 7       /* faces */
#define OSCAR_FIELD_PHI_VD_PREV 8  /* faces: u_vd^n of the current global step */
#define OSCAR_FIELD_PHI_CR 9       /* faces */
#define OSCAR_FIELD_KAPPA 10       /* interface curvature of the last capillary sub-step */
#define OSCAR_FIELD_RAU 11         /* V / a_P of the last momentum assembly */
#define OSCAR_FIELD_RHS 12         /* right-hand side of the last pressure equation */
#define OSCAR_FIELD_U_SUM 13       /* sum of u_cr over the last relaxation */
#define OSCAR_FIELD_HBYA 14        /* H / A of the last corrector */
#define OSCAR_FIELD_NHATF 15       /* face-normal component of the interface normal (faces) */

typedef struct oscar_ctx oscar_ctx;

/* How a pressure solve (every CG iteration, multigrid cycle and FP64
 * refinement step of Section 2.2's pressure equation) is executed:
 *   OSCAR_SOLVE_LAUNCHES:   one grid-wide kernel launch per step, enqueued by
 *                           the host in chunks; the host reads the solver
 *                           state back after each chunk;
 *   OSCAR_SOLVE_PERSISTENT: one launch for the whole solve: its workgroups
 *                           take the steps' tiles from a work queue in
 *                           device memory, and the host reads nothing back
 *                           until the sub-step (or viscous step) ends.
 * OSCAR_SOLVE_DEFAULT (0) selects the library's choice. */
#define OSCAR_SOLVE_DEFAULT 0
#define OSCAR_SOLVE_LAUNCHES 1
#define OSCAR_SOLVE_PERSISTENT 2

typedef struct {
  int32_t dim, nx, ny, nz;          /* dim 2 (nz = 1) or 3 */
  double h;                         /* uniform spacing [m], > 0 */
  const uint8_t *mask;              /* host, nx*ny*nz, 1 = solid; read during oscar_create only */
  const double *alpha0;             /* host, nx*ny*nz, initial phase-1 fraction; read during oscar_create only */
  double rho1, mu1, rho2, mu2;      /* densities [kg/m^3] and viscosities [Pa s] of phases 1 and 2, > 0 */
  double sigma;                     /* interfacial tension [N/m], >= 0 */
  double theta_deg;                 /* static contact angle measured through phase 1 */
  int32_t bc[6];                    /* x-, x+, y-, y+, z-, z+ : OSCAR_BC_* (z ignored in 2D) */
  double u_inlet;                   /* inward inlet speed of the viscous step [m/s] */
  int32_t precision;                /* OSCAR_FP64 or OSCAR_MIXED */
  int32_t n_corr;                   /* PISO correctors per step (the paper uses 3), >= 1 */
  double pcg_rtol;                  /* relative 2-norm residual of each pressure solve (mixed: of the FP64 refinement) */
  int32_t pcg_max_it;               /* conjugate-gradient iteration cap per solve */
  int32_t precond;                  /* OSCAR_PC_JACOBI (also the zero value) or OSCAR_PC_MG */
  int32_t mules_iter;               /* limiting passes of the alpha transport, 0..8 (0 and 1: the single
                                       Zalesak limiter).  Pass m > 1 limits the antidiffusive flux the
                                       passes before it left unused, (1 - lambda) A, against the first
                                       pass's local bounds (iterative flux correction); more than one pass
                                       takes one more face array of workspace */
  /* Tuning.  Zero selects the built-in value.  They change the iteration
   * counts or the order of the reductions, so a result is reproducible
   * bit for bit only with the same values. */
  int32_t mg_sweeps2;               /* OSCAR_PC_MG: bit l (l >= 1) gives grid-wide coarse level l two
                                       smoothing sweeps per side instead of one; 0 = built-in rule (every
                                       grid-wide level in 3D, none in 2D); < 0 = one sweep on every level */
  int32_t max_blocks;               /* workgroups per grid-wide launch and instance, 1..1024 (the cells
                                       are grid-strided beyond it; also the number of partials of each
                                       reduction); 0 = 1024 */
  double inner_rtol;                /* OSCAR_MIXED: smallest relative residual reduction asked of one
                                       FP32 inner solve, in (0, 1); 0 = 1e-6 */
  /* Execution (results are bitwise the same either way). */
  int32_t solve_mode;               /* OSCAR_SOLVE_*: how the pressure solves of a context run */
  int32_t reserved;                 /* must be 0 */
} oscar_desc;

typedef struct {
  double mass_phase1;     /* V * sum(alpha) after the last transport (FP64 sum) */
  double max_courant;     /* of the last transport */
  double mass_defect;     /* max |m_after - m_before + dt * boundary outflow| since creation */
  double last_E;          /* E_k of the last capillary sub-step */
  double last_res;        /* last pressure solve: ||b - M p||_2 / ||b||_2 (FP64) */
  int32_t last_pcg_iters; /* conjugate-gradient iterations of the last pressure solve */
  int32_t pcg_iters_call; /* summed over the last viscous step or relaxation */
  int32_t refine_steps_call; /* mixed precision: outer refinement steps over the last call */
  int32_t k_f;            /* completed sub-steps of the last relaxation */
  int32_t n_fluid;
  int32_t pcg_maxit_hits; /* solves that hit the cap since creation */
} oscar_stats_t;

/* Bytes of device workspace a descriptor needs (fields, matrices, solver
 * vectors, reduction scratch), 256-byte aligned sub-arrays.  bytes != NULL. */
int32_t oscar_workspace_size(const oscar_desc *desc, uint64_t *bytes);

/* Create a context on the current HIP device.  dev_workspace: device memory
 * of at least oscar_workspace_size bytes, 256-byte aligned, owned by the
 * caller and kept alive until oscar_destroy.  hip_stream: a hipStream_t (NULL
 * = the default stream).  Validates the descriptor (OSCAR_E_ARG) and the mask:
 * every fluid cell must connect through fluid faces to an outlet face
 * (OSCAR_E_MASK).  Uploads mask and alpha0; zeroes velocities, pressures and
 * fluxes.  On error *out is NULL and oscar_last_error(NULL) explains. */
int32_t oscar_create(const oscar_desc *desc, void *dev_workspace, uint64_t bytes, void *hip_stream,
                     oscar_ctx **out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): oscar_create
 * with the workspace taken from a static device array of the library,
 * OSCAR_STATIC_WORKSPACE_BYTES on each device it runs on (held until the
 * process ends), and the state readback through pageable host memory inside
 * the context.  Neither this call nor the steps, solves, field accesses and
 * oscar_destroy of the context allocate device or pinned memory
 * (oscar_timing does; do not call it on such a context).  One such context
 * per device at a time: OSCAR_E_CAPACITY while another holds the array
 * (oscar_destroy releases it; contexts on one device that overlapped would
 * race on the array).  OSCAR_E_WORKSPACE if oscar_workspace_size exceeds
 * the array.  Otherwise as oscar_create; a new context starts from a
 * cleared workspace, so nothing of an earlier context carries over. */
#define OSCAR_STATIC_WORKSPACE_BYTES (64ull << 20)
int32_t oscar_create_static(const oscar_desc *desc, void *hip_stream, oscar_ctx **out);

/* One viscous-drag step of length dt_vd (Section 3.1): alpha* from u_vd^n
 * (Eq. VOFd), then n_corr PISO correctors of Eq. NSE1d/md convected by
 * u_vd^n + u_cr^n.  OSCAR_E_UNSTABLE if the transport Courant number
 * exceeded 1 (the step is still completed). */
int32_t oscar_viscous_step(oscar_ctx *ctx, double dt_vd);

/* Capillary relaxation of one global step (Section 3.2): up to max_iters
 * (<= n_sub) sub-steps of dt_vd/n_sub; each transports alpha with u_cr
 * (Eq. VOFc), recomputes curvature and surface tension, and runs the PISO
 * correctors of Eq. NSEc/mc convected by u_vd^n + u_cr; E_k is the
 * normalised initial residual of the first corrector's pressure equation;
 * the loop stops after the first sub-step with E_k < tol.  Then
 * U = U_vd + (1/n_sub) sum u_cr and p = p_vd + p_cr.
 * k_f (may be NULL): completed sub-steps; E_last (may be NULL): last E_k.
 * OSCAR_E_UNSTABLE if dt_vd/n_sub >= sqrt(rho_bar h^3 / (2 pi sigma)),
 * rho_bar = (rho1 + rho2)/2 (Section 2.2), before any work is done. */
int32_t oscar_capillary_relax(oscar_ctx *ctx, double dt_vd, int32_t n_sub, int32_t max_iters, double tol,
                              int32_t *k_f, double *E_last);

/* E_k of each sub-step of the last relaxation: writes min(cap, k_f) values. */
int32_t oscar_relax_history(const oscar_ctx *ctx, double *E, int32_t cap, int32_t *n);

/* Assemble the pressure equation of a viscous (which = 0) or capillary
 * (which = 1) step of length dt from the current state, without moving alpha
 * (Section 2.2, PISO: div(A^-1 grad p) = div u*), and solve it for p_vd or
 * p_cr from the current pressure to relative residual rtol (at most max_it
 * iterations).  Velocities and fluxes are left untouched.  iters and
 * rel_residual_fp64 (may be NULL) receive the iteration count and the FP64
 * relative residual ||b - M p|| / ||b||. */
int32_t oscar_pressure_solve(oscar_ctx *ctx, int32_t which, double dt, double rtol, int32_t max_it,
                             int32_t *iters, double *rel_residual_fp64);

/* Copy a field to/from a host array of doubles (length from the layout above). */
int32_t oscar_get_field(oscar_ctx *ctx, int32_t field_id, double *host_dst);
int32_t oscar_set_field(oscar_ctx *ctx, int32_t field_id, const double *host_src);
int64_t oscar_field_len(const oscar_ctx *ctx, int32_t field_id);

int32_t oscar_stats(oscar_ctx *ctx, oscar_stats_t *out);

/* NULL-safe.  Does not free the caller's workspace. */
void oscar_destroy(oscar_ctx *ctx);

/* Message of the last error of ctx, or of the calling thread's last
 * oscar_create / engine failure when ctx is NULL.  Never NULL. */
const char *oscar_last_error(const oscar_ctx *ctx);

/* Measurement hook (not part of the method).  oscar_timing(ctx, period)
 * with period >= 1 resets the totals and samples every period-th
 * conjugate-gradient iteration of each solve (iteration index divisible by
 * period): its kernels stamp the device's constant-rate wall clock at the
 * start and end of every workgroup, and a part's duration is the span from
 * its first workgroup start to its last workgroup end (the kernel execution
 * time, without launch gaps); period = 0 stops.  The first enable allocates
 * 0.5 MiB of device memory per launch of a CG iteration (1 with
 * OSCAR_PC_JACOBI; about 8 with OSCAR_PC_MG) and a small pinned host
 * buffer, freed by oscar_destroy; OSCAR_E_ARG if a launch has more than 1040
 * workgroups.  While timing, at most 32 sampled iterations are enqueued
 * between two reads of the solver state.
 * oscar_timing_read(ctx, k, ...) returns the summed time [ms] and the number
 * of sampled iterations that did work (iterations enqueued past the
 * device-side convergence test exit at once and are not counted) for part k:
 *   k = 0  the whole iteration (when a read of the solver state by the host
 *          falls between its search-direction launch and the rest, the
 *          two spans without the gap);
 *   k = 1  the search-direction kernel (OSCAR_PC_JACOBI: the iteration kernel);
 *   k = 2  OSCAR_PC_MG: fine-grid pre-smoothing with the restriction and the
 *          vector updates;
 *   k = 3  OSCAR_PC_MG: the coarse levels of the V-cycle;
 *   k = 4  OSCAR_PC_MG: fine-grid prolongation, post-smoothing, reduction.
 * Parts 2-4 read zero with OSCAR_PC_JACOBI.  Reading synchronises the
 * stream. */
int32_t oscar_timing(oscar_ctx *ctx, int32_t period);
int32_t oscar_timing_read(oscar_ctx *ctx, int32_t kernel, double *total_ms, int64_t *launches);

/* ------------------------------------------------------------------------
 * Serving engine: continuous batching of independent relaxation requests.
 *
 * A request is one grid (descriptor) advanced by one viscous-drag step
 * followed by one capillary relaxation (Section 3) and fetched.  The engine
 * owns one caller-provided device workspace: a table part (see
 * oscar_engine_table_bytes) and a heap from which each admitted request
 * takes exactly oscar_workspace_size bytes.  Fields stay resident on the
 * device from admission to release.  oscar_engine_run advances every
 * resident request by one step per tick in shared launches (a viscous step
 * for a newly admitted request, a capillary sub-step otherwise); requests
 * admitted between ticks join the next tick.  Each request's arithmetic
 * depends only on its own data, so its results are bitwise the same alone
 * and in any mix.  All engine precision is fixed at creation (OSCAR_FP64 or
 * OSCAR_MIXED).  One host thread per engine.
 * ------------------------------------------------------------------------ */
typedef struct oscar_engine oscar_engine;

/* Bytes of the table part of an engine workspace for max_slots requests. */
int32_t oscar_engine_table_bytes(int32_t max_slots, uint64_t *bytes);

/* dev_workspace: caller-owned, 256-byte aligned, >= table bytes; the rest is
 * the request heap.  OSCAR_E_WORKSPACE if too small or misaligned. */
int32_t oscar_engine_create(int32_t max_slots, int32_t precision, void *dev_workspace, uint64_t bytes,
                            void *hip_stream, oscar_engine **out);

/* Admit a request if a slot is free and its footprint fits a free heap
 * region (else OSCAR_E_CAPACITY, nothing changed).  The descriptor is
 * validated as in oscar_create (its precision must equal the engine's);
 * dt_vd, n_sub, max_iters, tol as in oscar_capillary_relax.  Host arrays are
 * read during the call only.  *slot receives the slot index. */
int32_t oscar_engine_admit(oscar_engine *eng, const oscar_desc *desc, double dt_vd, int32_t n_sub,
                           int32_t max_iters, double tol, int32_t *slot);

/* Run `ticks` ticks (returns at once when nothing is resident). */
int32_t oscar_engine_run(oscar_engine *eng, int32_t ticks);

/* How the engine runs the pressure solves of a tick (OSCAR_SOLVE_*; the
 * requests' own solve_mode is not used).  With OSCAR_SOLVE_PERSISTENT one
 * launch per PISO corrector solves every resident request's equation (each
 * request advancing through its own iterations and refinement steps), and
 * the host reads the requests' state once per tick.  Results are bitwise
 * the same in both modes.  Takes effect at the next tick. */
int32_t oscar_engine_set_solve_mode(oscar_engine *eng, int32_t solve_mode);

/* Slots whose request has finished (up to cap), and the number still running. */
int32_t oscar_engine_poll(const oscar_engine *eng, int32_t *done_slots, int32_t cap, int32_t *n_done,
                          int32_t *n_active);

/* Copy a finished request's alpha (cells), p = p_vd + p_cr (cells) and
 * U = U_vd + (1/N) sum u_cr (dim*cells) to host arrays (any may be NULL),
 * with its completed sub-steps k_f and its status (OSCAR_* of the request). */
int32_t oscar_engine_fetch(oscar_engine *eng, int32_t slot, double *alpha, double *p, double *U, int32_t *k_f,
                           int32_t *status);

/* Free a slot and its heap region (a running request is cancelled). */
int32_t oscar_engine_release(oscar_engine *eng, int32_t slot);

int32_t oscar_engine_free_bytes(const oscar_engine *eng, uint64_t *largest_region, int32_t *free_slots);
int32_t oscar_engine_stats(const oscar_engine *eng, int64_t *ticks, int64_t *cg_iters);
void oscar_engine_destroy(oscar_engine *eng);   /* NULL-safe; does not free the workspace */
const char *oscar_engine_last_error(const oscar_engine *eng);

/* Brackbill capillary time-step limit sqrt(rho_bar h^3 / (2 pi sigma)),
 * rho_bar = (rho1 + rho2)/2 (Section 2.2). */
double oscar_dt_brackbill(double rho1, double rho2, double h, double sigma);

#ifdef __cplusplus
}
#endif
#endif
