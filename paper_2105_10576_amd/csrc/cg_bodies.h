// Bodies of the Jacobi-preconditioned conjugate gradient and of the FP64
// refinement of the mixed-precision path, shared by their grid-wide kernels
// (kernels.hip) and by the single-workgroup solve of small grids (mg.hip).
// A body works on block lb of its slot; the caller has checked that the
// slot's control block is active (and, for the CG bodies, that the solve is
// not done).
#pragma once
#include "device_common.h"

namespace oscar {

// Mixed precision: the FP32 inner solve of M e = r (|r| = rn) stops at the
// residual the FP64 test needs, 0.9 rtol |b| (|b| = bn), but is never asked
// for a relative reduction below rtol_inner, which FP32 reaches reliably;
// the outer refinement covers the rest.
__device__ __forceinline__ double inner_target(const SlotCtl &ctl, double bn, double rn) {
  double need = 0.9 * ctl.rtol * bn, floor = ctl.rtol_inner * rn;
  return need > floor ? need : floor;
}

// Conjugate gradient in the single-reduction form of Chronopoulos and Gear
// (1989), Jacobi preconditioner u = D^-1 r, w = A u, s = A p:
//   p_i = u_i + beta_i p_{i-1},  s_i = w_i + beta_i s_{i-1},
//   x_{i+1} = x_i + alpha_i p_i,  r_{i+1} = r_i - alpha_i s_i,
//   gamma = <r,u>, delta = <w,u>, beta_{i+1} = gamma_{i+1} / gamma_i,
//   alpha_{i+1} = gamma_{i+1} / (delta_{i+1} - beta_{i+1} gamma_{i+1} / alpha_i).
// Equal to the Hestenes-Stiefel recurrences in exact arithmetic; one launch
// and one reduction (<r,u>, <w,u>, <r,r>) per iteration.

// w_0 = A D^-1 r_0 and the first reduction
template <typename R>
__device__ __forceinline__ void cg_init_body(const Slot &s, int lb) {
  using T = R;
  const Grid G = grid_of(s);
  const uint8_t *flags = s.flags;
  const R *rAU = (const R *)s.rAU;
  const T *r = (const T *)s.cr[0], *invD = (const T *)s.invD;
  T *w = (T *)s.cw[0];
  double red[3] = {0.0, 0.0, 0.0};   // <r,u>, <w,u>, <r,r>
  for_cells(G, lb, [&](const Cell &c) {
    uint8_t fl = flags[c.P];
    if (fl & 0x40) return;   // solid entries of the CG vectors are never read
    auto uv = [&](int x) -> T { return invD[x] * r[x]; };
    T u = uv(c.P);
    T ww = matvec_row<T, R>(G, rAU, c, fl, uv);
    w[c.P] = ww;
    T rr = r[c.P];
    red[0] = red[0] + (double)(rr * u);
    red[1] = red[1] + (double)(ww * u);
    red[2] = red[2] + (double)(rr * rr);
  });
  put_partials<0u>(s, lb, CH_CG1, red);   // read by iteration 0
}

// iteration it (0-based): scalars from the previous reduction, convergence
// test (it > 0), vector updates, w_{it+1} = A D^-1 r_{it+1}, next reduction
// (false: the solve converged or hit the cap at this test; nothing was written)
template <typename R>
__device__ __forceinline__ bool cg_iter_body(const Slot &s, int lb, int it) {
  using T = R;
  const Grid G = grid_of(s);
  const uint8_t *flags = s.flags;
  const SlotCtl &ctl = *s.ctl;
  SlotState *st = s.st;
  const bool mixed = s.precision != 0;
  double v[3];
  get_totals<0u>(s, CH_CG0 + ((it + 1) & 1), v);   // written by iteration it - 1
  const double gam = v[0], del = v[1];
  double alpha, beta = 0.0;
  if (it == 0) {
    alpha = gam / del;
  } else {
    double rn = sqrt(v[2]);
    bool conv = rn <= (mixed ? st->tgt : ctl.rtol * st->bn);
    bool cap = !conv && it >= ctl.max_it;
    if (conv || cap) {
      if (lb == 0 && threadIdx.x == 0) {
        st->rn = rn;
        st->it = it;
        st->done = 1;
        if (cap) st->maxit_hit = st->maxit_hit + 1;
      }
      return false;
    }
    beta = gam / st->gam[(it - 1) & 1];
    alpha = gam / (del - beta * gam / st->alp[(it - 1) & 1]);
    if (lb == 0 && threadIdx.x == 0) st->rn = rn;
  }
  if (lb == 0 && threadIdx.x == 0) {
    st->gam[it & 1] = gam;
    st->alp[it & 1] = alpha;
    st->it = it + 1;
    st->total_it = st->total_it + 1;
  }
  const bool first = it == 0;
  const T al = (T)alpha, be = (T)beta;
  const R *rAU = (const R *)s.rAU;
  const T *invD = (const T *)s.invD;
  // s = w + beta s_old; on the first iteration beta = 0 and s_old = w, so
  // s = w exactly and every load is unconditional
  const T *r0 = (const T *)s.cr[it & 1], *w0 = (const T *)s.cw[it & 1];
  const T *so = first ? w0 : (const T *)s.cs[(it + 1) & 1];
  T *r1 = (T *)s.cr[(it + 1) & 1], *w1 = (T *)s.cw[(it + 1) & 1], *sn = (T *)s.cs[it & 1];
  T *pv = (T *)s.cp, *xe = (T *)s.e;
  double *xp = ctl.mode ? s.p_cr : s.p_vd;
  double red[3] = {0.0, 0.0, 0.0};
  for_cells(G, lb, [&](const Cell &c) {
    uint8_t fl = flags[c.P];
    if (fl & 0x40) return;   // solid entries of the CG vectors are never read
    // s = w + beta s_old and the updated residual, at any fluid cell
    auto s_at = [&](int x) -> T { return w0[x] + be * so[x]; };
    auto u_new = [&](int x) -> T { return invD[x] * (r0[x] - al * s_at(x)); };
    const int P = c.P;
    T u0 = invD[P] * r0[P];
    const T pold = pv[P];
    T pn = first ? u0 : u0 + be * pold;
    T sP = s_at(P);
    T rn = r0[P] - al * sP;
    T un = invD[P] * rn;
    T wn = matvec_row<T, R>(G, rAU, c, fl, u_new);
    pv[P] = pn;
    sn[P] = sP;
    r1[P] = rn;
    w1[P] = wn;
    if (mixed) xe[P] = xe[P] + al * pn;
    else xp[P] = xp[P] + (double)al * (double)pn;
    red[0] = red[0] + (double)(rn * un);
    red[1] = red[1] + (double)(wn * un);
    red[2] = red[2] + (double)(rn * rn);
  });
  put_partials<0u>(s, lb, CH_CG0 + (it & 1), red);
  return true;
}

// An outer refinement step acts only on a finished inner solve (done after at
// least one iteration).  Enqueued behind a chunk of iterations that did not
// reach the inner tolerance, it does nothing; after a refinement that met
// the outer tolerance (done, it = 0), a further one does nothing either.
__device__ __forceinline__ bool refine_due(const Slot &s, const SlotCtl &ctl) {
  const SlotState *st = s.st;
  return ctl.active && s.precision != 0 && !st->zero_rhs && st->done && st->it > 0;
}

// mixed precision, outer refinement: p += e, e = 0
template <typename R>
__device__ __forceinline__ void refine_x_body(const Slot &s, const SlotCtl &ctl, int lb) {
  if (!refine_due(s, ctl)) return;
  double *p = ctl.mode ? s.p_cr : s.p_vd;
  R *e = (R *)s.e;
  for_cells(s, lb, [&](const Cell &c) {
    if (solid_at(s, c.P)) return;
    p[c.P] = p[c.P] + (double)e[c.P];
    e[c.P] = (R)0;
  });
}

// mixed precision: r64 = rhs - M p in FP64; restart the FP32 inner solve on it
template <typename R>
__device__ __forceinline__ void refine_res_body(const Slot &s, const SlotCtl &ctl, int lb) {
  using T = R;
  const Grid G = grid_of(s);
  const uint8_t *flags = s.flags;
  if (!refine_due(s, ctl)) return;
  const R *rAU = (const R *)s.rAU;
  const double *p = ctl.mode ? s.p_cr : s.p_vd;
  T *r = (T *)s.cr[0];
  double red[2] = {0.0, 0.0};
  for_cells(G, lb, [&](const Cell &c) {
    uint8_t fl = flags[c.P];
    if (fl & 0x40) return;
    double Mp = matvec_row<double, R>(G, rAU, c, fl, [&](int x) { return p[x]; });
    double r64 = s.rhs[c.P] - Mp;
    T rr = (T)r64;
    r[c.P] = rr;
    red[0] = red[0] + r64 * r64;
    red[1] = red[1] + (double)(rr * rr);
  });
  put_partials<0u>(s, lb, CH_REF, red);
}

__device__ __forceinline__ void refine_fin_body(const Slot &s) {
  const SlotCtl &ctl = *s.ctl;
  if (!refine_due(s, ctl)) return;   // read by every thread before thread 0 writes below
  double v[2];
  get_totals<0u>(s, CH_REF, v);
  if (threadIdx.x == 0) {
    SlotState *st = s.st;
    st->rn64_prev = st->rn64;
    st->rn64 = sqrt(v[0]);
    st->bn = sqrt(v[1]);
    st->rn = st->bn;
    st->tgt = inner_target(ctl, st->bn64, st->bn);
    st->it = 0;
    st->refine_steps = st->refine_steps + 1;
    st->ref_solve = st->ref_solve + 1;
    const bool met = st->rn64 <= ctl.rtol * st->bn64;
    const bool stall = !met && (!(st->rn64 < 0.5 * st->rn64_prev) || st->ref_solve >= REFINE_MAX);
    st->stalled = stall;
    if (stall) st->stall_hits = st->stall_hits + 1;
    st->done = met || stall;
  }
}


}  // namespace oscar
