// OSCAR relaxation-path kernels for gfx950 (CDNA4).
//
// Discretisation (arXiv 2105.10576, Sections 2-4): cell-centred finite
// volumes on a uniform voxel grid, explicit alpha transport with van Leer
// (1974) face values, interface compression and a Zalesak (1979) limiter,
// continuum surface force with the Brackbill (1992) wall-adhesion normal,
// implicit-Euler momentum with upwind + linear-upwind convection and the
// transpose viscous term, PISO (Issa 1985) pressure correction in the
// balanced-force face form, Jacobi-preconditioned conjugate gradient.
//
// Layout: cells x-fastest, idx = i + nx*(j + ny*k); face arrays per
// direction (x-faces (nx+1)*ny*nz first, then y, then z), a face indexed by
// its high-side cell coordinates; vector fields component-major.
//
// Execution: one thread per cell, 256-thread workgroups; a thread also owns
// the low face of its cell in every direction and the far boundary face when
// it sits on the last layer.  Memory-bound stencil work: every kernel streams
// each array once; neighbour reuse comes from the L1/L2 caches.  Arithmetic is
// written operation by operation (no fused multiply-add: built with
// -ffp-contract=off) so that the FP64 instantiation rounds exactly like the
// sequential double-precision reference.
#include "device_common.h"
#include "cg_bodies.h"

namespace oscar {

// ---------------------------------------------------------------------------
// indexing and boundary classification
// ---------------------------------------------------------------------------

// a zeroed (inactive) control block for padding entries of a block table
__device__ SlotCtl g_padding_ctl;

__device__ __forceinline__ Block block_of(const Slot *slots, const int2 *btab) {
  int2 t = btab[blockIdx.x];
  Block b;
  b.s = slots + t.x;
  b.ctl = t.y < 0 ? &g_padding_ctl : b.s->ctl;
  b.st = b.s->st;
  b.lb = t.y;
  return b;
}

// ---------------------------------------------------------------------------
// control kernels
// ---------------------------------------------------------------------------

__global__ void k_ctl_update(Slot *slots, CtlUpdate u) {
  int t = threadIdx.x;
  if (t < u.n) *slots[u.slot[t]].ctl = u.ctl[t];
}

// copy every used slot's state into one array (one host read per poll)
__global__ void k_gather_states(const Slot *slots, int nslots, SlotState *out) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nslots) return;
  const Slot &s = slots[t];
  if (!s.st) return;
  out[t] = *s.st;
}

__global__ void k_state_reset(const Slot *slots, int nslots) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nslots) return;
  const Slot &s = slots[t];
  if (!s.ctl || !s.ctl->active) return;
  SlotState *st = s.st;
  st->nonfinite = 0;
  st->unstable = 0;
  st->maxit_hit = 0;
  st->total_it = 0;
  st->refine_steps = 0;
  st->stall_hits = 0;
}

// ---------------------------------------------------------------------------
// viscous step prologue: keep u_vd^n (face fluxes) for the transport and the
// convecting velocity of this global step
// ---------------------------------------------------------------------------

template <typename R>
__global__ void __launch_bounds__(BLOCK) k_copy_phi_prev(const Slot *slots, const int2 *btab) {
  Block B = block_of(slots, btab);
  const Slot &s = *B.s;
  if (!B.ctl->active || B.ctl->mode != 0) return;
  const R *src = (const R *)s.phi_vd;
  R *dst = (R *)s.phi_prev;
  for_cells(s, B.lb, [&](const Cell &c) {
    for_owned_faces(s, c, [&](int, int fi, const FView &) { dst[fi] = src[fi]; });
  });
}

// ---------------------------------------------------------------------------
// interface normal and curvature
// ---------------------------------------------------------------------------

// Gauss gradient of alpha at cells (face values: the two-cell mean on
// interior faces, the cell value elsewhere).  Like the corrector kernels,
// these take every operand of a batch of cells before the arithmetic.
template <typename R>
__global__ void __launch_bounds__(BLOCK) k_grad_alpha(const Slot *slots, const int2 *btab, int only_cr) {
  Block B = block_of(slots, btab);
  const Slot &s = *B.s;
  if (!B.ctl->active || (only_cr && B.ctl->mode != 1)) return;
  const int d = s.dim, nc = s.nc;
  const R *a = (const R *)s.alpha;
  R *g = (R *)s.grad;
  const R h = (R)s.h;
  struct Op {
    Cell c;
    uint8_t fl;   // 0x80: past the end
    R aP, an[6];
  };
  batched<2, Op>(
      B.lb * BLOCK + (int)threadIdx.x, s.nblocks * BLOCK, nc,
      [&](Op &o, int q) {
        o.fl = 0x80;
        if (q < nc) {
          o.c = cell_at(s, q);
          o.fl = s.flags[q];
        }
      },
      [&](Op &o) {
        if (o.fl & 0xC0) return;
        const Hood hd = hood_of(s, o.fl, o.c);
        o.aP = gld(a, o.c.P);
#pragma unroll
        for (int f = 0; f < 6; ++f) o.an[f] = gld(a, hd.nb[f]);
      },
      [&]() { return true; },
      [&](Op &o) {
        if (o.fl & 0x80) return;
#pragma unroll
        for (int e = 0; e < 3; ++e) {
          if (e >= d) continue;
          R ge = (R)0;
          if (!(o.fl & 0x40)) {
            R alo = ((o.fl >> (2 * e)) & 1u) ? (R)0.5 * (o.aP + o.an[2 * e]) : o.aP;
            R ahi = ((o.fl >> (2 * e + 1)) & 1u) ? (R)0.5 * (o.aP + o.an[2 * e + 1]) : o.aP;
            ge = (ahi - alo) / h;
          }
          gst(g, e * nc + o.c.P, ge);
        }
      });
}

// interface normal component of the faces each cell owns (the low face per
// direction, the far face on the last layer); walls carry the contact angle
template <typename R>
__global__ void __launch_bounds__(BLOCK) k_face_normals(const Slot *slots, const int2 *btab, int only_cr) {
  Block B = block_of(slots, btab);
  const Slot &s = *B.s;
  if (!B.ctl->active || (only_cr && B.ctl->mode != 1)) return;
  const R *g = (const R *)s.grad;
  R *nh = (R *)s.nhatf;
  const int d = s.dim, nc = s.nc;
  const R delta = (R)s.delta, cos_t = (R)s.cos_t;
  const int nn[3] = {s.nx, s.ny, s.nz}, st[3] = {1, s.nx, s.nxy};
  int bcf[6];
  for (int f = 0; f < 6; ++f) bcf[f] = s.bcf[f];
  struct Op {
    Cell c;
    uint8_t fl, flo[3];   // fl 0x80: past the end; flo: flags of the cell below per direction
    int fi[6];
    R gP[3], gl[3][3];    // gradient at the cell and at the cell below per direction
  };
  batched<2, Op>(
      B.lb * BLOCK + (int)threadIdx.x, s.nblocks * BLOCK, nc,
      [&](Op &o, int q) {
        o.fl = 0x80;
        if (q < nc) {
          o.c = cell_at(s, q);
          o.fl = s.flags[q];
        }
      },
      [&](Op &o) {
        if (o.fl & 0x80) return;
        const Cell &c = o.c;
        const Hood hd = hood_of(s, o.fl, c);
        const int cr[3] = {c.i, c.j, c.k};
#pragma unroll
        for (int f = 0; f < 6; ++f) o.fi[f] = hd.fi[f];
#pragma unroll
        for (int e = 0; e < 3; ++e) {
          const int lo = cr[e] > 0 ? c.P - st[e] : c.P;
          o.flo[e] = e < d ? s.flags[lo] : (uint8_t)0x40;
#pragma unroll
          for (int cc = 0; cc < 3; ++cc) {
            o.gl[e][cc] = (e < d && cc < d) ? gld(g, cc * nc + lo) : (R)0;
            if (e == 0) o.gP[cc] = cc < d ? gld(g, cc * nc + c.P) : (R)0;
          }
        }
      },
      [&]() { return true; },
      [&](Op &o) {
        if (o.fl & 0x80) return;
        const Cell &c = o.c;
        const int cr[3] = {c.i, c.j, c.k};
        // normal component on a face of type t whose fluid cell (boundary
        // faces) has gradient Gc, seen with orientation sign sf
        auto boundary = [&](int t, int e, const R (&Gc)[3], R sf) -> R {
          R G[3] = {Gc[0], Gc[1], Gc[2]};
          if (t == F_INLET || t == F_OUTLET) return G[e] / (vnorm(G, d) + delta);
          if (t == F_WALL) {
            // wall adhesion n.n_w = cos(theta): the wall-normal component of
            // the interface normal at the wall face, faded like the interior
            // normals
            R mg = vnorm(G, d);
            return (mg / (mg + delta)) * (cos_t * sf);
          }
          return (R)0;
        };
#pragma unroll
        for (int e = 0; e < 3; ++e) {
          if (e >= d) continue;
          int side;
          const int t = low_face_type(s, o.fl, o.flo[e], cr[e] == 0, e, side);
          R out;
          if (t == F_INT) {
            R G[3] = {(R)0, (R)0, (R)0};
#pragma unroll
            for (int cc = 0; cc < 3; ++cc)
              if (cc < d) G[cc] = (R)0.5 * (o.gl[e][cc] + o.gP[cc]);
            out = G[e] / (vnorm(G, d) + delta);
          } else {
            out = side ? boundary(t, e, o.gP, (R)-1) : boundary(t, e, o.gl[e], (R)1);
          }
          gst(nh, o.fi[2 * e], out);
          if (cr[e] == nn[e] - 1)
            gst(nh, o.fi[2 * e + 1], (o.fl & 0x40) ? (R)0 : boundary(bcf[2 * e + 1], e, o.gP, (R)1));
        }
      });
}

template <typename R>
__global__ void __launch_bounds__(BLOCK) k_curvature(const Slot *slots, const int2 *btab) {
  Block B = block_of(slots, btab);
  const Slot &s = *B.s;
  if (!B.ctl->active || B.ctl->mode != 1) return;
  const R *nh = (const R *)s.nhatf;
  R *kap = (R *)s.kappa;
  for_cells(s, B.lb, [&](const Cell &c) {
    uint8_t fl = s.flags[c.P];
    R out = (R)0;
    if (!(fl & 0x40)) {
      R acc = (R)0;
      for (int e = 0; e < s.dim; ++e) {
        CFace lo = cell_face(s, fl, c, 2 * e), hi = cell_face(s, fl, c, 2 * e + 1);
        acc = acc + (nh[hi.fi] - nh[lo.fi]);
      }
      out = -acc / (R)s.h;
    }
    kap[c.P] = out;
  });
}

// ---------------------------------------------------------------------------
// alpha transport: upwind + van Leer/compression, Zalesak limiter
// ---------------------------------------------------------------------------

// Face fluxes of the faces each cell owns (low-order F_L and antidiffusive
// A = F_H - F_L, with the van Leer face value and the compression flux),
// alpha_old, and per block the largest Courant number and the phase sum.
// The operands of a batch of cells (alpha two cells down and one up along
// each direction for the van Leer upwind cell) are loaded first.
template <typename R>
__global__ void __launch_bounds__(BLOCK) k_mules_flux(const Slot *slots, const int2 *btab) {
  Block B = block_of(slots, btab);
  const Slot &s = *B.s;
  const SlotCtl &ctl = *B.ctl;
  if (!ctl.active) return;
  const int d = s.dim, nc = s.nc;
  const R *a = (const R *)s.alpha;
  const R *phi = (const R *)(ctl.mode ? s.phi_cr : s.phi_prev);
  const R *nh = (const R *)s.nhatf;
  R *FL = (R *)s.FL, *Af = (R *)s.Af, *aold = (R *)s.alpha_old;
  const R dtV = (R)ctl.dt / (R)s.V;
  const int nn[3] = {s.nx, s.ny, s.nz}, st[3] = {1, s.nx, s.nxy};
  int bcf[6];
  for (int f = 0; f < 6; ++f) bcf[f] = s.bcf[f];
  double red[2] = {0.0, 0.0};   // max Courant, sum alpha
  struct Op {
    Cell c;
    uint8_t fl, flo[3];   // fl 0x80: past the end; flo: flags of the cell below per direction
    int fi[6];
    R aP, alo[3], alolo[3], ahi[3];   // alpha at the cell, one and two below, one above
    R ph[6], nhl[3];                  // flux of each face of the cell, normal of the low faces
  };
  batched<2, Op>(
      B.lb * BLOCK + (int)threadIdx.x, s.nblocks * BLOCK, nc,
      [&](Op &o, int q) {
        o.fl = 0x80;
        if (q < nc) {
          o.c = cell_at(s, q);
          o.fl = s.flags[q];
        }
      },
      [&](Op &o) {
        if (o.fl & 0x80) return;
        const Cell &c = o.c;
        const Hood hd = hood_of(s, o.fl, c);
        const int cr[3] = {c.i, c.j, c.k};
        o.aP = gld(a, c.P);
#pragma unroll
        for (int e = 0; e < 3; ++e) {
          const int lo = cr[e] > 0 ? c.P - st[e] : c.P;
          const int lolo = cr[e] > 1 ? c.P - 2 * st[e] : lo;
          const int hi = cr[e] < nn[e] - 1 ? c.P + st[e] : c.P;
          o.fi[2 * e] = hd.fi[2 * e];
          o.fi[2 * e + 1] = hd.fi[2 * e + 1];
          o.flo[e] = e < d ? s.flags[lo] : (uint8_t)0x40;
          o.alo[e] = gld(a, lo);
          o.alolo[e] = gld(a, lolo);
          o.ahi[e] = gld(a, hi);
          o.ph[2 * e] = e < d ? gld(phi, hd.fi[2 * e]) : (R)0;
          o.ph[2 * e + 1] = e < d ? gld(phi, hd.fi[2 * e + 1]) : (R)0;
          o.nhl[e] = e < d ? gld(nh, hd.fi[2 * e]) : (R)0;
        }
      },
      [&]() { return true; },
      [&](Op &o) {
        if (o.fl & 0x80) return;
        const Cell &c = o.c;
        const int cr[3] = {c.i, c.j, c.k};
        const bool fluid = !(o.fl & 0x40);
        gst(aold, c.P, o.aP);
#pragma unroll
        for (int e = 0; e < 3; ++e) {
          if (e >= d) continue;
          int side;
          const int t = low_face_type(s, o.fl, o.flo[e], cr[e] == 0, e, side);
          (void)side;
          R fl_ = (R)0, af = (R)0, ph = o.ph[2 * e];
          if (t == F_INT) {
            // upwind cell C, downwind D, and the cell beyond C away from D
            // (C itself when that one is solid or outside)
            const bool up = ph >= (R)0;
            const R aC = up ? o.alo[e] : o.aP, aD = up ? o.aP : o.alo[e];
            const bool uu = up ? ((o.flo[e] >> (2 * e)) & 1u) : ((o.fl >> (2 * e + 1)) & 1u);
            R aUU = aC;
            if (uu) aUU = up ? o.alolo[e] : o.ahi[e];
            R dD = aD - aC, dU = aC - aUU;
            R avl = aC + (dU * dD > (R)0 ? (dU * dD) / (dU + dD) : (R)0);
            R abar = (R)0.5 * (o.alo[e] + o.aP);
            R phir = fabs(ph) * o.nhl[e];
            R Fc = (phir * abar) * ((R)1 - abar);
            R FH = ph * avl + Fc;
            fl_ = ph * aC;
            af = FH - fl_;
          } else if (t == F_INLET || t == F_OUTLET) {
            fl_ = ph * o.aP;   // open sides: this cell is the fluid one
          }
          gst(FL, o.fi[2 * e], fl_);
          gst(Af, o.fi[2 * e], af);
          if (cr[e] == nn[e] - 1) {
            const int tf = fluid ? bcf[2 * e + 1] : F_NONE;
            gst(FL, o.fi[2 * e + 1], (tf == F_INLET || tf == F_OUTLET) ? o.ph[2 * e + 1] * o.aP : (R)0);
            gst(Af, o.fi[2 * e + 1], (R)0);
          }
        }
        if (fluid) {
          R acc = (R)0;
#pragma unroll
          for (int f = 0; f < 6; ++f) {
            if (f >= 2 * d) continue;
            R sp = ((f & 1) ? (R)1 : (R)-1) * o.ph[f];
            if (sp > (R)0) acc = acc + sp;
          }
          double co = (double)(acc * dtV);
          red[0] = co > red[0] ? co : red[0];
          red[1] = red[1] + (double)o.aP;
        }
      });
  put_partials<1u>(s, B.lb, CH_ADV1, red);
}

// Zalesak limiter: R+ and R- of every fluid cell from the fluxes of its
// faces and the local bounds; operands first
template <typename R>
__global__ void __launch_bounds__(BLOCK) k_mules_limiter(const Slot *slots, const int2 *btab) {
  Block B = block_of(slots, btab);
  const Slot &s = *B.s;
  const SlotCtl &ctl = *B.ctl;
  if (!ctl.active) return;
  const int d = s.dim, nc = s.nc;
  const R *a = (const R *)s.alpha;
  const R *FLv = (const R *)s.FL, *Afv = (const R *)s.Af;
  R *Rp = (R *)s.Rp, *Rm = (R *)s.Rm;
  const R dtV = (R)ctl.dt / (R)s.V, Vdt = (R)s.V / (R)ctl.dt;
  struct Op {
    Cell c;
    uint8_t fl;   // 0x80: past the end
    R aP, an[6], F[6], A[6];
  };
  batched<2, Op>(
      B.lb * BLOCK + (int)threadIdx.x, s.nblocks * BLOCK, nc,
      [&](Op &o, int q) {
        o.fl = 0x80;
        if (q < nc) {
          o.c = cell_at(s, q);
          o.fl = s.flags[q];
        }
      },
      [&](Op &o) {
        if (o.fl & 0xC0) return;
        const Hood hd = hood_of(s, o.fl, o.c);
        o.aP = gld(a, o.c.P);
#pragma unroll
        for (int f = 0; f < 6; ++f) {
          o.an[f] = gld(a, hd.nb[f]);
          o.F[f] = f < 2 * d ? gld(FLv, hd.fi[f]) : (R)0;
          o.A[f] = f < 2 * d ? gld(Afv, hd.fi[f]) : (R)0;
        }
      },
      [&]() { return true; },
      [&](Op &o) {
        if (o.fl & 0x80) return;
        R rp = (R)0, rm = (R)0;
        if (!(o.fl & 0x40)) {
          R sumL = (R)0, Pp = (R)0, Pm = (R)0, amax = o.aP, amin = o.aP;
#pragma unroll
          for (int f = 0; f < 6; ++f) {
            if (f >= 2 * d) continue;
            R sg = (f & 1) ? (R)1 : (R)-1;
            sumL = sumL + sg * o.F[f];
            R sA = sg * o.A[f];
            Pp = Pp + (sA < (R)0 ? -sA : (R)0);
            Pm = Pm + (sA > (R)0 ? sA : (R)0);
            if ((o.fl >> f) & 1u) {
              R an = o.an[f];
              if (an > amax) amax = an;
              if (an < amin) amin = an;
            }
          }
          R aL = o.aP - dtV * sumL;
          if (amax > (R)1) amax = (R)1;
          if (amin < (R)0) amin = (R)0;
          R Qp = Vdt * (amax - aL > (R)0 ? amax - aL : (R)0);
          R Qm = Vdt * (aL - amin > (R)0 ? aL - amin : (R)0);
          rp = Pp > (R)0 ? (Qp / Pp < (R)1 ? Qp / Pp : (R)1) : (R)0;
          rm = Pm > (R)0 ? (Qm / Pm < (R)1 ? Qm / Pm : (R)1) : (R)0;
        }
        gst(Rp, o.c.P, rp);
        gst(Rm, o.c.P, rm);
      });
}

// limited update alpha -= dt/V sum_f s_f (F_L + lambda A); with more than
// one limiting pass the lower cell of each interior face also writes the
// unused flux (1 - lambda) A for the next pass
template <typename R>
__global__ void __launch_bounds__(BLOCK) k_mules_update(const Slot *slots, const int2 *btab) {
  Block B = block_of(slots, btab);
  const Slot &s = *B.s;
  const SlotCtl &ctl = *B.ctl;
  if (!ctl.active) return;
  const int d = s.dim, nc = s.nc;
  R *a = (R *)s.alpha;
  const R *FLv = (const R *)s.FL, *Afv = (const R *)s.Af, *Rpv = (const R *)s.Rp, *Rmv = (const R *)s.Rm;
  R *Arest = (R *)s.Af2;   // unused flux for the next limiting pass
  const bool more = s.mules_iter > 1;
  const R dtV = (R)ctl.dt / (R)s.V;
  double red[2] = {0.0, 0.0};   // sum alpha_new, boundary flux
  struct Op {
    Cell c;
    uint8_t fl;   // 0x80: past the end
    int fi[6];
    R aP, rpP, rmP, rpn[6], rmn[6], F[6], A[6];
  };
  batched<2, Op>(
      B.lb * BLOCK + (int)threadIdx.x, s.nblocks * BLOCK, nc,
      [&](Op &o, int q) {
        o.fl = 0x80;
        if (q < nc) {
          o.c = cell_at(s, q);
          o.fl = s.flags[q];
        }
      },
      [&](Op &o) {
        if (o.fl & 0xC0) return;
        const int P = o.c.P;
        const Hood hd = hood_of(s, o.fl, o.c);
        o.aP = gld(a, P);
        o.rpP = gld(Rpv, P);
        o.rmP = gld(Rmv, P);
#pragma unroll
        for (int f = 0; f < 6; ++f) {
          o.fi[f] = hd.fi[f];
          o.rpn[f] = gld(Rpv, hd.nb[f]);
          o.rmn[f] = gld(Rmv, hd.nb[f]);
          o.F[f] = f < 2 * d ? gld(FLv, hd.fi[f]) : (R)0;
          o.A[f] = f < 2 * d ? gld(Afv, hd.fi[f]) : (R)0;
        }
      },
      [&]() { return true; },
      [&](Op &o) {
        if (o.fl & 0xC0) return;
        R acc = (R)0, bfl = (R)0;
#pragma unroll
        for (int f = 0; f < 6; ++f) {
          if (f >= 2 * d) continue;
          R sg = (f & 1) ? (R)1 : (R)-1;
          R lam = (R)0;
          if ((o.fl >> f) & 1u) {
            // R of the lower and upper cell of the face
            const R A = o.A[f];
            const R rplo = (f & 1) ? o.rpP : o.rpn[f], rmlo = (f & 1) ? o.rmP : o.rmn[f];
            const R rphi = (f & 1) ? o.rpn[f] : o.rpP, rmhi = (f & 1) ? o.rmn[f] : o.rmP;
            R x1 = A >= (R)0 ? rmlo : rplo;
            R x2 = A >= (R)0 ? rphi : rmhi;
            lam = x1 < x2 ? x1 : x2;
            if (more && (f & 1)) gst(Arest, o.fi[f], ((R)1 - lam) * A);
          } else {
            bfl = bfl + sg * o.F[f];
          }
          acc = acc + sg * (o.F[f] + lam * o.A[f]);
        }
        R an = o.aP - dtV * acc;
        gst(a, o.c.P, an);
        red[0] = red[0] + (double)an;
        red[1] = red[1] + (double)bfl;
      });
  put_partials<0u>(s, B.lb, CH_ADV2, red);
}

// Limiting pass `pass` >= 2 (iterative flux correction): the antidiffusive
// flux the earlier passes left unused sits in Af2 (even passes) or Af (odd
// passes); the local bounds are those of the first pass, taken from
// alpha_old, and Q+- from the current alpha.
template <typename R>
__global__ void __launch_bounds__(BLOCK) k_mules_limiter_again(const Slot *slots, const int2 *btab, int pass) {
  Block B = block_of(slots, btab);
  const Slot &s = *B.s;
  const SlotCtl &ctl = *B.ctl;
  if (!ctl.active || pass > s.mules_iter) return;
  const R *a = (const R *)s.alpha, *ab = (const R *)s.alpha_old;
  const R *Ar = (const R *)((pass & 1) ? s.Af : s.Af2);
  R *Rp = (R *)s.Rp, *Rm = (R *)s.Rm;
  const R Vdt = (R)s.V / (R)ctl.dt;
  for_cells(s, B.lb, [&](const Cell &c) {
    uint8_t fl = s.flags[c.P];
    R rp = (R)0, rm = (R)0;
    if (!(fl & 0x40)) {
      R Pp = (R)0, Pm = (R)0, amax = ab[c.P], amin = ab[c.P];
      for (int f = 0; f < 2 * s.dim; ++f) {
        CFace cf = cell_face(s, fl, c, f);
        if (cf.type != F_INT) continue;   // only interior faces carry antidiffusive flux
        R sA = ((f & 1) ? (R)1 : (R)-1) * Ar[cf.fi];
        Pp = Pp + (sA < (R)0 ? -sA : (R)0);
        Pm = Pm + (sA > (R)0 ? sA : (R)0);
        R an = ab[cf.nb];
        if (an > amax) amax = an;
        if (an < amin) amin = an;
      }
      if (amax > (R)1) amax = (R)1;
      if (amin < (R)0) amin = (R)0;
      R cur = a[c.P];
      R Qp = Vdt * (amax - cur > (R)0 ? amax - cur : (R)0);
      R Qm = Vdt * (cur - amin > (R)0 ? cur - amin : (R)0);
      rp = Pp > (R)0 ? (Qp / Pp < (R)1 ? Qp / Pp : (R)1) : (R)0;
      rm = Pm > (R)0 ? (Qm / Pm < (R)1 ? Qm / Pm : (R)1) : (R)0;
    }
    Rp[c.P] = rp;
    Rm[c.P] = rm;
  });
}

template <typename R>
__global__ void __launch_bounds__(BLOCK) k_mules_update_again(const Slot *slots, const int2 *btab, int pass) {
  Block B = block_of(slots, btab);
  const Slot &s = *B.s;
  const SlotCtl &ctl = *B.ctl;
  if (!ctl.active || pass > s.mules_iter) return;
  R *a = (R *)s.alpha;
  const R *FL = (const R *)s.FL, *Rp = (const R *)s.Rp, *Rm = (const R *)s.Rm;
  const R *Ar = (const R *)((pass & 1) ? s.Af : s.Af2);
  R *An = (R *)((pass & 1) ? s.Af2 : s.Af);
  const bool more = pass < s.mules_iter;
  const R dtV = (R)ctl.dt / (R)s.V;
  double red[2] = {0.0, 0.0};   // sum alpha_new, boundary flux
  for_cells(s, B.lb, [&](const Cell &c) {
    uint8_t fl = s.flags[c.P];
    if (fl & 0x40) return;
    R acc = (R)0, bfl = (R)0;
    for (int f = 0; f < 2 * s.dim; ++f) {
      CFace cf = cell_face(s, fl, c, f);
      if (cf.type == F_NONE) continue;
      R sg = (f & 1) ? (R)1 : (R)-1;
      if (cf.type != F_INT) {
        bfl = bfl + sg * FL[cf.fi];
        continue;
      }
      int lo = (f & 1) ? c.P : cf.nb, hi = (f & 1) ? cf.nb : c.P;
      R A = Ar[cf.fi];
      R x1 = A >= (R)0 ? Rm[lo] : Rp[lo];
      R x2 = A >= (R)0 ? Rp[hi] : Rm[hi];
      R lam = x1 < x2 ? x1 : x2;
      if (more && (f & 1)) An[cf.fi] = ((R)1 - lam) * A;
      acc = acc + sg * (lam * A);
    }
    R an = a[c.P] - dtV * acc;
    a[c.P] = an;
    red[0] = red[0] + (double)an;
    red[1] = red[1] + (double)bfl;
  });
  put_partials<0u>(s, B.lb, CH_ADV2, red);
}

// one block per slot: Courant number, phase mass before/after, boundary flux
__global__ void __launch_bounds__(BLOCK) k_transport_fin(const Slot *slots) {
  const Slot &s = slots[blockIdx.x];
  if (!s.ctl) return;   // unused table entry
  const SlotCtl &ctl = *s.ctl;
  if (!ctl.active) return;
  double v1[2], v2[2];
  get_totals<1u>(s, CH_ADV1, v1);
  get_totals<0u>(s, CH_ADV2, v2);
  if (threadIdx.x == 0) {
    SlotState *st = s.st;
    st->comax = v1[0];
    st->mass0 = v1[1] * s.V;
    st->mass1 = v2[0] * s.V;
    st->bflux = v2[1];
    if (v1[0] > 1.0) st->unstable = 1;
    double defect = fabs(st->mass1 - st->mass0 + ctl.dt * v2[1]);
    if (defect > st->mass_defect) st->mass_defect = defect;
  }
}

// ---------------------------------------------------------------------------
// momentum matrix
// ---------------------------------------------------------------------------

template <typename R>
__device__ __forceinline__ R inlet_u(int cc, int e, R sg, R ub) {
  return cc == e ? -sg * ub : (R)0;
}

// Gauss gradient of the velocity, gU[(c*d+e)*nc + P] = dU_c/dx_e; operands
// of a batch of cells first
template <typename R>
__global__ void __launch_bounds__(BLOCK) k_grad_u(const Slot *slots, const int2 *btab) {
  Block B = block_of(slots, btab);
  const Slot &s = *B.s;
  const SlotCtl &ctl = *B.ctl;
  if (!ctl.active) return;
  const int d = s.dim, nc = s.nc;
  const R *Uo = (const R *)(ctl.mode ? s.U_cr : s.U_vd);
  R *gU = (R *)s.gradU;
  const R ub = (R)ctl.ub, h = (R)s.h;
  struct Op {
    Cell c;
    uint8_t fl;   // 0x80: past the end
    R uP[3], un[6][3];
  };
  batched<2, Op>(
      B.lb * BLOCK + (int)threadIdx.x, s.nblocks * BLOCK, nc,
      [&](Op &o, int q) {
        o.fl = 0x80;
        if (q < nc) {
          o.c = cell_at(s, q);
          o.fl = s.flags[q];
        }
      },
      [&](Op &o) {
        if (o.fl & 0xC0) return;
        const Hood hd = hood_of(s, o.fl, o.c);
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) {
          o.uP[cc] = cc < d ? gld(Uo, cc * nc + o.c.P) : (R)0;
#pragma unroll
          for (int f = 0; f < 6; ++f) o.un[f][cc] = (cc < d && f < 2 * d) ? gld(Uo, cc * nc + hd.nb[f]) : (R)0;
        }
      },
      [&]() { return true; },
      [&](Op &o) {
        if (o.fl & 0x80) return;
        const Cell &c = o.c;
#pragma unroll
        for (int e = 0; e < 3; ++e) {
          if (e >= d) continue;
          int ty[2];
          ty[0] = cell_face(s, o.fl, c, 2 * e).type;
          ty[1] = cell_face(s, o.fl, c, 2 * e + 1).type;
#pragma unroll
          for (int cc = 0; cc < 3; ++cc) {
            if (cc >= d) continue;
            R out = (R)0;
            if (!(o.fl & 0x40)) {
              R fv[2];
#pragma unroll
              for (int sd = 0; sd < 2; ++sd) {
                if (ty[sd] == F_INT) fv[sd] = (R)0.5 * (o.uP[cc] + o.un[2 * e + sd][cc]);
                else if (ty[sd] == F_WALL) fv[sd] = (R)0;
                else if (ty[sd] == F_INLET) fv[sd] = inlet_u<R>(cc, e, sd ? (R)1 : (R)-1, ub);
                else fv[sd] = o.uP[cc];
              }
              out = (fv[1] - fv[0]) / h;
            }
            gst(gU, (cc * d + e) * nc + c.P, out);
          }
        }
      });
}

// mass flux rho_f (phi_vd^n + phi_cr) of the faces each cell owns
template <typename R>
__global__ void __launch_bounds__(BLOCK) k_mass_flux(const Slot *slots, const int2 *btab) {
  Block B = block_of(slots, btab);
  const Slot &s = *B.s;
  if (!B.ctl->active) return;
  const int d = s.dim, nc = s.nc;
  const R *a = (const R *)s.alpha;
  const R *pa = (const R *)s.phi_prev, *pc = (const R *)s.phi_cr;
  R *Fm = (R *)s.Fm;
  const R rho1 = (R)s.rho1, rho2 = (R)s.rho2;
  const int nn[3] = {s.nx, s.ny, s.nz}, st[3] = {1, s.nx, s.nxy};
  int bcf[6];
  for (int f = 0; f < 6; ++f) bcf[f] = s.bcf[f];
  auto rho = [&](R x) -> R { return x * rho1 + ((R)1 - x) * rho2; };
  struct Op {
    Cell c;
    uint8_t fl, flo[3];
    int fi[6];
    R pa[6], pc[6], aP, al[3];   // fluxes of the low (and far) faces; alpha at the cell and below it
  };
  batched<2, Op>(
      B.lb * BLOCK + (int)threadIdx.x, s.nblocks * BLOCK, nc,
      [&](Op &o, int q) {
        o.fl = 0x80;
        if (q < nc) {
          o.c = cell_at(s, q);
          o.fl = s.flags[q];
        }
      },
      [&](Op &o) {
        if (o.fl & 0x80) return;
        const Cell &c = o.c;
        const Hood hd = hood_of(s, o.fl, c);
        const int cr[3] = {c.i, c.j, c.k};
        o.aP = gld(a, c.P);
#pragma unroll
        for (int e = 0; e < 3; ++e) {
          const int lo = cr[e] > 0 ? c.P - st[e] : c.P;
          o.fi[2 * e] = hd.fi[2 * e];
          o.fi[2 * e + 1] = hd.fi[2 * e + 1];
          o.flo[e] = e < d ? s.flags[lo] : (uint8_t)0x40;
          o.al[e] = gld(a, lo);
          const bool far = e < d && cr[e] == nn[e] - 1;
          o.pa[2 * e] = e < d ? gld(pa, hd.fi[2 * e]) : (R)0;
          o.pc[2 * e] = e < d ? gld(pc, hd.fi[2 * e]) : (R)0;
          o.pa[2 * e + 1] = far ? gld(pa, hd.fi[2 * e + 1]) : (R)0;
          o.pc[2 * e + 1] = far ? gld(pc, hd.fi[2 * e + 1]) : (R)0;
        }
      },
      [&]() { return true; },
      [&](Op &o) {
        if (o.fl & 0x80) return;
        const Cell &c = o.c;
        const int cr[3] = {c.i, c.j, c.k};
#pragma unroll
        for (int e = 0; e < 3; ++e) {
          if (e >= d) continue;
          int side;
          const int t = low_face_type(s, o.fl, o.flo[e], cr[e] == 0, e, side);
          (void)side;
          R phic = o.pa[2 * e] + o.pc[2 * e];
          R F = (R)0;
          if (t == F_INT) F = rho((R)0.5 * (o.al[e] + o.aP)) * phic;
          else if (t == F_INLET || t == F_OUTLET) F = rho(o.aP) * phic;   // open sides: this cell is the fluid one
          gst(Fm, o.fi[2 * e], F);
          if (cr[e] == nn[e] - 1) {
            const int tf = (o.fl & 0x40) ? F_NONE : bcf[2 * e + 1];
            R phf = o.pa[2 * e + 1] + o.pc[2 * e + 1];
            gst(Fm, o.fi[2 * e + 1], (tf == F_INLET || tf == F_OUTLET) ? rho(o.aP) * phf : (R)0);
          }
        }
      });
}

// momentum matrix of a fluid cell: diagonal a_P and explicit b (old-time
// term, upwind convection with the linear-upwind correction, implicit
// diffusion with the explicit transpose term, inlet and wall terms).  One
// cell per thread (register budget), all operands loaded first.
template <typename R>
__global__ void __launch_bounds__(BLOCK) k_assemble(const Slot *slots, const int2 *btab) {
  Block B = block_of(slots, btab);
  const Slot &s = *B.s;
  const SlotCtl &ctl = *B.ctl;
  if (!ctl.active) return;
  const int d = s.dim;
  const int nc = s.nc;
  const R *an = (const R *)s.alpha, *ao = (const R *)s.alpha_old;
  const R *Uo = (const R *)(ctl.mode ? s.U_cr : s.U_vd);
  const R *gU = (const R *)s.gradU, *Fm = (const R *)s.Fm;
  R *aPo = (R *)s.aP, *rAUo = (R *)s.rAU, *bo = (R *)s.b;
  const R Vdt = (R)s.V / (R)ctl.dt, V = (R)s.V;
  const R hh = (R)s.hh, Sh = (R)s.Sh, S = (R)s.S, S2h = (R)s.S2h, ub = (R)ctl.ub;
  const R rho1 = (R)s.rho1, rho2 = (R)s.rho2, mu1 = (R)s.mu1, mu2 = (R)s.mu2;
  auto rho = [&](R x) -> R { return x * rho1 + ((R)1 - x) * rho2; };
  auto mu = [&](R x) -> R { return x * mu1 + ((R)1 - x) * mu2; };
  struct Op {
    Cell c;
    uint8_t fl;   // 0x80: past the end
    R aoP, anP, uP[3], F[6], anb[6], gP[3][3], ga[6][3], gb[6][3];   // gP[c][e] = dU_c/dx_e at the cell
  };
  batched<1, Op>(
      B.lb * BLOCK + (int)threadIdx.x, s.nblocks * BLOCK, nc,
      [&](Op &o, int q) {
        o.fl = 0x80;
        if (q < nc) {
          o.c = cell_at(s, q);
          o.fl = s.flags[q];
        }
      },
      [&](Op &o) {
        if (o.fl & 0xC0) return;
        const int P = o.c.P;
        const Hood hd = hood_of(s, o.fl, o.c);
        o.aoP = gld(ao, P);
        o.anP = gld(an, P);
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) o.uP[cc] = cc < d ? gld(Uo, cc * nc + P) : (R)0;
#pragma unroll
        for (int cc = 0; cc < 3; ++cc)
#pragma unroll
          for (int e = 0; e < 3; ++e) o.gP[cc][e] = (cc < d && e < d) ? gld(gU, (cc * d + e) * nc + P) : (R)0;
#pragma unroll
        for (int f = 0; f < 6; ++f) {
          const int e = f >> 1, n = hd.nb[f];
          o.F[f] = f < 2 * d ? gld(Fm, hd.fi[f]) : (R)0;
          o.anb[f] = gld(an, n);
#pragma unroll
          for (int cc = 0; cc < 3; ++cc) {
            const bool in = f < 2 * d && cc < d;
            o.ga[f][cc] = in ? gld(gU, (cc * d + e) * nc + n) : (R)0;   // dU_cc/dx_e
            o.gb[f][cc] = in ? gld(gU, (e * d + cc) * nc + n) : (R)0;   // dU_e/dx_cc
          }
        }
      },
      [&]() { return true; },
      [&](Op &o) {
        if (o.fl & 0x80) return;
        const Cell &c = o.c;
        if (o.fl & 0x40) {
          gst(aPo, c.P, (R)0);
          gst(rAUo, c.P, (R)0);
          for (int cc = 0; cc < d; ++cc) gst(bo, cc * nc + c.P, (R)0);
          return;
        }
        R rho_o = rho(o.aoP), rho_n = rho(o.anP), mu_n = mu(o.anP);
        R aP = rho_n * Vdt;
        R b[3];
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) b[cc] = cc < d ? (rho_o * o.uP[cc]) * Vdt : (R)0;
#pragma unroll
        for (int f = 0; f < 6; ++f) {
          if (f >= 2 * d) continue;
          const int ty = cell_face(s, o.fl, c, f).type;
          const int e = f >> 1;
          R sg = (f & 1) ? (R)1 : (R)-1;
          if (ty == F_INT) {
            R F = o.F[f], sF = sg * F;
            R muf = mu((R)0.5 * (o.anP + o.anb[f]));
            R D = muf * Sh;
            aP = aP + (sF > (R)0 ? sF : (R)0);
            aP = aP + D;
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) {
              if (cc >= d) continue;
              // gradient component dU_cc/dx_e at the lower and upper cell
              const R glo = (f & 1) ? o.gP[cc][e] : o.ga[f][cc];
              const R ghi = (f & 1) ? o.ga[f][cc] : o.gP[cc][e];
              R lu = F >= (R)0 ? hh * glo : -(hh * ghi);
              b[cc] = b[cc] - sg * (F * lu);
              R tv = (muf * S) * ((R)0.5 * (o.gP[e][cc] + o.gb[f][cc]));
              b[cc] = b[cc] + sg * tv;
            }
          } else if (ty == F_WALL) {
            aP = aP + mu_n * S2h;
          } else if (ty == F_INLET) {
            R F = o.F[f];
            aP = aP + mu_n * S2h;
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) {
              if (cc >= d) continue;
              R ubc = inlet_u<R>(cc, e, sg, ub);
              b[cc] = b[cc] + (mu_n * S2h) * ubc;
              b[cc] = b[cc] - sg * (F * ubc);
            }
          } else if (ty == F_OUTLET) {
            aP = aP + sg * o.F[f];
          }
        }
        gst(aPo, c.P, aP);
        gst(rAUo, c.P, V / aP);
#pragma unroll
        for (int cc = 0; cc < 3; ++cc)
          if (cc < d) gst(bo, cc * nc + c.P, b[cc]);
      });
}

// ---------------------------------------------------------------------------
// PISO corrector
// ---------------------------------------------------------------------------

// cells per thread and batch of the corrector kernels: two in FP32, one in
// FP64 (register budget)
template <typename R>
constexpr int CORR_NB = sizeof(R) == 4 ? 2 : 1;
template <typename R>
constexpr int CORRECT_NB = CORR_NB<R>;

// H = b - sum_N a_N U_N, HbyA = H / a_P.  The operands of every face are
// loaded before any arithmetic (and for all cells of a batch together), the
// arithmetic then runs face by face in the oracle's order.
template <typename R>
__global__ void __launch_bounds__(BLOCK) k_predictor(const Slot *slots, const int2 *btab) {
  Block B = block_of(slots, btab);
  const Slot &s = *B.s;
  const SlotCtl &ctl = *B.ctl;
  if (!ctl.active) return;
  const int d = s.dim;
  const int nc = s.nc;
  const R *an = (const R *)s.alpha, *U = (const R *)(ctl.mode ? s.U_cr : s.U_vd);
  const R *Fm = (const R *)s.Fm, *b = (const R *)s.b, *aPv = (const R *)s.aP;
  R *HbyA = (R *)s.HbyA;
  const R mu1 = (R)s.mu1, mu2 = (R)s.mu2, Sh = (R)s.Sh;
  struct Op {
    Cell c;
    uint8_t fl;   // 0x80: past the end
    R F[6], al[6], Un[6][3], bb[3], aC, aP;
  };
  batched<CORR_NB<R>, Op>(
      B.lb * BLOCK + (int)threadIdx.x, s.nblocks * BLOCK, nc,
      [&](Op &o, int g) {
        o.fl = 0x80;
        if (g < nc) {
          o.c = cell_at(s, g);
          o.fl = s.flags[g];
        }
      },
      [&](Op &o) {
        if (o.fl & 0xC0) return;
        const Hood h = hood_of(s, o.fl, o.c);
        o.aC = gld(an, o.c.P);
        o.aP = gld(aPv, o.c.P);
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) o.bb[cc] = cc < d ? gld(b, cc * nc + o.c.P) : (R)0;
#pragma unroll
        for (int f = 0; f < 6; ++f) {
          o.F[f] = gld(Fm, h.fi[f]);
          o.al[f] = gld(an, h.nb[f]);
#pragma unroll
          for (int cc = 0; cc < 3; ++cc) o.Un[f][cc] = cc < d ? gld(U, cc * nc + h.nb[f]) : (R)0;
        }
      },
      [&]() { return true; },
      [&](Op &o) {
        if (o.fl & 0x80) return;
        const Cell &c = o.c;
        if (o.fl & 0x40) {
          for (int cc = 0; cc < d; ++cc) gst(HbyA, cc * nc + c.P, (R)0);
          return;
        }
        R H[3] = {o.bb[0], o.bb[1], o.bb[2]};
#pragma unroll
        for (int f = 0; f < 6; ++f) {
          if (!((o.fl >> f) & 1u)) continue;   // interior faces only
          R sF = ((f & 1) ? (R)1 : (R)-1) * o.F[f];
          R m = (R)0.5 * (o.aC + o.al[f]);
          R D = (m * mu1 + ((R)1 - m) * mu2) * Sh;
          R aN = (sF < (R)0 ? sF : (R)0) - D;
#pragma unroll
          for (int cc = 0; cc < 3; ++cc)
            if (cc < d) H[cc] = H[cc] - aN * o.Un[f][cc];
        }
#pragma unroll
        for (int cc = 0; cc < 3; ++cc)
          if (cc < d) gst(HbyA, cc * nc + c.P, H[cc] / o.aP);
      });
}

// predicted face flux phiH of the faces each cell owns (the low face per
// direction, the far face on the last layer): interpolated HbyA plus the
// surface-tension term, inlet and outlet values on open sides
template <typename R>
__global__ void __launch_bounds__(BLOCK) k_phiH(const Slot *slots, const int2 *btab) {
  Block B = block_of(slots, btab);
  const Slot &s = *B.s;
  const SlotCtl &ctl = *B.ctl;
  if (!ctl.active) return;
  const int d = s.dim;
  const int nc = s.nc;
  const R *HbyA = (const R *)s.HbyA, *rAU = (const R *)s.rAU, *kap = (const R *)s.kappa, *a = (const R *)s.alpha;
  double *phiH = s.phiH;
  const double S = s.S, ub = ctl.ub, h = s.h, sigma = s.sigma;
  const int with_st = ctl.with_st;
  const int nn[3] = {s.nx, s.ny, s.nz};
  int bcf[6];
  for (int f = 0; f < 6; ++f) bcf[f] = s.bcf[f];
  struct Op {
    Cell c;
    uint8_t fl;   // 0x80: past the end
    int fi[6];
    R hP[3], hn[3], rP, rn[3], kP, kn[3], aP, an[3];   // at the cell and below it per direction
  };
  batched<CORR_NB<R>, Op>(
      B.lb * BLOCK + (int)threadIdx.x, s.nblocks * BLOCK, nc,
      [&](Op &o, int g) {
        o.fl = 0x80;
        if (g < nc) {
          o.c = cell_at(s, g);
          o.fl = s.flags[g];
        }
      },
      [&](Op &o) {
        if (o.fl & 0x80) return;
        const Hood hd = hood_of(s, o.fl, o.c);
#pragma unroll
        for (int f = 0; f < 6; ++f) o.fi[f] = hd.fi[f];
        if (o.fl & 0x40) return;
        const int P = o.c.P;
        o.rP = gld(rAU, P);
        o.kP = gld(kap, P);
        o.aP = gld(a, P);
#pragma unroll
        for (int e = 0; e < 3; ++e) {
          const int lo = hd.nb[2 * e];
          o.hP[e] = e < d ? gld(HbyA, e * nc + P) : (R)0;
          o.hn[e] = e < d ? gld(HbyA, e * nc + lo) : (R)0;
          o.rn[e] = gld(rAU, lo);
          o.kn[e] = gld(kap, lo);
          o.an[e] = gld(a, lo);
        }
      },
      [&]() { return true; },
      [&](Op &o) {
        if (o.fl & 0x80) return;
        const bool fluid = !(o.fl & 0x40);
        const int cr[3] = {o.c.i, o.c.j, o.c.k};
        // value of an open side face of this fluid cell (orientation sign sf
        // seen from the cell)
        auto open = [&](int type, int e, double sf) -> double {
          if (type == F_INLET) return -sf * (ub * S);
          if (type == F_OUTLET) return (double)o.hP[e] * S;
          return 0.0;
        };
#pragma unroll
        for (int e = 0; e < 3; ++e) {
          if (e >= d) continue;
          double ph = 0.0;
          if (fluid && ((o.fl >> (2 * e)) & 1u)) {
            ph = (0.5 * ((double)o.hn[e] + (double)o.hP[e])) * S;
            if (with_st) {
              double rAUf = 0.5 * ((double)o.rn[e] + (double)o.rP);
              double st = (sigma * (0.5 * ((double)o.kn[e] + (double)o.kP))) * (((double)o.aP - (double)o.an[e]) / h);
              ph = ph + (rAUf * st) * S;
            }
          } else if (fluid && cr[e] == 0) {
            ph = open(bcf[2 * e], e, -1.0);
          }
          gst(phiH, o.fi[2 * e], ph);
          if (cr[e] == nn[e] - 1) gst(phiH, o.fi[2 * e + 1], fluid ? open(bcf[2 * e + 1], e, 1.0) : 0.0);
        }
      });
}

// rhs = -div(phiH), r = rhs - M p, Jacobi diagonal; operands first
template <typename R>
__global__ void __launch_bounds__(BLOCK) k_pressure_setup(const Slot *slots, const int2 *btab) {
  using T = R;
  Block B = block_of(slots, btab);
  const Slot &s = *B.s;
  const Grid G = grid_of(s);
  const SlotCtl &ctl = *B.ctl;
  if (!ctl.active) return;
  const int d = G.dim;
  const R *rAU = (const R *)s.rAU;
  const double *phiH = s.phiH;
  const double *p = ctl.mode ? s.p_cr : s.p_vd;
  const bool mixed = s.precision != 0;
  T *r = (T *)s.cr[0], *invD = (T *)s.invD, *e = (T *)s.e;
  double *rhsv = s.rhs, *Mpv = s.Mp;
  const uint8_t *flags = s.flags;
  double red[3] = {0.0, 0.0, 0.0};   // |rhs|^2, |rhs - M p|^2, sum p
  struct Op {
    Cell c;
    uint8_t fl;   // 0x80: past the end
    double ph[6], pP, pn[6];
    R rP, rn[6];
  };
  batched<CORR_NB<R>, Op>(
      B.lb * BLOCK + (int)threadIdx.x, G.nblocks * BLOCK, G.nc,
      [&](Op &o, int g) {
        o.fl = 0x80;
        if (g < G.nc) {
          o.c = cell_at(G, g);
          o.fl = flags[g];
        }
      },
      [&](Op &o) {
        if (o.fl & 0xC0) return;
        const Hood hd = hood_of(s, o.fl, o.c);
        o.pP = gld(p, o.c.P);
        o.rP = gld(rAU, o.c.P);
#pragma unroll
        for (int f = 0; f < 6; ++f) {
          o.ph[f] = f < 2 * d ? gld(phiH, hd.fi[f]) : 0.0;
          o.pn[f] = gld(p, hd.nb[f]);
          o.rn[f] = gld(rAU, hd.nb[f]);
        }
      },
      [&]() { return true; },
      [&](Op &o) {
        if (o.fl & 0x80) return;
        const Cell &c = o.c;
        if (o.fl & 0x40) {
          gst(rhsv, c.P, 0.0);
          gst(Mpv, c.P, 0.0);
          gst(r, c.P, (T)0);
          gst(invD, c.P, (T)0);
          if (mixed) gst(e, c.P, (T)0);
          return;
        }
        double acc = 0.0;
        T dg = (T)0;
#pragma unroll
        for (int f = 0; f < 6; ++f) {
          if (f >= 2 * d) continue;
          acc = acc + ((f & 1) ? 1.0 : -1.0) * o.ph[f];
          if ((o.fl >> f) & 1u) dg = dg + ((T)0.5 * ((T)o.rP + (T)o.rn[f])) * (T)G.Sh;
          else if (((G.outlet >> f) & 1u) && on_edge(G, c, f)) dg = dg + (T)o.rP * (T)G.S2h;
        }
        double rhs = -acc;
        double xn[6], rn[6];
#pragma unroll
        for (int f = 0; f < 6; ++f) {
          xn[f] = o.pn[f];
          rn[f] = (double)o.rn[f];
        }
        double Mp = matvec_pre<double>(G, c, o.fl, o.pP, (double)o.rP, xn, rn);
        double r64 = rhs - Mp;
        T rr = (T)r64;
        gst(rhsv, c.P, rhs);
        gst(Mpv, c.P, Mp);
        gst(r, c.P, rr);
        gst(invD, c.P, (T)1 / dg);
        if (mixed) gst(e, c.P, (T)0);
        red[0] = red[0] + rhs * rhs;
        red[1] = red[1] + (mixed ? r64 * r64 : (double)(rr * rr));
        red[2] = red[2] + o.pP;
      });
  put_partials<0u>(s, B.lb, CH_SETUP, red);
}

// Norms of the pressure equation and the initial convergence test, from the
// set-up's partials summed in every block (the same fixed order in each);
// block 0 of the slot records them.  p = 0 when the right-hand side
// vanishes (the unique solution).
__global__ void __launch_bounds__(BLOCK) k_setup_fin(const Slot *slots, const int2 *btab) {
  Block B = block_of(slots, btab);
  const Slot &s = *B.s;
  const SlotCtl &ctl = *B.ctl;
  if (!ctl.active) return;
  double v[3];
  get_totals<0u>(s, CH_SETUP, v);
  const double bn = sqrt(v[0]);
  if (B.lb == 0 && threadIdx.x == 0) {
    SlotState *st = B.st;
    double rn = sqrt(v[1]);
    st->pbar = v[2] / (double)s.n_fluid;
    st->it = 0;
    st->zero_rhs = bn == 0.0;
    st->done = (bn == 0.0) || (rn <= ctl.rtol * bn);
    st->rn = rn;
    st->bn64 = bn;
    st->rn64 = rn;
    st->ref_solve = 0;
    st->stalled = 0;
    // mixed precision: the FP32 inner system is M e = r, measured against |r|
    st->bn = s.precision != 0 ? rn : bn;
    st->tgt = inner_target(ctl, bn, rn);
  }
  if (bn != 0.0) return;
  double *p = ctl.mode ? s.p_cr : s.p_vd;
  for_cells(s, B.lb, [&](const Cell &c) { p[c.P] = 0.0; });
}

// normalised residual E = sum|b - Mp| / (sum(|Mp - M pbar| + |b - M pbar|) + 1e-20)
template <typename R>
__global__ void __launch_bounds__(BLOCK) k_normres(const Slot *slots, const int2 *btab) {
  Block B = block_of(slots, btab);
  const Slot &s = *B.s;
  const Grid G = grid_of(s);
  const uint8_t *flags = s.flags;
  const SlotCtl &ctl = *B.ctl;
  if (!ctl.active || ctl.mode != 1) return;
  const R *rAU = (const R *)s.rAU;
  const double pbar = B.st->pbar;
  double red[2] = {0.0, 0.0};
  for_cells(G, B.lb, [&](const Cell &c) {
    uint8_t fl = flags[c.P];
    if (fl & 0x40) return;
    double Mpb = matvec_row<double, R>(G, rAU, c, fl, [&](int) { return pbar; });
    double rhs = s.rhs[c.P], Mp = s.Mp[c.P];
    red[0] = red[0] + fabs(rhs - Mp);
    red[1] = red[1] + (fabs(Mp - Mpb) + fabs(rhs - Mpb));
  });
  put_partials<0u>(s, B.lb, CH_NORM, red);
}

__global__ void __launch_bounds__(BLOCK) k_norm_fin(const Slot *slots) {
  const Slot &s = slots[blockIdx.x];
  if (!s.ctl) return;   // unused table entry
  const SlotCtl &ctl = *s.ctl;
  if (!ctl.active || ctl.mode != 1) return;
  double v[2];
  get_totals<0u>(s, CH_NORM, v);
  if (threadIdx.x == 0) s.st->E = v[0] / (v[1] + 1e-20);
}


// grid-wide kernels over the bodies of cg_bodies.h
template <typename R>
__global__ void __launch_bounds__(BLOCK) k_cg_init(const Slot *slots, const int2 *btab) {
  Block B = block_of(slots, btab);
  if (!B.ctl->active || B.st->done) return;
  cg_init_body<R>(*B.s, B.lb);
}

template <typename R>
__global__ void __launch_bounds__(BLOCK) k_cg(const Slot *slots, const int2 *btab, int it, unsigned long long *ts) {
  Stamp stamp(ts);
  Block B = block_of(slots, btab);
  if (!B.ctl->active || B.st->done) return;
  if (cg_iter_body<R>(*B.s, B.lb, it)) stamp.done();
}

template <typename R>
__global__ void __launch_bounds__(BLOCK) k_refine_x(const Slot *slots, const int2 *btab) {
  Block B = block_of(slots, btab);
  refine_x_body<R>(*B.s, *B.ctl, B.lb);
}

template <typename R>
__global__ void __launch_bounds__(BLOCK) k_refine_res(const Slot *slots, const int2 *btab) {
  Block B = block_of(slots, btab);
  refine_res_body<R>(*B.s, *B.ctl, B.lb);
}

__global__ void __launch_bounds__(BLOCK) k_refine_fin(const Slot *slots) {
  const Slot &s = slots[blockIdx.x];
  if (!s.ctl) return;   // unused table entry
  refine_fin_body(s);
}

// phi = phiH - rAU_f S/h (p_hi - p_lo); u = HbyA + rAU * mean of the face
// accelerations (f - grad p) of the two faces of each direction.  Operands
// first, as in k_predictor; each thread writes the faces its cell owns (the
// low face per direction, and the far face on the last layer).
template <typename R>
__global__ void __launch_bounds__(BLOCK) k_correct(const Slot *slots, const int2 *btab, int corr) {
  Block B = block_of(slots, btab);
  const Slot &s = *B.s;
  const SlotCtl &ctl = *B.ctl;
  if (!ctl.active) return;
  const int d = s.dim;
  const int nc = s.nc;
  const double *p = ctl.mode ? s.p_cr : s.p_vd;
  const double *phiH = s.phiH;
  const R *rAU = (const R *)s.rAU, *HbyA = (const R *)s.HbyA;
  const R *kap = (const R *)s.kappa, *a = (const R *)s.alpha;
  R *phi = (R *)(ctl.mode ? s.phi_cr : s.phi_vd);
  R *U = (R *)(ctl.mode ? s.U_cr : s.U_vd);
  R *Us = (R *)s.U_sum;
  const double Sh = s.Sh, S2h = s.S2h, h = s.h, hh = s.hh, sigma = s.sigma;
  const int with_st = ctl.with_st;
  const bool acc_sum = corr == ctl.last_corr && ctl.mode == 1;
  const int nn[3] = {s.nx, s.ny, s.nz};
  int bcf[6];
  for (int f = 0; f < 6; ++f) bcf[f] = s.bcf[f];
  bool bad = false;
  struct Op {
    Cell c;
    uint8_t fl;   // 0x80: past the end
    int fi[6];
    double pP, pn[6], ph[6];   // ph: phiH of the low face, and of the far face on the last layer
    R rP, rn[3], kP, kn[6], aP, an[6], hb[3], us[3];
  };
  batched<CORRECT_NB<R>, Op>(
      B.lb * BLOCK + (int)threadIdx.x, s.nblocks * BLOCK, nc,
      [&](Op &o, int g) {
        o.fl = 0x80;
        if (g < nc) {
          o.c = cell_at(s, g);
          o.fl = s.flags[g];
        }
      },
      [&](Op &o) {
        if (o.fl & 0x80) return;
        const Cell &c = o.c;
        const Hood hd = hood_of(s, o.fl, c);
        const int cr[3] = {c.i, c.j, c.k};
#pragma unroll
        for (int f = 0; f < 6; ++f) o.fi[f] = hd.fi[f];
#pragma unroll
        for (int e = 0; e < 3; ++e) {
          o.ph[2 * e] = 0.0;
          o.ph[2 * e + 1] = 0.0;
          if (e < d) {
            o.ph[2 * e] = gld(phiH, hd.fi[2 * e]);
            if (cr[e] == nn[e] - 1) o.ph[2 * e + 1] = gld(phiH, hd.fi[2 * e + 1]);
          }
        }
        if (acc_sum)
#pragma unroll
          for (int cc = 0; cc < 3; ++cc) o.us[cc] = cc < d ? gld(Us, cc * nc + c.P) : (R)0;
        if (o.fl & 0x40) return;
        o.pP = gld(p, c.P);
        o.rP = gld(rAU, c.P);
        o.kP = gld(kap, c.P);
        o.aP = gld(a, c.P);
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) o.hb[cc] = cc < d ? gld(HbyA, cc * nc + c.P) : (R)0;
#pragma unroll
        for (int f = 0; f < 6; ++f) {
          o.pn[f] = gld(p, hd.nb[f]);
          o.kn[f] = gld(kap, hd.nb[f]);
          o.an[f] = gld(a, hd.nb[f]);
          if (!(f & 1)) o.rn[f >> 1] = gld(rAU, hd.nb[f]);
        }
      },
      [&]() { return true; },
      [&](Op &o) {
        if (o.fl & 0x80) return;
        const Cell &c = o.c;
        const bool fluid = !(o.fl & 0x40);
        const int cr[3] = {c.i, c.j, c.k};
        // owned faces: the low face of direction e has the neighbour below
        // as lo and this cell as hi; it is interior when both are fluid, an
        // outlet when this fluid cell lies on an outlet side
#pragma unroll
        for (int e = 0; e < 3; ++e) {
          if (e >= d) continue;
          double ph = o.ph[2 * e];
          if (fluid && ((o.fl >> (2 * e)) & 1u)) {
            double cf = (0.5 * ((double)o.rn[e] + (double)o.rP)) * Sh;
            ph = ph - cf * (o.pP - o.pn[2 * e]);
          } else if (fluid && cr[e] == 0 && bcf[2 * e] == F_OUTLET) {
            double cf = (double)o.rP * S2h;
            ph = ph + -1.0 * (cf * o.pP);
          }
          gst(phi, o.fi[2 * e], (R)ph);
          if (cr[e] == nn[e] - 1) {
            double pf = o.ph[2 * e + 1];
            if (fluid && bcf[2 * e + 1] == F_OUTLET) {
              double cf = (double)o.rP * S2h;
              pf = pf + 1.0 * (cf * o.pP);
            }
            gst(phi, o.fi[2 * e + 1], (R)pf);
          }
        }
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) {
          if (cc >= d) continue;
          R u = (R)0;
          if (fluid) {
            double qv[2];
#pragma unroll
            for (int sd = 0; sd < 2; ++sd) {
              const int f = 2 * cc + sd;
              double qq = 0.0;
              if ((o.fl >> f) & 1u) {
                // lo and hi cells of the face
                const double plo = sd ? o.pP : o.pn[f], phi_ = sd ? o.pn[f] : o.pP;
                double ff = 0.0;
                if (with_st) {
                  const R klo = sd ? o.kP : o.kn[f], khi = sd ? o.kn[f] : o.kP;
                  const R alo = sd ? o.aP : o.an[f], ahi = sd ? o.an[f] : o.aP;
                  ff = (sigma * (0.5 * ((double)klo + (double)khi))) * (((double)ahi - (double)alo) / h);
                }
                qq = ff - (phi_ - plo) / h;
              } else if (cr[cc] == (sd ? nn[cc] - 1 : 0) && bcf[f] == F_OUTLET) {
                double pplus = sd ? 0.0 : o.pP, pminus = sd ? o.pP : 0.0;
                qq = -(pplus - pminus) / hh;
              }
              qv[sd] = qq;
            }
            double uu = (double)o.hb[cc] + (double)o.rP * (0.5 * (qv[0] + qv[1]));
            u = (R)uu;
            if (!(uu == uu) || fabs(uu) > 1e30) bad = true;
          }
          gst(U, cc * nc + c.P, u);
          if (acc_sum) gst(Us, cc * nc + c.P, o.us[cc] + u);
        }
      });
  if (bad) B.st->nonfinite = 1;
}

// U = U_vd + (1/N) sum u_cr, p = p_vd + p_cr
template <typename R>
__global__ void __launch_bounds__(BLOCK) k_finalize(const Slot *slots, const int2 *btab) {
  Block B = block_of(slots, btab);
  const Slot &s = *B.s;
  const SlotCtl &ctl = *B.ctl;
  if (!ctl.active || ctl.mode != 1) return;
  const R *Uvd = (const R *)s.U_vd, *Us = (const R *)s.U_sum;
  R *U = (R *)s.U;
  for_cells(s, B.lb, [&](const Cell &c) {
    for (int cc = 0; cc < s.dim; ++cc) {
      int x = cc * s.nc + c.P;
      U[x] = Uvd[x] + Us[x] / (R)ctl.n_sub;
    }
    s.p[c.P] = s.p_vd[c.P] + s.p_cr[c.P];
  });
}

template <typename R>
__global__ void __launch_bounds__(BLOCK) k_zero_usum(const Slot *slots, const int2 *btab) {
  Block B = block_of(slots, btab);
  const Slot &s = *B.s;
  if (!B.ctl->active || B.ctl->mode != 1 || B.ctl->substep != 0) return;
  R *Us = (R *)s.U_sum;
  for_cells(s, B.lb, [&](const Cell &c) {
    for (int cc = 0; cc < s.dim; ++cc) Us[cc * s.nc + c.P] = (R)0;
  });
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------

#define GRID(L) dim3((unsigned)(L).nblocks), dim3(BLOCK), 0, (L).stream
#define SLOTGRID(L) dim3((unsigned)(L).nslots), dim3(BLOCK), 0, (L).stream

template <typename R> void launch_copy_phi_prev(const Launch &L) {
  hipLaunchKernelGGL(k_copy_phi_prev<R>, GRID(L), L.slots, L.btab);
}

template <typename R> void launch_normals(const Launch &L, bool curvature) {
  int only_cr = curvature ? 1 : 0;
  hipLaunchKernelGGL(k_grad_alpha<R>, GRID(L), L.slots, L.btab, only_cr);
  hipLaunchKernelGGL(k_face_normals<R>, GRID(L), L.slots, L.btab, only_cr);
  if (curvature) hipLaunchKernelGGL(k_curvature<R>, GRID(L), L.slots, L.btab);
}

template <typename R> void launch_advect(const Launch &L, int npass) {
  hipLaunchKernelGGL(k_mules_flux<R>, GRID(L), L.slots, L.btab);
  hipLaunchKernelGGL(k_mules_limiter<R>, GRID(L), L.slots, L.btab);
  hipLaunchKernelGGL(k_mules_update<R>, GRID(L), L.slots, L.btab);
  for (int m = 2; m <= npass; ++m) {
    hipLaunchKernelGGL(k_mules_limiter_again<R>, GRID(L), L.slots, L.btab, m);
    hipLaunchKernelGGL(k_mules_update_again<R>, GRID(L), L.slots, L.btab, m);
  }
  hipLaunchKernelGGL(k_transport_fin, SLOTGRID(L), L.slots);
}

template <typename R> void launch_assemble(const Launch &L) {
  hipLaunchKernelGGL(k_grad_u<R>, GRID(L), L.slots, L.btab);
  hipLaunchKernelGGL(k_mass_flux<R>, GRID(L), L.slots, L.btab);
  hipLaunchKernelGGL(k_assemble<R>, GRID(L), L.slots, L.btab);
}

template <typename R> void launch_predictor(const Launch &L) {
  hipLaunchKernelGGL(k_predictor<R>, GRID(L), L.slots, L.btab);
  hipLaunchKernelGGL(k_phiH<R>, GRID(L), L.slots, L.btab);
}

template <typename R> void launch_pressure_setup(const Launch &L, bool normres) {
  hipLaunchKernelGGL(k_pressure_setup<R>, GRID(L), L.slots, L.btab);
  hipLaunchKernelGGL(k_setup_fin, GRID(L), L.slots, L.btab);
  if (normres) {
    hipLaunchKernelGGL(k_normres<R>, GRID(L), L.slots, L.btab);
    hipLaunchKernelGGL(k_norm_fin, SLOTGRID(L), L.slots);
  }
}

template <typename R> void launch_cg_init(const Launch &L) {
  hipLaunchKernelGGL(k_cg_init<R>, GRID(L), L.slots, L.btab);
}

template <typename R> void launch_cg_iters(const Launch &L, int it0, int n, unsigned long long *ts) {
  for (int x = 0; x < n; ++x) hipLaunchKernelGGL(k_cg<R>, GRID(L), L.slots, L.btab, it0 + x, ts);
}

template <typename R> void launch_refine(const Launch &L) {
  hipLaunchKernelGGL(k_refine_x<R>, GRID(L), L.slots, L.btab);
  hipLaunchKernelGGL(k_refine_res<R>, GRID(L), L.slots, L.btab);
  hipLaunchKernelGGL(k_refine_fin, SLOTGRID(L), L.slots);
}

template <typename R> void launch_correct(const Launch &L, int corr) {
  hipLaunchKernelGGL(k_correct<R>, GRID(L), L.slots, L.btab, corr);
}

template <typename R> void launch_finalize(const Launch &L) {
  hipLaunchKernelGGL(k_finalize<R>, GRID(L), L.slots, L.btab);
}

template <typename R> void launch_zero_usum(const Launch &L) {
  hipLaunchKernelGGL(k_zero_usum<R>, GRID(L), L.slots, L.btab);
}

void launch_ctl_update(const Launch &L, const CtlUpdate &u) {
  hipLaunchKernelGGL(k_ctl_update, dim3(1), dim3(64), 0, L.stream, const_cast<Slot *>(L.slots), u);
}

void launch_gather_states(const Launch &L, int nslots, SlotState *out) {
  hipLaunchKernelGGL(k_gather_states, dim3((nslots + 63) / 64), dim3(64), 0, L.stream, L.slots, nslots, out);
}

// measurement only: span (earliest start, latest end) of each stamp region;
// workgroups that stamped nothing (zero words) are skipped.  Regions of the
// groups of `per` regions whose bit is set in `clear` are zeroed once read.
__global__ void __launch_bounds__(BLOCK) k_ts_span(unsigned long long *ts, unsigned long long *out, int per,
                                                   unsigned long long clear) {
  unsigned long long *r = ts + (size_t)blockIdx.x * TS_WORDS;
  const bool zero = (clear >> (blockIdx.x / (unsigned)per)) & 1ull;
  unsigned long long lo = ~0ull, hi = 0ull;
  for (int b = threadIdx.x; b < TS_WORDS / 2; b += BLOCK) {
    const unsigned long long a = r[2 * b], e = r[2 * b + 1];
    if (a != 0ull && a < lo) lo = a;
    if (e > hi) hi = e;
    if (zero) {
      r[2 * b] = 0ull;
      r[2 * b + 1] = 0ull;
    }
  }
  __shared__ unsigned long long sl[BLOCK], sh[BLOCK];
  sl[threadIdx.x] = lo;
  sh[threadIdx.x] = hi;
  __syncthreads();
  for (int w = BLOCK / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      if (sl[threadIdx.x + w] < sl[threadIdx.x]) sl[threadIdx.x] = sl[threadIdx.x + w];
      if (sh[threadIdx.x + w] > sh[threadIdx.x]) sh[threadIdx.x] = sh[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[2 * blockIdx.x] = sl[0];
    out[2 * blockIdx.x + 1] = sh[0];
  }
}

void launch_ts_span(unsigned long long *ts, int nregions, unsigned long long *out, int per, unsigned long long clear,
                    hipStream_t stream) {
  hipLaunchKernelGGL(k_ts_span, dim3((unsigned)nregions), dim3(BLOCK), 0, stream, ts, out, per, clear);
}

void launch_state_reset(const Launch &L, int nslots) {
  hipLaunchKernelGGL(k_state_reset, dim3((nslots + 63) / 64), dim3(64), 0, L.stream, L.slots, nslots);
}

#define INST(R)                                                   \
  template void launch_copy_phi_prev<R>(const Launch &);          \
  template void launch_normals<R>(const Launch &, bool);          \
  template void launch_advect<R>(const Launch &, int);            \
  template void launch_assemble<R>(const Launch &);               \
  template void launch_predictor<R>(const Launch &);              \
  template void launch_pressure_setup<R>(const Launch &, bool);   \
  template void launch_cg_init<R>(const Launch &);                \
  template void launch_cg_iters<R>(const Launch &, int, int, unsigned long long *); \
  template void launch_refine<R>(const Launch &);                 \
  template void launch_correct<R>(const Launch &, int);           \
  template void launch_finalize<R>(const Launch &);               \
  template void launch_zero_usum<R>(const Launch &);

INST(double)
INST(float)

}  // namespace oscar
