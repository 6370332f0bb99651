// Geometric multigrid preconditioner for the pressure equation of the PISO
// correctors (Section 2.2) on the voxel grid, and the conjugate gradient it
// preconditions (Hestenes-Stiefel recurrences: one search-direction launch
// plus one V-cycle per iteration).
//
// Hierarchy: coarse cell = 2 x 2 (x 2) block of the finer level.  A coarse
// face coefficient is a fixed fraction of the sum of the fine face
// coefficients crossing it (the piecewise-constant Galerkin product, scaled
// by one half to match a rediscretisation on the doubled spacing, by 0.8
// (2D) or 0.9 (3D) on the first level); outlet coefficients are aggregated
// the same way.
// Cycle: Jacobi sweeps (damped by 0.9 on the fine grid, plain on the coarse
// levels) from zero before restriction and after prolongation, one on the
// fine grid, one or two (the host's per-level choice, MGInfo::nu2) on the
// grid-wide coarse levels and MG_TAIL_NU on the levels of the
// single-workgroup tail,
// the exact solve on the coarsest level (at most a few dozen cells) with its
// dense inverse, formed at setup; pre- and post-smoothing are the same
// sweeps, so the cycle is a symmetric linear operator, as the conjugate
// gradient needs.  A second sweep is fused into the same launch: each cell
// re-evaluates the first sweep at its neighbours (a radius-2 stencil) rather
// than waiting for another launch.
//
// Execution: the pre-smoothing kernels walk their level in tile order (the
// 2^dim cells of one coarser cell are lanes of the same wavefront), so
// the restriction of the residual is a lane-shuffle sum inside the same
// kernel and no restriction launch or residual array exists.  The small
// levels (from the one the host marks as the tail down to the coarsest) run
// inside one workgroup.  No atomics.
#include "device_common.h"
#include "cg_bodies.h"

namespace oscar {

// Smoothing sweeps before and after the coarse correction on the grid-wide
// levels (below the fine grid, above the tail): one, or two where the host
// sets the level's bit in MGInfo::nu2.  The second sweep is evaluated at the
// neighbours in the same launch (sweep_matvec: a radius-2 stencil, each
// operand loaded once), which makes these latency-bound kernels slower.
// Measured (mixed / FP64 step time; A/B on one box each):
//   128 x 64 x 64 channel: level 2 twice against once -1.5 % / +0.9 % (CG
//     iterations 566 -> 516), levels 1 and 2 against level 2 alone -0.9 % /
//     -1.3 % (516 -> 470);
//   256^3 sphere pack: levels from 2 on against none -9 % / -13 % (2006 ->
//     1741), all against levels from 2 on -3.1 % / -1.2 % (1741 -> 1488);
//   1024 x 512 micromodel (2D): level 2 +1 % / +5 %, levels 2 and 3 +2 % /
//     +7 %.
// Hence two sweeps on every grid-wide level in 3D, one in 2D.
// Sweeps on the levels of the single-workgroup tail, where they run out of
// LDS with barriers between them: two instead of one cut the CG iterations
// of a mixed step 12 % on the 128 x 64 x 64 channel, 11 % on the 1024 x 512
// micromodel and 13 % on the 256^3 sphere pack for 2.3 us more per cycle
// (step time -7 %, -5 %, -10 %); three gain a little more on the sphere
// pack and lose on the other two.
constexpr int MG_TAIL_NU = 2;
constexpr int MG_TAIL_THREADS = 1024;   // workgroup of the tail kernel
constexpr int MG_INV_THREADS = 1024;    // workgroup of the coarse inversion
// Jacobi damping: plain Jacobi (1.0) on the coarse levels, 0.9 on the fine
// grid.  Every level's operator has non-positive off-diagonal entries and a
// diagonal at least the sum of their magnitudes (the fine one by
// construction, a coarse one as a scaled sum of those), so 2 D - A is
// positive semi-definite and the symmetric cycle stays positive definite up
// to a damping of 1.  Measured (total CG iterations of one mixed step, the
// coarse scale below): coarse damping 1.0 against 0.9 cut them 8 % on the
// 128 x 64 x 64 channel and the 1024 x 512 micromodel and 11 % on the 256^3
// sphere pack (0.95 lies between); the fine grid needs damping: 1.0 there
// multiplied the iterations by five, 0.85 and 0.95 were worse than 0.9 on
// the channel.
constexpr double MG_OMEGA = 1.0;
constexpr double MG_OMEGA_FINE = 0.9;
// Scale of a coarse coefficient against the sum of the fine ones crossing
// it: one half matches a rediscretisation on the doubled spacing and is
// kept on the deeper levels; the first level takes a stiffer 0.8 (with the
// damping above: 0.62 -> 0.8 cut the iterations 4 % on the channel, 1 % on
// the micromodel, 0.3 % on the sphere pack; 0.7-0.9 lie within 1 %, 0.55 was
// worse everywhere; larger scales on the deeper levels cost iterations on
// the sphere pack and the micromodel).  With two sweeps on the grid-wide
// coarse levels (3D), 0.9 on the first level cut the channel's iterations
// 470 -> 454 (mixed step -3.6 %, FP64 -2.9 %) for +0.5 % on the sphere pack
// (0.95 and 1.0: -4.8 % and -4.5 % on the channel, +1.2 % and +1.8 % on the
// pack); in 2D 0.9 cost the micromodel 2 %.
constexpr double MG_SCALE = 0.5;
constexpr double MG_SCALE1_2D = 0.8;
constexpr double MG_SCALE1_3D = 0.9;


struct LCell {
  int P, i, j, k;
};

__device__ __forceinline__ LCell lcell(const MGLevel &L, int g) {
  LCell c;
  unsigned ug = (unsigned)g, nx = (unsigned)L.nx, ny = (unsigned)L.ny;
  unsigned row = ug / nx;
  c.P = g;
  c.i = (int)(ug - row * nx);
  unsigned k = row / ny;
  c.j = (int)(row - k * ny);
  c.k = (int)k;
  return c;
}

// A kernel's register copy of one level: dimensions and array pointers.
template <typename T>
struct LV {
  int nx, ny, nz, nxy, nc;
  const T *cf[3];
  const T *cout, *invD;
  T *b, *x, *t;
};

template <typename T>
__device__ __forceinline__ LV<T> lview(const MGLevel &L) {
  LV<T> v;
  v.nx = L.nx;
  v.ny = L.ny;
  v.nz = L.nz;
  v.nxy = L.nxy;
  v.nc = L.nc;
  for (int e = 0; e < 3; ++e) v.cf[e] = (const T *)L.cf[e];
  v.cout = (const T *)L.cout;
  v.invD = (const T *)L.invD;
  v.b = (T *)L.b;
  v.x = (T *)L.x;
  v.t = (T *)L.t;
  return v;
}

__device__ __forceinline__ LCell lcell(int nx, int ny, int g) {
  LCell c;
  unsigned ug = (unsigned)g, row = ug / (unsigned)nx;
  c.P = g;
  c.i = (int)(ug - row * (unsigned)nx);
  unsigned k = row / (unsigned)ny;
  c.j = (int)(row - k * (unsigned)ny);
  c.k = (int)k;
  return c;
}

// Index arithmetic on the tail levels (at most MG_TAIL_CELLS cells, far
// below 2^24): a quotient by d from the float reciprocal of d, exact up to
// one for any dividend below 2^24 (the product's relative error is a few
// units of 2^-24), corrected by the sign and size of the remainder, and
// products by 24-bit multiplies.  Both are full-rate VALU operations where
// 32-bit division and multiplication take sequences of quarter-rate ones.
struct Div24 {
  float r;      // 1 / d
  unsigned d;   // the divisor, 1 <= d < 2^24
};
__device__ __forceinline__ Div24 div24(int d) {
  Div24 q;
  q.d = (unsigned)d;
  q.r = 1.0f / (float)d;
  return q;
}
__device__ __forceinline__ unsigned quot24(unsigned g, const Div24 &D) {
  unsigned q = (unsigned)((float)g * D.r);
  const int r = (int)(g - __umul24(q, D.d));
  if (r < 0) q -= 1u;
  else if (r >= (int)D.d) q += 1u;
  return q;
}
// lcell on a tail level (DX, DY: the divisors nx and ny)
__device__ __forceinline__ LCell lcell24(const Div24 &DX, const Div24 &DY, int g) {
  LCell c;
  const unsigned ug = (unsigned)g, row = quot24(ug, DX);
  c.P = g;
  c.i = (int)(ug - __umul24(row, DX.d));
  const unsigned k = quot24(row, DY);
  c.j = (int)(row - __umul24(k, DY.d));
  c.k = (int)k;
  return c;
}

// (A x)_P on a coarse level, unrolled over the DIM directions.  xv(n, e,
// side) returns x at cell n: the neighbour across the low (side = -1) or
// high (+1) face of direction e, or the cell itself (side = 0), which is
// also read where a neighbour is missing (its coefficient is zero), so all
// loads are unconditional.
template <int DIM, typename T, class XV>
__device__ __forceinline__ T lmatvec(const LV<T> &L, const LCell &c, XV &&xv) {
  const int st[3] = {1, L.nx, L.nxy};
  const int q[3] = {c.i, c.j, c.k};
  const int n[3] = {L.nx, L.ny, L.nz};
  const T xP = xv(c.P, 0, 0);
  T cl[DIM], ch[DIM], xl[DIM], xh[DIM];
#pragma unroll
  for (int e = 0; e < DIM; ++e) {
    const bool lo = q[e] > 0, hi = q[e] < n[e] - 1;
    const int pl = lo ? c.P - st[e] : c.P, ph = hi ? c.P + st[e] : c.P;
    cl[e] = L.cf[e][c.P];
    const T chv = L.cf[e][ph];
    ch[e] = hi ? chv : (T)0;
    xl[e] = xv(pl, e, lo ? -1 : 0);
    xh[e] = xv(ph, e, hi ? 1 : 0);
  }
  const T co = L.cout[c.P];
  T acc = (T)0;
#pragma unroll
  for (int e = 0; e < DIM; ++e) {
    acc = acc + cl[e] * (xP - xl[e]);
    acc = acc + ch[e] * (xP - xh[e]);
  }
  acc = acc + co * xP;
  return acc;
}

// the cell next to c across the low (side = -1) or high (+1) face of
// direction e; c itself for side = 0
__device__ __forceinline__ LCell lshift(const LCell &c, int e, int side, const int (&st)[3]) {
  LCell q = c;
  q.P += side * st[e];
  if (e == 0) q.i += side;
  else if (e == 1) q.j += side;
  else q.k += side;
  return q;
}

// parent on the next coarser level of the neighbour across a face: moving
// up from coordinate q changes the parent iff q is odd, down iff q is even
__device__ __forceinline__ int parent_shift(int q, int side, int cstep) {
  if (side > 0) return (q & 1) ? cstep : 0;
  if (side < 0) return (q & 1) ? 0 : -cstep;
  return 0;
}

// Tile order of the pre-smoothing with restriction: wavefront w of a level
// covers a tile of 16 x 2 x 2 fine cells (2D: 32 x 2), the children of 8
// (2D: 16) consecutive parents along x, and lane l holds the fine cell at
// offset (l mod 16, (l / 16) mod 2, l / 32) in the tile (2D: (l mod 32,
// l / 32)).  Each 16-lane quarter of a wavefront so reads 16 consecutive
// cells of one row, a single coalesced access; the 2^dim children of a
// parent are lanes l, l^1, l^16, l^17, l^32, ... (2D: l, l^1, l^32, l^33),
// so the restriction is a lane-shuffle sum.  Cells outside the level (an
// odd dimension, the padding of a row's last tile) are invalid and
// contribute zero.
struct Kid {
  int P, i, j, k, parent;
  bool valid, lead;
};

__host__ __device__ inline unsigned kid_px(int dim) { return dim == 3 ? 8u : 16u; }   // parents per tile along x

// number of thread indices (a multiple of 64) covering a level whose
// parents have dims (cnx, cny, cnz)
__host__ __device__ inline unsigned kid_total(int dim, int cnx, int cny, int cnz) {
  const unsigned px = kid_px(dim);
  return ((unsigned)cnx + px - 1u) / px * (unsigned)cny * (unsigned)cnz * 64u;
}

__device__ __forceinline__ Kid kid_at(unsigned tau, int dim, int nx, int ny, int nz, int cnx, int cny) {
  Kid q;
  const unsigned l = tau & 63u, w = tau >> 6;
  const unsigned px = kid_px(dim);
  const unsigned nbx = ((unsigned)cnx + px - 1u) / px;
  const unsigned row = w / nbx, bx = w - row * nbx;
  const unsigned ck = dim == 3 ? row / (unsigned)cny : 0u, cj = row - ck * (unsigned)cny;
  const unsigned xr = dim == 3 ? (l & 15u) : (l & 31u);
  const unsigned jy = dim == 3 ? ((l >> 4) & 1u) : (l >> 5);
  const unsigned kz = dim == 3 ? (l >> 5) : 0u;
  const int ci = (int)(bx * px + (xr >> 1));
  const bool pin = ci < cnx;
  q.i = (int)(2u * bx * px + xr);
  q.j = 2 * (int)cj + (int)jy;
  q.k = 2 * (int)ck + (int)kz;
  q.valid = pin && q.i < nx && q.j < ny && q.k < nz;
  q.P = q.i + nx * (q.j + ny * q.k);
  q.parent = ci + cnx * ((int)cj + cny * (int)ck);
  q.lead = pin && (xr & 1u) == 0u && jy == 0u && kz == 0u;
  return q;
}

// kid_at on a tail level (DNB: the divisor ceil(cnx / kid_px), DCY: cny)
__device__ __forceinline__ Kid kid_at_tail(unsigned tau, int dim, int nx, int ny, int nz, int cnx, int cny,
                                           const Div24 &DNB, const Div24 &DCY) {
  Kid q;
  const unsigned l = tau & 63u, w = tau >> 6;
  const unsigned px = kid_px(dim);
  const unsigned row = quot24(w, DNB), bx = w - __umul24(row, DNB.d);
  const unsigned ck = dim == 3 ? quot24(row, DCY) : 0u, cj = row - __umul24(ck, DCY.d);
  const unsigned xr = dim == 3 ? (l & 15u) : (l & 31u);
  const unsigned jy = dim == 3 ? ((l >> 4) & 1u) : (l >> 5);
  const unsigned kz = dim == 3 ? (l >> 5) : 0u;
  const int ci = (int)(__umul24(bx, px) + (xr >> 1));
  const bool pin = ci < cnx;
  q.i = (int)(2u * __umul24(bx, px) + xr);
  q.j = 2 * (int)cj + (int)jy;
  q.k = 2 * (int)ck + (int)kz;
  q.valid = pin && q.i < nx && q.j < ny && q.k < nz;
  q.P = q.i + (int)__umul24((unsigned)nx, (unsigned)(q.j + (int)__umul24((unsigned)ny, (unsigned)q.k)));
  q.parent = ci + (int)__umul24((unsigned)cnx, cj + __umul24((unsigned)cny, ck));
  q.lead = pin && (xr & 1u) == 0u && jy == 0u && kz == 0u;
  return q;
}

// sum over the 2^dim lanes of one parent: pairs along x, then y, then z;
// every lane of the wavefront must call it
template <typename T>
__device__ __forceinline__ T kid_sum(T v, int dim) {
  v = v + lane_move(v, lane_x1);
  if (dim == 3) {
    v = v + lane_move(v, lane_x16);
    v = v + lane_move(v, lane_x32);
  } else {
    v = v + lane_move(v, lane_x32);
  }
  return v;
}

// ---------------------------------------------------------------------------
// setup: coefficients of level l from level l-1 (l = 1 from rAU and flags)
// ---------------------------------------------------------------------------

template <typename T, typename R>
__device__ void setup_cell(const Slot &s, int l, int g) {
  const MGLevel &C = s.mg.lv[l];
  const LCell c = lcell(C, g);
  const int dim = s.dim;
  int nf[3], f0[3], f1[3];
  if (l == 1) { nf[0] = s.nx; nf[1] = s.ny; nf[2] = s.nz; }
  else { nf[0] = s.mg.lv[l - 1].nx; nf[1] = s.mg.lv[l - 1].ny; nf[2] = s.mg.lv[l - 1].nz; }
  const int cc[3] = {c.i, c.j, c.k};
  for (int e = 0; e < 3; ++e) {
    f0[e] = e < dim ? 2 * cc[e] : 0;
    f1[e] = e < dim ? (2 * cc[e] + 1 < nf[e] ? 2 * cc[e] + 1 : 2 * cc[e]) : 0;
  }
  const int fnx = nf[0], fnxy = nf[0] * nf[1];
  const R *rAU = (const R *)s.rAU;
  // fine low-face coefficient of fine cell F in direction e
  auto fine_low = [&](int F, int e) -> T {
    if (l == 1) {
      uint8_t fl = s.flags[F];
      if (!(fl & (1u << (2 * e)))) return (T)0;
      int st = e == 0 ? 1 : (e == 1 ? s.nx : s.nxy);
      return ((T)0.5 * ((T)rAU[F] + (T)rAU[F - st])) * (T)s.Sh;
    }
    return ((const T *)s.mg.lv[l - 1].cf[e])[F];
  };
  auto fine_out = [&](int F, int fi, int fj, int fk) -> T {
    if (l == 1) {
      uint8_t fl = s.flags[F];
      if (fl & 0x40) return (T)0;
      T acc = (T)0;
      const int q[3] = {fi, fj, fk}, n[3] = {s.nx, s.ny, s.nz};
      for (int f = 0; f < 2 * dim; ++f) {
        int e = f >> 1;
        bool edge = (f & 1) ? q[e] == n[e] - 1 : q[e] == 0;
        if (edge && s.bcf[f] == F_OUTLET) acc = acc + (T)rAU[F] * (T)s.S2h;
      }
      return acc;
    }
    return ((const T *)s.mg.lv[l - 1].cout)[F];
  };
  T low[3] = {(T)0, (T)0, (T)0}, high[3] = {(T)0, (T)0, (T)0}, out = (T)0;
  for (int fk = f0[2]; fk <= f1[2]; ++fk)
    for (int fj = f0[1]; fj <= f1[1]; ++fj)
      for (int fi = f0[0]; fi <= f1[0]; ++fi) {
        const int F = fi + fnx * fj + fnxy * fk;
        const int q[3] = {fi, fj, fk};
        out = out + fine_out(F, fi, fj, fk);
        for (int e = 0; e < dim; ++e) {
          const int st = e == 0 ? 1 : (e == 1 ? fnx : fnxy);
          // lowest child layer: its low face is the coarse low face (inside the box)
          if (q[e] == f0[e] && cc[e] > 0) low[e] = low[e] + fine_low(F, e);
          // highest child layer (a second layer exists): its high face
          if (q[e] == 2 * cc[e] + 1 && q[e] + 1 < nf[e]) high[e] = high[e] + fine_low(F + st, e);
        }
      }
  const T sc = (T)(l == 1 ? (s.dim == 3 ? MG_SCALE1_3D : MG_SCALE1_2D) : MG_SCALE);
  T diag = (T)0;
  for (int e = 0; e < 3; ++e) {
    if (e < dim) ((T *)C.cf[e])[g] = sc * low[e];
    diag = diag + sc * low[e] + sc * high[e];
  }
  ((T *)C.cout)[g] = sc * out;
  diag = diag + sc * out;
  ((T *)C.invD)[g] = diag > (T)0 ? (T)1 / diag : (T)0;
}

// workgroups of a launch over n items of one slot (at most 1024, grid-stride beyond)
__host__ __device__ inline int lvl_blocks(int n) {
  const int b = (n + BLOCK - 1) / BLOCK;
  return b < 1 ? 1 : (b > 1024 ? 1024 : b);
}

// Batched launches over a device list `act` of multigrid slots use a
// slot-major grid of maxb workgroups per slot; workgroup q of a slot works
// only if q is below the slot's own count for the launch (and the slot has
// the level).
__device__ __forceinline__ const Slot &batch_slot(const Slot *slots, const int *act, int maxb, int &q) {
  q = (int)blockIdx.x % maxb;
  return slots[act[(int)blockIdx.x / maxb]];
}

template <typename T, typename R>
__device__ __forceinline__ void mg_setup_body(const Slot &s, int l, int q, int nb) {
  const int nc = s.mg.lv[l].nc;
  for (int g = q * BLOCK + (int)threadIdx.x; g < nc; g += nb * BLOCK) setup_cell<T, R>(s, l, g);
}

template <typename T, typename R>
__global__ void __launch_bounds__(BLOCK) k_mg_setup(const Slot S, int l) {
  mg_setup_body<T, R>(S, l, (int)blockIdx.x, (int)gridDim.x);
}

template <typename T, typename R>
__global__ void __launch_bounds__(BLOCK) k_mg_setup_b(const Slot *slots, const int *act, int maxb, int l) {
  int q;
  const Slot &s = batch_slot(slots, act, maxb, q);
  if (l > s.mg.L) return;
  const int nb = lvl_blocks(s.mg.lv[l].nc);
  if (q < nb) mg_setup_body<T, R>(s, l, q, nb);
}

// Dense inverse of the coarsest operator (n <= MG_DENSE_MAX cells) by
// Gauss-Jordan elimination in LDS without pivoting (the operator is
// symmetric positive definite on its cells with fluid); a cell without fluid
// has an empty row and column and gets a zero row and column in the inverse.
template <typename T>
__device__ __forceinline__ void mg_coarse_inv_body(const Slot &s, T *A) {
  const MGLevel &C = s.mg.lv[s.mg.L];
  const int n = C.nc, dim = s.dim;
  if (n > MG_DENSE_MAX) return;   // excluded by the host's hierarchy check
  const int nn = n * n;
  for (int x = threadIdx.x; x < nn; x += MG_INV_THREADS) A[x] = (T)0;
  __syncthreads();
  if ((int)threadIdx.x < n) {
    const int g = threadIdx.x;
    const LCell c = lcell(C.nx, C.ny, g);
    const int st[3] = {1, C.nx, C.nxy}, q[3] = {c.i, c.j, c.k}, nd[3] = {C.nx, C.ny, C.nz};
    T diag = ((const T *)C.cout)[g];
    for (int e = 0; e < dim; ++e) {
      const T *cf = (const T *)C.cf[e];
      const T cl = cf[g];
      const T ch = q[e] < nd[e] - 1 ? cf[g + st[e]] : (T)0;
      diag = diag + cl + ch;
      if (q[e] > 0) A[g * n + g - st[e]] = -cl;
      if (q[e] < nd[e] - 1) A[g * n + g + st[e]] = -ch;
    }
    A[g * n + g] = diag;
  }
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    const T akk = A[k * n + k];
    T nv[(MG_DENSE_MAX * MG_DENSE_MAX + MG_INV_THREADS - 1) / MG_INV_THREADS];
    int m = 0;
    for (int x = threadIdx.x; x < nn; x += MG_INV_THREADS, ++m) {
      const int i = x / n, j = x - i * n;
      const T aij = A[x], aik = A[i * n + k], akj = A[k * n + j];
      if (akk == (T)0) nv[m] = aij;   // empty row and column: nothing to eliminate
      else if (i == k && j == k) nv[m] = (T)1 / akk;
      else if (i == k) nv[m] = akj / akk;
      else if (j == k) nv[m] = -(aik / akk);
      else nv[m] = aij - aik * (akj / akk);
    }
    __syncthreads();
    m = 0;
    for (int x = threadIdx.x; x < nn; x += MG_INV_THREADS, ++m) A[x] = nv[m];
    __syncthreads();
  }
  T *out = (T *)s.mg.Ainv;
  for (int x = threadIdx.x; x < nn; x += MG_INV_THREADS) out[x] = A[x];
}

template <typename T>
__global__ void __launch_bounds__(MG_INV_THREADS) k_mg_coarse_inv(const Slot S) {
  __shared__ T A[MG_DENSE_MAX * MG_DENSE_MAX];
  mg_coarse_inv_body<T>(S, A);
}

template <typename T>
__global__ void __launch_bounds__(MG_INV_THREADS) k_mg_coarse_inv_b(const Slot *slots, const int *act) {
  __shared__ T A[MG_DENSE_MAX * MG_DENSE_MAX];
  mg_coarse_inv_body<T>(slots[act[blockIdx.x]], A);
}

// ---------------------------------------------------------------------------
// cycle pieces on coarse levels (DIM = 2 or 3)
// ---------------------------------------------------------------------------

// Offsets of the radius-2 stencil (the cell, its 2 DIM neighbours, then the
// cells two faces away) and the index of an offset in that list.
constexpr int kStar[25][3] = {{0, 0, 0},   {-1, 0, 0},  {1, 0, 0},   {0, -1, 0},  {0, 1, 0},
                              {0, 0, -1},  {0, 0, 1},   {-2, 0, 0},  {2, 0, 0},   {0, -2, 0},
                              {0, 2, 0},   {-1, -1, 0}, {1, -1, 0},  {-1, 1, 0},  {1, 1, 0},
                              {0, 0, -2},  {0, 0, 2},   {-1, 0, -1}, {1, 0, -1},  {-1, 0, 1},
                              {1, 0, 1},   {0, -1, -1}, {0, 1, -1},  {0, -1, 1},  {0, 1, 1}};
template <int DIM>
constexpr int kStarN = DIM == 3 ? 25 : 13;   // 2D: the 13 entries of the first 15 with a zero z offset
template <int DIM>
constexpr int star_entry(int m) {   // m-th entry of the DIM stencil in kStar
  return DIM == 3 ? m : (m < 5 ? m : m + 2);
}
template <int DIM>
constexpr int star_find(int dx, int dy, int dz) {
  for (int m = 0; m < kStarN<DIM>; ++m) {
    const int k = star_entry<DIM>(m);
    if (kStar[k][0] == dx && kStar[k][1] == dy && kStar[k][2] == dz) return m;
  }
  return -1;
}

// every neighbour of every radius-1 entry is in the stencil
template <int DIM>
constexpr bool star_complete() {
  for (int m = 0; m < 2 * DIM + 1; ++m)
    for (int e = 0; e < DIM; ++e)
      for (int sgn = -1; sgn <= 1; sgn += 2) {
        const int *o = kStar[star_entry<DIM>(m)];
        if (star_find<DIM>(o[0] + sgn * (e == 0), o[1] + sgn * (e == 1), o[2] + sgn * (e == 2)) < 0) return false;
      }
  return true;
}
static_assert(star_complete<2>() && star_complete<3>(), "radius-2 stencil table");

// One Jacobi sweep from v0 evaluated on the cell and its neighbours, then A
// applied to the result at the cell: v1 = v0 + w D^-1 (b - A v0) on the
// radius-1 star, returns (A v1)_c and v1 at c in v1c.  v0(B, ci, cj, ck)
// gives the starting iterate at the cell of byte offset B (elements of T)
// and coordinates (ci, cj, ck).  Every operand of the radius-2 stencil is
// loaded once, unconditionally, at its cell or (outside the box) at c, by a
// 32-bit byte offset that serves every array of the level; faces across the
// box boundary then add nothing, as in lmatvec, whose terms there vanish
// exactly.  The level's arrays are in global memory.
template <int DIM, typename T, class V0>
__device__ __forceinline__ T sweep_matvec(const LV<T> &L, const LCell &c, V0 &&v0, T &v1c) {
  constexpr int N = kStarN<DIM>, M = 2 * DIM + 1;
  const T w = (T)MG_OMEGA;
  const int n[3] = {L.nx, L.ny, L.nz};
  const int q[3] = {c.i, c.j, c.k};
  unsigned B[N];
  bool in[N];
  T u0[N];
#pragma unroll
  for (int m = 0; m < N; ++m) {
    const int *o = kStar[star_entry<DIM>(m)];
    bool b = true;
#pragma unroll
    for (int e = 0; e < 3; ++e) b = b && q[e] + o[e] >= 0 && q[e] + o[e] < n[e];
    in[m] = b;
    B[m] = (unsigned)(b ? c.P + o[0] + L.nx * o[1] + L.nxy * o[2] : c.P) * (unsigned)sizeof(T);
    u0[m] = v0(B[m], b ? c.i + o[0] : c.i, b ? c.j + o[1] : c.j, b ? c.k + o[2] : c.k);
  }
  // (A u)_m for the star entry m < M from u at the entries it reaches
  auto mv = [&](int m, const T *u) -> T {
    const int *o = kStar[star_entry<DIM>(m)];
    T acc = (T)0;
#pragma unroll
    for (int e = 0; e < DIM; ++e) {
      const int ml = star_find<DIM>(o[0] - (e == 0), o[1] - (e == 1), o[2] - (e == 2));
      const int mh = star_find<DIM>(o[0] + (e == 0), o[1] + (e == 1), o[2] + (e == 2));
      const T cl = ldo(L.cf[e], B[m]), ch = ldo(L.cf[e], B[mh]);
      const T tl = acc + cl * (u[m] - u[ml]);
      acc = in[ml] ? tl : acc;
      const T th = acc + ch * (u[m] - u[mh]);
      acc = in[mh] ? th : acc;
    }
    return acc + ldo(L.cout, B[m]) * u[m];
  };
  T u1[N];
#pragma unroll
  for (int m = 0; m < N; ++m) u1[m] = u0[m];
#pragma unroll
  for (int m = 0; m < M; ++m) u1[m] = u0[m] + w * (ldo(L.invD, B[m]) * (ldo((const T *)L.b, B[m]) - mv(m, u0)));
  v1c = u1[0];
  return mv(0, u1);
}

// Pre-smoothing from zero on level L in tile order, with the restriction:
// x_1 = w D^-1 b, x_{m+1} = x_m + w D^-1 (b - A x_m) up to NU sweeps,
// t = b - A x, b_next[parent] = sum of the children's t.  (cnx, cny, cnz)
// are the dimensions of the next coarser level; bnext may point to global
// memory or to LDS.  With GATE, done (uniform): the solve had converged
// before the launch, nothing is written (tested once the first cell's loads
// are in).
template <int DIM, typename T, int NU, bool GATE = false>
__device__ __forceinline__ void smooth_restrict(const LV<T> &L, int cnx, int cny, int cnz, T *bnext, unsigned start,
                                                unsigned stride, int done = 0) {
  const T w = (T)MG_OMEGA;
  const unsigned total = kid_total(DIM, cnx, cny, cnz);
  for (unsigned tau = start; tau < total; tau += stride) {
    const Kid q = kid_at(tau, DIM, L.nx, L.ny, L.nz, cnx, cny);
    T tv = (T)0, xP = (T)0;
    if (q.valid) {
      LCell c;
      c.P = q.P;
      c.i = q.i;
      c.j = q.j;
      c.k = q.k;
      auto x1 = [&](int n, int, int) -> T { return w * (L.invD[n] * L.b[n]); };
      T Ax;
      if constexpr (NU == 1) {
        xP = x1(c.P, 0, 0);
        Ax = lmatvec<DIM, T>(L, c, x1);
      } else {
        static_assert(NU == 2, "one or two sweeps");
        auto x1o = [&](unsigned b, int, int, int) -> T { return w * (ldo(L.invD, b) * ldo((const T *)L.b, b)); };
        Ax = sweep_matvec<DIM, T>(L, c, x1o, xP);
      }
      tv = L.b[c.P] - Ax;
    }
    if constexpr (GATE) {
      keep_live(tv);
      if (read_late(done)) return;
    }
    if (q.valid) L.x[q.P] = xP;
    tv = kid_sum(tv, DIM);
    if (q.lead) bnext[q.parent] = tv;
  }
}

// prolongation and post-smoothing on level L: y = x + P xc (xc on the next
// coarser level, of dims (cnx, ., .) and plane size cnxy; global memory or
// LDS), then NU sweeps y <- y + w D^-1 (b - A y); out = y.  GATE, done: as
// in smooth_restrict.
template <int DIM, typename T, int NU, bool GATE = false>
__device__ __forceinline__ void up_range(const LV<T> &L, int cnx, int cnxy, const T *xc, T *out, int start, int stride,
                                         int done = 0) {
  const T w = (T)MG_OMEGA;
  const int st[3] = {1, L.nx, L.nxy};
  for (int g = start; g < L.nc; g += stride) {
    const LCell c = lcell(L.nx, L.ny, g);
    auto y0at = [&](const LCell &p) -> T { return L.x[p.P] + xc[(p.i >> 1) + cnx * (p.j >> 1) + cnxy * (p.k >> 1)]; };
    // one sweep evaluated at cell p from y0 at p and its neighbours
    auto y1at = [&](const LCell &p) -> T {
      auto y0 = [&](int, int e, int side) -> T { return y0at(lshift(p, e, side, st)); };
      return y0at(p) + w * (L.invD[p.P] * (L.b[p.P] - lmatvec<DIM, T>(L, p, y0)));
    };
    T res;
    if constexpr (NU == 1) {
      res = y1at(c);
    } else {
      auto y0o = [&](unsigned b, int i, int j, int k) -> T {
        return ldo((const T *)L.x, b) + ldo(xc, (unsigned)((i >> 1) + cnx * (j >> 1) + cnxy * (k >> 1)) * (unsigned)sizeof(T));
      };
      T y1P;
      const T Ay1 = sweep_matvec<DIM, T>(L, c, y0o, y1P);
      res = y1P + w * (L.invD[g] * (L.b[g] - Ay1));
    }
    if constexpr (GATE) {
      keep_live(res);
      if (read_late(done)) return;
    }
    out[g] = res;
  }
}

// Large levels (MG_SPLIT_MIN cells or more) with two sweeps per side run
// each sweep as a launch of its own.  The fused kernels above evaluate the
// first sweep again at every neighbour (a radius-2 stencil: about 100 loads
// per cell, and registers for three waves per SIMD); on a large level a
// launch costs little beside that, so the sweep is stored and the next step
// reads it on the radius-1 star.  star1, matvec_center and sweep_center
// take the operations of sweep_matvec at the star's centre in the same order,
// so every stored value is bitwise the one the fused kernels recompute, and
// the results are those of the fused kernels.

// byte offsets of the radius-1 star of cell c (m = 0 the cell, 1 + 2e and
// 2 + 2e its low and high neighbour in direction e; the cell itself outside
// the box) and whether each neighbour exists
template <int DIM, typename T>
__device__ __forceinline__ void star1(const LV<T> &L, const LCell &c, unsigned (&B)[7], bool (&in)[7]) {
  const int n[3] = {L.nx, L.ny, L.nz};
  const int q[3] = {c.i, c.j, c.k};
  const int st[3] = {1, L.nx, L.nxy};
  B[0] = (unsigned)c.P * (unsigned)sizeof(T);
  in[0] = true;
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    const bool lo = e < DIM && q[e] > 0, hi = e < DIM && q[e] < n[e] - 1;
    in[1 + 2 * e] = lo;
    in[2 + 2 * e] = hi;
    B[1 + 2 * e] = lo ? (unsigned)(c.P - st[e]) * (unsigned)sizeof(T) : B[0];
    B[2 + 2 * e] = hi ? (unsigned)(c.P + st[e]) * (unsigned)sizeof(T) : B[0];
  }
}

// (A u) at the star's centre from u(m) on the star (sweep_matvec's mv at m = 0)
template <int DIM, typename T, class U>
__device__ __forceinline__ T matvec_center(const LV<T> &L, const unsigned (&B)[7], const bool (&in)[7], U &&u) {
  T acc = (T)0;
#pragma unroll
  for (int e = 0; e < DIM; ++e) {
    const int ml = 1 + 2 * e, mh = 2 + 2 * e;
    const T cl = ldo(L.cf[e], B[0]), ch = ldo(L.cf[e], B[mh]);
    const T tl = acc + cl * (u(0) - u(ml));
    acc = in[ml] ? tl : acc;
    const T th = acc + ch * (u(0) - u(mh));
    acc = in[mh] ? th : acc;
  }
  return acc + ldo(L.cout, B[0]) * u(0);
}

// one Jacobi sweep from u0 at the star's centre: u0 + w D^-1 (b - A u0)
template <int DIM, typename T, class U>
__device__ __forceinline__ T sweep_center(const LV<T> &L, const unsigned (&B)[7], const bool (&in)[7], U &&u0) {
  const T w = (T)MG_OMEGA;
  return u0(0) + w * (ldo(L.invD, B[0]) * (ldo((const T *)L.b, B[0]) - matvec_center<DIM, T>(L, B, in, u0)));
}

// pre-smoothing, first launch: x = both sweeps from zero at every cell
template <int DIM, typename T>
__device__ __forceinline__ void split_smooth(const LV<T> &L, int start, int stride, int done) {
  const T w = (T)MG_OMEGA;
  for (int g = start; g < L.nc; g += stride) {
    const LCell c = lcell(L.nx, L.ny, g);
    unsigned B[7];
    bool in[7];
    star1<DIM, T>(L, c, B, in);
    auto x1 = [&](int m) -> T { return w * (ldo(L.invD, B[m]) * ldo((const T *)L.b, B[m])); };
    const T x2 = sweep_center<DIM, T>(L, B, in, x1);
    keep_live(x2);
    if (read_late(done)) return;
    L.x[g] = x2;
  }
}

// pre-smoothing, second launch: the residual b - A x restricted in tile order
template <int DIM, typename T>
__device__ __forceinline__ void split_restrict(const LV<T> &L, int cnx, int cny, int cnz, T *bnext, unsigned start,
                                               unsigned stride, int done) {
  const unsigned total = kid_total(DIM, cnx, cny, cnz);
  for (unsigned tau = start; tau < total; tau += stride) {
    const Kid q = kid_at(tau, DIM, L.nx, L.ny, L.nz, cnx, cny);
    T tv = (T)0;
    if (q.valid) {
      LCell c;
      c.P = q.P;
      c.i = q.i;
      c.j = q.j;
      c.k = q.k;
      unsigned B[7];
      bool in[7];
      star1<DIM, T>(L, c, B, in);
      auto x2 = [&](int m) -> T { return ldo((const T *)L.x, B[m]); };
      tv = L.b[c.P] - matvec_center<DIM, T>(L, B, in, x2);
    }
    keep_live(tv);
    if (read_late(done)) return;
    tv = kid_sum(tv, DIM);
    if (q.lead) bnext[q.parent] = tv;
  }
}

// prolongation and first post-sweep: y1 = y0 + w D^-1 (b - A y0), y0 = x + P xc
template <int DIM, typename T>
__device__ __forceinline__ void split_up_first(const LV<T> &L, int cnx, int cnxy, const T *xc, T *y1out, int start,
                                               int stride, int done) {
  const int st[3] = {1, L.nx, L.nxy};
  for (int g = start; g < L.nc; g += stride) {
    const LCell c = lcell(L.nx, L.ny, g);
    unsigned B[7];
    bool in[7];
    star1<DIM, T>(L, c, B, in);
    auto y0 = [&](int m) -> T {
      const LCell p = m == 0 || !in[m] ? c : lshift(c, (m - 1) >> 1, (m & 1) ? -1 : 1, st);
      return ldo((const T *)L.x, B[m]) +
             ldo(xc, (unsigned)((p.i >> 1) + cnx * (p.j >> 1) + cnxy * (p.k >> 1)) * (unsigned)sizeof(T));
    };
    const T y1 = sweep_center<DIM, T>(L, B, in, y0);
    keep_live(y1);
    if (read_late(done)) return;
    y1out[g] = y1;
  }
}

// second post-sweep: out = y1 + w D^-1 (b - A y1)
template <int DIM, typename T>
__device__ __forceinline__ void split_up_second(const LV<T> &L, const T *y1in, T *out, int start, int stride,
                                                int done) {
  const T w = (T)MG_OMEGA;
  for (int g = start; g < L.nc; g += stride) {
    const LCell c = lcell(L.nx, L.ny, g);
    unsigned B[7];
    bool in[7];
    star1<DIM, T>(L, c, B, in);
    auto y1 = [&](int m) -> T { return ldo(y1in, B[m]); };
    const T res = y1(0) + w * (L.invD[g] * (L.b[g] - matvec_center<DIM, T>(L, B, in, y1)));
    keep_live(res);
    if (read_late(done)) return;
    out[g] = res;
  }
}

// The levels of the single-workgroup tail live in LDS, where a barrier is
// cheap: their sweeps run one after the other over the whole level with a
// barrier between them (rather than re-evaluating earlier sweeps at the
// neighbours, as the grid-wide kernels must).
//
// Pre-smoothing of an LDS level: nu Jacobi sweeps from zero into x (t as
// scratch), then the residual b - A x restricted into bnext in tile order.
// The first sweep from zero, w D^-1 b, is evaluated where the second one
// reads it (its value at the cell and the neighbours, as the grid-wide
// kernels do), so the two take one pass and one barrier.
template <int DIM, typename T>
__device__ __forceinline__ void tail_down(const LV<T> &L, int cnx, int cny, int cnz, T *bnext, int t0, int ns,
                                          int nu) {
  const T w = (T)MG_OMEGA;
  const Div24 DX = div24(L.nx), DY = div24(L.ny);
  auto x1 = [&](int n, int, int) -> T { return w * (L.invD[n] * L.b[n]); };
  if (nu >= 2) {
    for (int g = t0; g < L.nc; g += ns) {
      const LCell c = lcell24(DX, DY, g);
      L.x[g] = x1(g, 0, 0) + w * (L.invD[g] * (L.b[g] - lmatvec<DIM, T>(L, c, x1)));
    }
  } else {
    for (int g = t0; g < L.nc; g += ns) L.x[g] = x1(g, 0, 0);
  }
  __syncthreads();
  T *src = L.x, *dst = L.t;
  for (int m = 2; m < nu; ++m) {
    for (int g = t0; g < L.nc; g += ns) {
      const LCell c = lcell24(DX, DY, g);
      auto xs = [&](int n, int, int) -> T { return src[n]; };
      dst[g] = src[g] + w * (L.invD[g] * (L.b[g] - lmatvec<DIM, T>(L, c, xs)));
    }
    __syncthreads();
    T *tmp = src;
    src = dst;
    dst = tmp;
  }
  const unsigned total = kid_total(DIM, cnx, cny, cnz);
  const Div24 DNB = div24((int)(((unsigned)cnx + kid_px(DIM) - 1u) / kid_px(DIM))), DCY = div24(cny);
  for (unsigned tau = (unsigned)t0; tau < total; tau += (unsigned)ns) {
    const Kid q = kid_at_tail(tau, DIM, L.nx, L.ny, L.nz, cnx, cny, DNB, DCY);
    T tv = (T)0;
    if (q.valid) {
      LCell c;
      c.P = q.P;
      c.i = q.i;
      c.j = q.j;
      c.k = q.k;
      auto xs = [&](int n, int, int) -> T { return src[n]; };
      tv = L.b[c.P] - lmatvec<DIM, T>(L, c, xs);
      if (src != L.x) L.x[c.P] = src[c.P];
    }
    tv = kid_sum(tv, DIM);
    if (q.lead) bnext[q.parent] = tv;
  }
}

// Prolongation and post-smoothing of an LDS level: y = x + P xc, then nu
// Jacobi sweeps alternating between t and x (x is free once the first sweep
// has read it); returns the array holding the result.  With out (an array
// that none of the level's arrays aliases), the last sweep writes there
// instead, and no barrier follows it (out is returned).
template <int DIM, typename T>
__device__ __forceinline__ const T *tail_up(const LV<T> &L, int cnx, int cnxy, const T *xc, int t0, int ns, int nu,
                                            T *out = nullptr) {
  const T w = (T)MG_OMEGA;
  const int st[3] = {1, L.nx, L.nxy};
  const Div24 DX = div24(L.nx), DY = div24(L.ny);
  T *first = nu == 1 && out ? out : L.t;
  for (int g = t0; g < L.nc; g += ns) {
    const LCell c = lcell24(DX, DY, g);
    auto y0at = [&](const LCell &p) -> T {
      return L.x[p.P] + xc[(p.i >> 1) + (int)__umul24((unsigned)cnx, (unsigned)(p.j >> 1)) +
                           (int)__umul24((unsigned)cnxy, (unsigned)(p.k >> 1))];
    };
    auto y0 = [&](int, int e, int side) -> T { return y0at(lshift(c, e, side, st)); };
    first[g] = y0at(c) + w * (L.invD[g] * (L.b[g] - lmatvec<DIM, T>(L, c, y0)));
  }
  if (first == out) return out;
  __syncthreads();
  T *src = L.t, *dst = L.x;
  for (int m = 1; m < nu; ++m) {
    const bool last = m == nu - 1 && out;
    T *to = last ? out : dst;
    for (int g = t0; g < L.nc; g += ns) {
      const LCell c = lcell24(DX, DY, g);
      auto ys = [&](int n, int, int) -> T { return src[n]; };
      to[g] = src[g] + w * (L.invD[g] * (L.b[g] - lmatvec<DIM, T>(L, c, ys)));
    }
    if (last) return out;
    __syncthreads();
    T *tmp = src;
    src = dst;
    dst = tmp;
  }
  return src;
}

// Each multigrid kernel comes in two forms over one body: for one context
// (its record passed by value: the fields are read from the constant
// argument segment) and batched over the serving engine's slot table.
// Either returns at once for a slot whose solve has converged.
__device__ __forceinline__ bool mg_idle(const Slot &s) { return s.st->done != 0; }

// workgroups of the pre-smoothing launch of level l (tile order over the
// next coarser level) and of its prolongation launch
__host__ __device__ inline int smooth_blocks(const MGInfo &mg, int l, int dim) {
  const MGLevel &C = mg.lv[l + 1];
  return lvl_blocks((int)kid_total(dim, C.nx, C.ny, C.nz));
}
__host__ __device__ inline int up_blocks(const MGInfo &mg, int l) { return lvl_blocks(mg.lv[l].nc); }

template <int DIM, typename T, int NU>
__device__ __forceinline__ void mg_smooth_body(const Slot &s, int l, unsigned start, unsigned stride) {
  const LV<T> L = lview<T>(s.mg.lv[l]);
  const MGLevel &C = s.mg.lv[l + 1];
  smooth_restrict<DIM, T, NU>(L, C.nx, C.ny, C.nz, (T *)C.b, start, stride);
}

// final correction of level l goes to t_l (x_l keeps the pre-smoothed one)
template <int DIM, typename T, int NU>
__device__ __forceinline__ void mg_up_body(const Slot &s, int l, int start, int stride) {
  const LV<T> L = lview<T>(s.mg.lv[l]);
  const MGLevel &C = s.mg.lv[l + 1];
  up_range<DIM, T, NU>(L, C.nx, C.nxy, (const T *)C.t, L.t, start, stride);
}

// One context: the slot's state and the levels F = l and C = l + 1 by value
// (their fields at fixed offsets of the argument segment, requested at
// entry).  NU: the sweeps of level l, (mg.nu2 >> l & 1) + 1, chosen by the
// host.
#define OSCAR_PRIME_LEVELS(F, C)                                                                                      \
  OSCAR_PRIME("s"(F.nx), "s"(F.ny), "s"(F.nz), "s"(F.nxy), "s"(F.nc), "s"(F.cf[0]), "s"(F.cf[1]), "s"(F.cf[2]),       \
              "s"(F.cout), "s"(F.invD), "s"(F.b), "s"(F.x), "s"(F.t), "s"(C.nx), "s"(C.ny), "s"(C.nz));               \
  OSCAR_PRIME("s"(C.nxy), "s"(C.b), "s"(C.t))

template <int DIM, typename T, int NU>
__global__ void __launch_bounds__(BLOCK) k_mg_smooth(SlotState *st, const MGLevel F, const MGLevel C,
                                                     unsigned long long *ts) {
  OSCAR_PRIME("s"(ts), "s"(st), "s"(gridDim.x));
  OSCAR_PRIME_LEVELS(F, C);
  Stamp stamp(ts);
  const int done = st->done;
  smooth_restrict<DIM, T, NU, true>(lview<T>(F), C.nx, C.ny, C.nz, (T *)C.b, blockIdx.x * BLOCK + threadIdx.x,
                                    gridDim.x * BLOCK, done);
  if (!done) stamp.done();
}

template <int DIM, typename T, int NU>
__global__ void __launch_bounds__(BLOCK) k_mg_up(SlotState *st, const MGLevel F, const MGLevel C,
                                                 unsigned long long *ts) {
  OSCAR_PRIME("s"(ts), "s"(st), "s"(gridDim.x));
  OSCAR_PRIME_LEVELS(F, C);
  Stamp stamp(ts);
  const int done = st->done;
  const LV<T> L = lview<T>(F);
  up_range<DIM, T, NU, true>(L, C.nx, C.nxy, (const T *)C.t, L.t, (int)(blockIdx.x * BLOCK + threadIdx.x),
                       (int)(gridDim.x * BLOCK), done);
  if (!done) stamp.done();
}

// the two launches of each side of a split level (one context)
template <int DIM, typename T>
__global__ void __launch_bounds__(BLOCK) k_mg_split_smooth(SlotState *st, const MGLevel F, const MGLevel C,
                                                           unsigned long long *ts) {
  OSCAR_PRIME("s"(ts), "s"(st), "s"(gridDim.x));
  OSCAR_PRIME_LEVELS(F, C);
  Stamp stamp(ts);
  const int done = st->done;
  split_smooth<DIM, T>(lview<T>(F), (int)(blockIdx.x * BLOCK + threadIdx.x), (int)(gridDim.x * BLOCK), done);
  if (!done) stamp.done();
}

template <int DIM, typename T>
__global__ void __launch_bounds__(BLOCK) k_mg_split_restrict(SlotState *st, const MGLevel F, const MGLevel C,
                                                             unsigned long long *ts) {
  OSCAR_PRIME("s"(ts), "s"(st), "s"(gridDim.x));
  OSCAR_PRIME_LEVELS(F, C);
  Stamp stamp(ts);
  const int done = st->done;
  split_restrict<DIM, T>(lview<T>(F), C.nx, C.ny, C.nz, (T *)C.b, blockIdx.x * BLOCK + threadIdx.x,
                         gridDim.x * BLOCK, done);
  if (!done) stamp.done();
}

// tmp: the first post-sweep (a free array of at least F.nc elements)
template <int DIM, typename T>
__global__ void __launch_bounds__(BLOCK) k_mg_split_up1(SlotState *st, const MGLevel F, const MGLevel C, T *tmp,
                                                        unsigned long long *ts) {
  OSCAR_PRIME("s"(ts), "s"(st), "s"(gridDim.x), "s"(tmp));
  OSCAR_PRIME_LEVELS(F, C);
  Stamp stamp(ts);
  const int done = st->done;
  split_up_first<DIM, T>(lview<T>(F), C.nx, C.nxy, (const T *)C.t, tmp, (int)(blockIdx.x * BLOCK + threadIdx.x),
                         (int)(gridDim.x * BLOCK), done);
  if (!done) stamp.done();
}

template <int DIM, typename T>
__global__ void __launch_bounds__(BLOCK) k_mg_split_up2(SlotState *st, const MGLevel F, const MGLevel C, const T *tmp,
                                                        unsigned long long *ts) {
  OSCAR_PRIME("s"(ts), "s"(st), "s"(gridDim.x), "s"(tmp));
  OSCAR_PRIME_LEVELS(F, C);
  Stamp stamp(ts);
  const int done = st->done;
  const LV<T> L = lview<T>(F);
  split_up_second<DIM, T>(L, tmp, L.t, (int)(blockIdx.x * BLOCK + threadIdx.x), (int)(gridDim.x * BLOCK), done);
  if (!done) stamp.done();
}

// batched: level l of the slots whose tail starts below it
template <int DIM, typename T>
__global__ void __launch_bounds__(BLOCK) k_mg_smooth_b(const Slot *slots, const int *act, int maxb, int l) {
  int q;
  const Slot &s = batch_slot(slots, act, maxb, q);
  if (l >= s.mg.tail || mg_idle(s)) return;
  const int nb = smooth_blocks(s.mg, l, DIM);
  if (q >= nb) return;
  if ((s.mg.nu2 >> l) & 1) mg_smooth_body<DIM, T, 2>(s, l, (unsigned)(q * BLOCK) + threadIdx.x, (unsigned)(nb * BLOCK));
  else mg_smooth_body<DIM, T, 1>(s, l, (unsigned)(q * BLOCK) + threadIdx.x, (unsigned)(nb * BLOCK));
}

template <int DIM, typename T>
__global__ void __launch_bounds__(BLOCK) k_mg_up_b(const Slot *slots, const int *act, int maxb, int l) {
  int q;
  const Slot &s = batch_slot(slots, act, maxb, q);
  if (l >= s.mg.tail || mg_idle(s)) return;
  const int nb = up_blocks(s.mg, l);
  if (q >= nb) return;
  if ((s.mg.nu2 >> l) & 1) mg_up_body<DIM, T, 2>(s, l, q * BLOCK + (int)threadIdx.x, nb * BLOCK);
  else mg_up_body<DIM, T, 1>(s, l, q * BLOCK + (int)threadIdx.x, nb * BLOCK);
}

// Levels tail..L in one workgroup of ns threads, out of LDS.  The tail block
// is laid out in LDS as in global memory; its first part (the dense inverse
// of the coarsest operator, per level the face and outlet coefficients and
// inverse diagonal, and the tail level's right-hand side) is copied into LDS
// with one round of 16-byte loads, the rest (the arrays the tail writes
// before it reads them) is not.  The down-sweep to the coarsest level, its
// solve with the dense inverse and the up-sweep then touch LDS only, and the
// tail level's last sweep writes its correction to global memory for the
// next finer level's prolongation.  Without IN_LDS the same steps run on
// the block in global memory (the persistent solve, when the block exceeds
// its LDS).
// (done: the solve had converged before the launch; nothing is written to
// global memory, tested once the block's loads are in; returns !done)
template <int DIM, typename T, bool IN_LDS>
__device__ __forceinline__ bool mg_tail_body(const Slot &s, uint4 *mg_lds, int t0, int ns, int done = 0) {
  const int tl = s.mg.tail, L = s.mg.L;
  const char *gbase = (const char *)s.mg.tail_base;
  if constexpr (IN_LDS) {
    constexpr int U = 8;   // 16-byte loads in flight per thread
    typedef unsigned v4u __attribute__((ext_vector_type(4)));
    const OSCAR_GLOBAL v4u *src = (const OSCAR_GLOBAL v4u *)gbase;
    v4u *dst = (v4u *)mg_lds;
    const int n16 = s.mg.tail_load >> 4;   // the arrays read before they are written
    for (int x0 = t0; x0 < n16; x0 += U * ns) {
      v4u v[U];
#pragma unroll
      for (int u = 0; u < U; ++u)   // lanes past the end load nothing (a wavefront past it skips the load)
        if (x0 + u * ns < n16) v[u] = src[x0 + u * ns];
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (x0 + u * ns < n16) dst[x0 + u * ns] = v[u];
    }
  }
  if (done) return false;   // uniform
  __syncthreads();
  // an array of the block at its LDS position (itself without LDS; the
  // choice is made at compile time so that LDS accesses stay LDS
  // instructions rather than generic ones)
  auto in_lds = [&](const void *g) -> T * {
    if constexpr (IN_LDS) return (T *)((char *)mg_lds + ((const char *)g - gbase));
    else return (T *)g;
  };
  auto lds_view = [&](int l) -> LV<T> {
    const MGLevel &M = s.mg.lv[l];
    LV<T> v;
    v.nx = M.nx;
    v.ny = M.ny;
    v.nz = M.nz;
    v.nxy = M.nxy;
    v.nc = M.nc;
#pragma unroll
    for (int e = 0; e < 3; ++e) v.cf[e] = in_lds(M.cf[e < DIM ? e : 0]);
    v.cout = in_lds(M.cout);
    v.invD = in_lds(M.invD);
    v.b = in_lds(M.b);
    v.x = in_lds(M.x);
    v.t = in_lds(M.t);
    return v;
  };
  for (int l = tl; l < L; ++l) {
    const MGLevel &N = s.mg.lv[l + 1];
    tail_down<DIM, T>(lds_view(l), N.nx, N.ny, N.nz, in_lds(N.b), t0, ns, MG_TAIL_NU);
    __syncthreads();
  }
  // coarsest level: t = A^-1 b with the dense inverse (row t0, fixed order)
  {
    const LV<T> C = lds_view(L);
    const int n = C.nc;
    for (int row = t0; row < n; row += ns) {
      const T *Ai = in_lds(s.mg.Ainv) + row * n;
      T acc = (T)0;
      for (int m = 0; m < n; ++m) acc = acc + Ai[m] * C.b[m];
      C.t[row] = acc;
    }
  }
  __syncthreads();
  const T *tc = in_lds(s.mg.lv[L].t);   // correction of the level below, wherever its sweeps left it
  // the tail level's last sweep goes straight to its array in global memory
  // (out of LDS; in global memory that array is one the sweeps alternate on)
  T *const tout = (T *)s.mg.lv[tl].t;
  for (int l = L - 1; l >= tl; --l) {
    const LV<T> Lv = lds_view(l);
    const MGLevel &N = s.mg.lv[l + 1];
    tc = tail_up<DIM, T>(Lv, N.nx, N.nxy, tc, t0, ns, MG_TAIL_NU, IN_LDS && l == tl ? tout : nullptr);
    if (IN_LDS && l == tl) break;
    __syncthreads();
  }
  if constexpr (!IN_LDS) {
    const MGLevel &M = s.mg.lv[tl];
    const T *tsrc = tc;
    T *tdst = (T *)M.t;
    if (tsrc != tdst)
      for (int g = t0; g < M.nc; g += ns) tdst[g] = tsrc[g];
  }
  return true;
}

template <int DIM, typename T>
__global__ void __launch_bounds__(MG_TAIL_THREADS) k_mg_tail(const Slot S, unsigned long long *ts) {
  OSCAR_PRIME("s"(ts), "s"(S.st), "s"(S.mg.tail_base), "s"(S.mg.tail_load), "s"(S.mg.tail), "s"(S.mg.L),
              "s"(S.mg.Ainv));
  Stamp stamp(ts);
  const int done = S.st->done;
  extern __shared__ uint4 mg_lds[];
  if (mg_tail_body<DIM, T, true>(S, mg_lds, threadIdx.x, MG_TAIL_THREADS, done)) stamp.done();
}

// batched: one workgroup per slot
template <int DIM, typename T>
__global__ void __launch_bounds__(MG_TAIL_THREADS) k_mg_tail_b(const Slot *slots, const int *act) {
  const Slot &s = slots[act[blockIdx.x]];
  if (mg_idle(s)) return;
  extern __shared__ uint4 mg_lds[];
  mg_tail_body<DIM, T, true>(s, mg_lds, threadIdx.x, MG_TAIL_THREADS);
}

// ---------------------------------------------------------------------------
// fine level: conjugate-gradient pieces fused with the cycle's fine steps
// (block-table launches like the other fine-grid kernels)
// ---------------------------------------------------------------------------

// This workgroup's block within the slot, or -1 for padding: the launch
// deals its workgroups round-robin to the 8 XCDs and each XCD runs a
// contiguous run of the slot's blocks (the host's block table for one slot,
// computed here rather than loaded).
__device__ __forceinline__ int xcd_block(int p, int nb) {
  const int X = 8, q = nb / X, rem = nb % X;
  const int x = p % X, i = p / X;
  const int cnt = q + (x < rem ? 1 : 0);
  const int start = x * q + (x < rem ? x : rem);
  return i < cnt ? start + i : -1;
}

// cells per thread and batch in the fine-grid kernels: two in FP32; one in
// FP64, whose operands of two cells would exceed the 128 registers that
// keep four waves per SIMD resident
template <typename R>
constexpr int FINE_NB = sizeof(R) == 4 ? 2 : 1;
// The search direction holds fewer operands per cell: a context's launch of
// it takes four cells per batch in FP32 (125 registers) and two in FP64
// (108).  A thread uses its cells in index order whatever the batch, so the
// results are those of FINE_NB.
template <typename R>
constexpr int DIR_NB = sizeof(R) == 4 ? 4 : 2;

// The three fine-grid kernels below take each thread's cells NB at a time:
// the flags of the batch, then all stencil operands of its fluid cells, are
// loaded before the reduction of the previous launch's partials is read, so
// a wave waits for about two memory round trips rather than one per cell
// plus one for the partials.

// Search direction of iteration it: gamma_it = <r,z> and |r|^2 from the
// previous cycle's reduction, convergence test (it > 0), beta, d = z + beta
// d_old (d = z when it = 0), q = A d and <d,q>.
// (false: the solve converged at this test, or, with gate, had converged
// before the launch; nothing was written)
template <typename R, int NB>
__device__ __forceinline__ bool mgcg_dir_body(const Slot &s, int lb, int it, bool gate = false) {
  using T = R;
  const Grid G = grid_of(s);
  const SlotCtl &ctl = *s.ctl;
  SlotState *st = s.st;
  const bool mixed = s.precision != 0;
  // d = z + beta d_old; on the first iteration beta = 0 and d_old = z, so
  // d = z exactly and every load is unconditional
  const bool first = it == 0;
  const R *rAU = (const R *)s.rAU;
  const uint8_t *flags = s.flags;
  T *const cs0 = (T *)s.cs[0], *const cs1 = (T *)s.cs[1];
  const T *z = (const T *)s.cw[0], *dold = first ? z : ((it & 1) ? cs0 : cs1);
  T *dn = (it & 1) ? cs1 : cs0, *q = (T *)s.cp;
  // q = A d is formed as A z + beta q_old (the same vector in exact
  // arithmetic, as in Chronopoulos and Gear's CG), which needs d_old and
  // q_old at the cell only: one array fewer at the six neighbours.  The
  // rounding the recurrence adds stays at the level of the solve's own
  // (in the mixed path the outer FP64 refinement measures the true
  // residual; over 50 steps of the channel bubble the FP64 path stays within
  // the oracle's own round-off sensitivity).
  constexpr bool rec = true;
  struct Op {
    Cell c;
    uint8_t fl;
    T z[7], o[7];   // z and d_old across faces 0..5, then at the cell (rec: d_old at the cell only)
    R ra[7];        // rAU likewise
    T qo;           // rec: q_old at the cell
  };
  bool stop = false;
  T be = (T)0;
  double red[1] = {0.0};
  Partials<2> pt;   // the previous cycle's reduction, loaded ahead of the stencil operands
  prefetch_totals(s, CH_CG0 + ((it + 1) & 1), pt);
  const int done = gate ? st->done : 0;   // converged before this launch (tested with the totals)
  const Walk wk = cell_walk(G, lb);
  batched<NB, Op>(
      wk.first, wk.stride, wk.end,
      [&](Op &o, int t) {
        o.fl = 0x40;
        if (t < wk.end) {
          const int g = walk_at(wk, t);
          o.c = cell_at(G, g);
          o.fl = flags[g];
        }
      },
      [&](Op &o) {
        if (o.fl & 0x40) return;
        unsigned oP, on[6];
        nb_offsets(G, (unsigned)o.c.P, o.fl, sizeof(T), oP, on);
        o.z[6] = ldo(z, oP);
        o.o[6] = ldo(dold, oP);
        o.ra[6] = ldo(rAU, oP);
        if constexpr (rec) o.qo = ldo((const T *)q, oP);
#pragma unroll
        for (int f = 0; f < 6; ++f) {
          o.z[f] = ldo(z, on[f]);
          if constexpr (!rec) o.o[f] = ldo(dold, on[f]);
          o.ra[f] = ldo(rAU, on[f]);
        }
      },
      [&]() {
        if (done) {
          stop = true;
          return false;
        }
        // the scalars of the convergence test and of beta, read behind the
        // stencil operands (a wait for them ahead of the walk's set-up
        // would hold back the first loads)
        const double tgt = st->tgt, rtol = ctl.rtol, bn = st->bn;
        const int max_it = ctl.max_it;
        const double gam_old = st->gam[(it + 1) & 1];   // gamma of iteration it - 1 (unused when it = 0)
        double v[2];
        finish_totals(pt, v);   // written by the cycle of iteration it - 1
        const double gam = v[0];
        double beta = 0.0;
        if (it > 0) {
          double rn = sqrt(v[1]);
          bool conv = rn <= (mixed ? tgt : rtol * bn);
          bool cap = !conv && it >= max_it;
          if (conv || cap) {
            if (lb == 0 && threadIdx.x == 0) {
              st->rn = rn;
              st->it = it;
              st->done = 1;
              if (cap) st->maxit_hit = st->maxit_hit + 1;
            }
            stop = true;
            return false;
          }
          beta = gam / gam_old;
          if (lb == 0 && threadIdx.x == 0) st->rn = rn;
        }
        if (lb == 0 && threadIdx.x == 0) st->gam[it & 1] = gam;
        be = (T)beta;
        return true;
      },
      [&](Op &o) {
        if (o.fl & 0x40) return;
        auto dv = [&](int m) -> T { return o.z[m] + be * o.o[m]; };
        const T dP = dv(6);
        T xn[6], rn[6];
        T qq;
        if constexpr (rec) {
#pragma unroll
          for (int f = 0; f < 6; ++f) {
            xn[f] = o.z[f];
            rn[f] = (T)o.ra[f];
          }
          const T Az = matvec_pre<T>(G, o.c, o.fl, o.z[6], (T)o.ra[6], xn, rn);
          qq = first ? Az : Az + be * o.qo;
        } else {
#pragma unroll
          for (int f = 0; f < 6; ++f) {
            xn[f] = dv(f);
            rn[f] = (T)o.ra[f];
          }
          qq = matvec_pre<T>(G, o.c, o.fl, dP, (T)o.ra[6], xn, rn);
        }
        const unsigned oP = (unsigned)o.c.P * sizeof(T);
        sto(dn, oP, dP);
        sto(q, oP, qq);
        red[0] = red[0] + (double)(dP * qq);
      });
  if (stop) return false;   // uniform: every thread read the same totals
  put_partials<0u>(s, lb, CH_DQ, red);
  return true;
}

template <typename R, int NB>
__global__ void __launch_bounds__(BLOCK) k_mgcg_dir(const Slot S, int it, unsigned long long *ts) {
  OSCAR_PRIME("s"(ts), "s"(S.st), "s"(S.ctl), "s"(S.flags), "s"(S.part), "s"(S.rAU), "s"(S.cw[0]), "s"(S.cs[0]),
              "s"(S.cs[1]), "s"(S.cp), "s"(S.nblocks), "s"(S.dim), "s"(S.nx), "s"(S.ny), "s"(S.nz), "s"(S.nxy));
  OSCAR_PRIME("s"(S.nc), "s"(S.outlet), "s"(S.Sh), "s"(S.S2h), "s"(S.precision), "s"(it));
  Stamp stamp(ts);
  const int lb = xcd_block(blockIdx.x, S.nblocks);
  if (lb < 0) return;
  if (mgcg_dir_body<R, NB>(S, lb, it, true)) stamp.done();
}

// batched: the engine's block table of its multigrid slots
template <typename R, int NB>
__global__ void __launch_bounds__(BLOCK) k_mgcg_dir_b(const Slot *slots, const int2 *btab, int it) {
  const int2 t = btab[blockIdx.x];
  const Slot &s = slots[t.x];
  if (t.y < 0 || s.st->done) return;
  mgcg_dir_body<R, NB>(s, t.y, it);
}

// Iteration it >= 0: alpha = gamma / <d,q>, x += alpha d, r -= alpha q; for
// it = -1 (the cycle before the first iteration) r is the initial residual.
// Then the cycle's fine pre-smoothing z0 = w D^-1 r and the restriction of
// its residual r - A z0 into level 1, walking the fine grid in tile order.
// (with gate, false: the solve had converged before the launch; nothing was
// written)
template <typename R, int NB>
__device__ __forceinline__ bool mg_fine_down_body(const Slot &s, int lb, int it, int mode, bool gate = false) {
  using T = R;
  const Grid G = grid_of(s);
  SlotState *st = s.st;
  // the unknown the iterations update: the FP32 correction of the mixed
  // path (R = float), the FP64 pressure otherwise
  constexpr bool mixed = sizeof(T) == 4;
  const bool upd = it >= 0;
  const R *rAU = (const R *)s.rAU;
  const T *invD = (const T *)s.invD;
  // r_new = r - alpha q; for the initial cycle alpha = 0 and q = r, so
  // r_new = r exactly and every load is unconditional
  T *const cr0 = (T *)s.cr[0], *const cr1 = (T *)s.cr[1];
  const T *r0 = upd && (it & 1) ? cr1 : cr0;
  T *r1 = upd && !(it & 1) ? cr1 : cr0;
  const T *d = upd && (it & 1) ? (const T *)s.cs[1] : (const T *)s.cs[0], *q = upd ? (const T *)s.cp : r0;
  T *z0 = (T *)s.cw[1];
  T *xv = mixed ? (T *)s.e : (T *)(mode ? s.p_cr : s.p_vd);
  const int cnx = s.mg.lv[1].nx, cny = s.mg.lv[1].ny;
  T *b1 = (T *)s.mg.lv[1].b;
  const uint8_t *flags = s.flags;
  const T w = (T)MG_OMEGA_FINE;
  const int dim = G.dim;
  const int total = (int)kid_total(dim, cnx, cny, s.mg.lv[1].nz);
  // tiles in slabs of parent planes (3D): kid_total is a whole number of
  // parent rows of tiles of 64 lanes
  const int cnz1 = s.mg.lv[1].nz;
  const Walk wk = slab_walk(lb, G.nblocks, cnz1, cny, total / (cnz1 * cny), dim == 3);
  struct Op {
    Cell c;
    int parent;
    bool lead;
    uint8_t fl;
    T r[7], q[7], iD[7];   // r, q, D^-1 across faces 0..5, then at the cell
    R ra[7];               // rAU likewise
    T d, x;                // search direction and unknown at the cell (read also when unused)
  };
  T al = (T)0;
  Partials<1> pt;   // <d,q> of the search-direction launch, loaded ahead of the stencil operands
  prefetch_totals(s, CH_DQ, pt);   // (unused by the initial cycle; loading it anyway avoids a branch)
  const int done = gate ? st->done : 0;   // converged before this launch (tested with the first loads)
  batched<NB, Op>(
      wk.first, wk.stride, wk.end,
      [&](Op &o, int t) {
        o.fl = 0x40;
        o.lead = false;
        o.parent = 0;
        if (t < wk.end) {
          const Kid k = kid_at((unsigned)walk_at(wk, t), dim, G.nx, G.ny, G.nz, cnx, cny);
          o.parent = k.parent;
          o.lead = k.lead;
          if (k.valid) {
            o.c.P = k.P;
            o.c.i = k.i;
            o.c.j = k.j;
            o.c.k = k.k;
            o.c.row = k.j + G.ny * k.k;
            o.c.valid = true;
            o.fl = flags[k.P];
          }
        }
      },
      [&](Op &o) {
        if (o.fl & 0x40) return;
        unsigned oP, on[6];
        nb_offsets(G, (unsigned)o.c.P, o.fl, sizeof(T), oP, on);
        o.r[6] = ldo(r0, oP);
        o.q[6] = ldo(q, oP);
        o.iD[6] = ldo(invD, oP);
        o.ra[6] = ldo(rAU, oP);
#pragma unroll
        for (int f = 0; f < 6; ++f) {
          o.r[f] = ldo(r0, on[f]);
          o.q[f] = ldo(q, on[f]);
          o.iD[f] = ldo(invD, on[f]);
          o.ra[f] = ldo(rAU, on[f]);
        }
        o.d = ldo(d, oP);
        o.x = ldo(xv, oP);
      },
      [&]() {
        if (done) return false;
        if (!upd) return true;
        double v[1];
        finish_totals(pt, v);
        al = (T)(st->gam[it & 1] / v[0]);
        if (lb == 0 && threadIdx.x == 0) {
          st->it = it + 1;
          st->total_it = st->total_it + 1;
        }
        return true;
      },
      [&](Op &o) {
        T tv = (T)0;
        if (!(o.fl & 0x40)) {
          const int P = o.c.P;
          auto rv = [&](int m) -> T { return o.r[m] - al * o.q[m]; };
          auto zv = [&](int m) -> T { return w * (o.iD[m] * rv(m)); };
          const T rn = rv(6);
          const T zz = zv(6);
          T xn[6], ran[6];
#pragma unroll
          for (int f = 0; f < 6; ++f) {
            xn[f] = zv(f);
            ran[f] = (T)o.ra[f];
          }
          const T Az = matvec_pre<T>(G, o.c, o.fl, zz, (T)o.ra[6], xn, ran);
          const unsigned oP = (unsigned)P * sizeof(T);
          if (upd) {
            sto(xv, oP, o.x + al * o.d);
            sto(r1, oP, rn);
          }
          sto(z0, oP, zz);
          tv = rn - Az;
        }
        tv = kid_sum(tv, dim);
        if (o.lead) b1[o.parent] = tv;
      });
  return !done;
}

// ---------------------------------------------------------------------------
// the same step on LDS-staged bricks (large 3D FP32 grids)
// ---------------------------------------------------------------------------
// The single-cell kernel above holds every stencil operand of its cells in
// registers, so the registers bound the loads a wavefront keeps in flight
// and, on a grid that streams from HBM, the kernel waits on memory latency.
// Here a workgroup takes bricks of 32 x 8 x 4 fine cells: the halo brick of
// r, q, D^-1 and rAU (34 x 10 x 6 cells, read as rows of ten 16-byte chunks
// from x0 - 4) goes straight from memory into LDS with global_load_lds
// (no registers held), all of it in flight at once; after one wait the
// cells are computed from LDS.  Thread t holds the four children at z
// offset t & 1 of parent t >> 1 of the brick (16 x 4 x 2 parents), so the
// restriction sums x, then y in the thread and z across lanes t, t ^ 1: the
// order of kid_sum.  Each cell's arithmetic is the single-cell kernel's.
// Rows and chunks outside the grid read the nearest in-grid ones (only
// faces that are not interior see them).
typedef float f2v __attribute__((ext_vector_type(2)));
typedef double d2v __attribute__((ext_vector_type(2)));
template <typename T>
struct PairOf;   // two elements of T as one vector (an x pair of cells)
template <>
struct PairOf<float> {
  typedef f2v type;
};
template <>
struct PairOf<double> {
  typedef d2v type;
};

// store the fluid cells of an x pair (one store when both are fluid)
template <typename T>
__device__ __forceinline__ void sto_pair(T *base, unsigned off, bool fa, bool fb, T a, T b) {
  typedef typename PairOf<T>::type P2;
  if (fa && fb) {
    P2 v;
    v.x = a;
    v.y = b;
    sto((P2 *)base, off, v);
  } else {
    if (fa) sto(base, off, a);
    if (fb) sto(base, off + (unsigned)sizeof(T), b);
  }
}

constexpr int BRX = 32, BRY = 8, BRZ = 4;
constexpr int BRP = BRX + 8;                    // LDS row pitch (elements: x0 - 4 .. x0 + 35)
constexpr int BRROWS = (BRY + 2) * (BRZ + 2);   // halo rows
constexpr int BRH = BRROWS * BRP;               // elements per staged array
static_assert(BRX * BRY * BRZ == 4 * BLOCK, "four cells per thread");
template <typename T>
constexpr int BRCW = 16 / (int)sizeof(T);       // elements per 16-byte chunk
template <typename T>
constexpr int BRCH = BRROWS * (BRP / BRCW<T>);  // 16-byte chunks per staged array

// 3D grids of at least WALK_MIN cells whose dimensions are multiples of the brick
__host__ __device__ inline bool brick_ok(int dim, int nx, int ny, int nz) {
  return dim == 3 && nx % BRX == 0 && ny % BRY == 0 && nz % BRZ == 0 && (long long)nx * ny * nz >= WALK_MIN;
}

// Chunk c of the halo brick (row c / (BRP / BRCW) of the (BRY + 2) x
// (BRZ + 2) halo rows, 16-byte chunk c % (BRP / BRCW) from x0 - 4), clamped
// into the grid: its element offset.
template <typename T>
__device__ __forceinline__ unsigned brick_chunk(const Grid &G, int c, int x0, int y0, int z0) {
  constexpr int W = BRCW<T>, PER = BRP / W;
  const int row = c / PER, ch = c - row * PER;
  const int zz = row / (BRY + 2), yy = row - zz * (BRY + 2);
  int y = y0 - 1 + yy, z = z0 - 1 + zz, x = x0 - 4 + W * ch;
  y = y < 0 ? 0 : (y >= G.ny ? G.ny - 1 : y);
  z = z < 0 ? 0 : (z >= G.nz ? G.nz - 1 : z);
  x = x < 0 ? 0 : (x > G.nx - W ? G.nx - W : x);
  return (unsigned)x + (unsigned)G.nx * ((unsigned)y + (unsigned)G.ny * (unsigned)z);
}

template <typename T>
constexpr int BRM = (BRCH<T> + BLOCK - 1) / BLOCK;   // chunk rounds of a workgroup

// stage the halo brick of one array to LDS (chunk c at byte 16 c;
// wavefront-uniform LDS bases), skipping the chunks whose cells are all
// solid (need[m] false): solid cells' values are never read
template <typename T>
__device__ __forceinline__ void brick_stage(const T *src, T *lds, const unsigned (&off)[BRM<T>],
                                            const bool (&need)[BRM<T>]) {
  const int wave = (int)threadIdx.x >> 6, lane = (int)threadIdx.x & 63;
#pragma unroll
  for (int m = 0; m < BRM<T>; ++m) {
    const int c = m * BLOCK + wave * 64 + lane;
    if (m * BLOCK + wave * 64 < BRCH<T> && c < BRCH<T> && need[m])
      __builtin_amdgcn_global_load_lds(
          (const OSCAR_GLOBAL void *)(src + off[m]),
          (__attribute__((address_space(3))) void *)(lds + BRCW<T> * (m * BLOCK + wave * 64)), 16, 0, 0);
  }
}

// the bricks of workgroup lb: the 8 XCDs (contiguous runs of lb, as
// xcd_block deals them) each take a slab of brick planes, and a run's
// workgroups take its bricks in turn; without 8 planes, bricks lb,
// lb + nblocks, ...
struct BrickWalk {
  int first, stride, end;
};
__device__ __forceinline__ BrickWalk brick_walk(int lb, int nblocks, int nbx, int nby, int nbz) {
  BrickWalk w;
  if (nblocks < 8 || nbz < 8) {
    w.first = lb;
    w.stride = nblocks;
    w.end = nbx * nby * nbz;
    return w;
  }
  const int X = 8, q = nblocks / X, rem = nblocks % X;
  int x, l0;
  if (lb < rem * (q + 1)) {
    x = lb / (q + 1);
    l0 = x * (q + 1);
  } else {
    x = rem + (lb - rem * (q + 1)) / q;
    l0 = x * q + rem;
  }
  const int cnt = q + (x < rem ? 1 : 0);
  const int per = nbx * nby;
  w.first = (x * nbz / X) * per + (lb - l0);
  w.stride = cnt;
  w.end = ((x + 1) * nbz / X) * per;
  return w;
}

// (false: the solve had converged before the launch; nothing was written)
template <typename T>
__device__ __forceinline__ bool mg_fine_down_brick(const Slot &s, int lb, int it, int mode) {
  const Grid G = grid_of(s);
  SlotState *st = s.st;
  const int done = st->done;   // converged before this launch (tested once the first brick is in flight)
  const bool upd = it >= 0;
  const T *rAU = (const T *)s.rAU;
  const T *invD = (const T *)s.invD;
  T *const cr0 = (T *)s.cr[0], *const cr1 = (T *)s.cr[1];
  const T *r0 = upd && (it & 1) ? cr1 : cr0;
  T *r1 = upd && !(it & 1) ? cr1 : cr0;
  const T *d = upd && (it & 1) ? (const T *)s.cs[1] : (const T *)s.cs[0], *q = upd ? (const T *)s.cp : r0;
  T *z0 = (T *)s.cw[1];
  // the unknown the iterations update (as in the single-cell kernel)
  T *xv = sizeof(T) == 4 ? (T *)s.e : (T *)(mode ? s.p_cr : s.p_vd);
  const int cnx = s.mg.lv[1].nx, cny = s.mg.lv[1].ny;
  T *b1 = (T *)s.mg.lv[1].b;
  const uint8_t *flags = s.flags;
  const T w = (T)MG_OMEGA_FINE;
  typedef typename PairOf<T>::type P2;
  constexpr int NM = BRM<T>;
  __shared__ __align__(16) T sr[BRH];
  __shared__ __align__(16) T sq[BRH];
  __shared__ __align__(16) T si[BRH];
  __shared__ __align__(16) T sa[BRH];
  const int nbx = G.nx / BRX, nby = G.ny / BRY, nbz = G.nz / BRZ;
  const BrickWalk wk = brick_walk(lb, G.nblocks, nbx, nby, nbz);
  const int tid = (int)threadIdx.x;
  const int p = tid >> 1, h = tid & 1;
  const int px = p & 15, py = (p >> 4) & 3, pz = p >> 6;
  const int cx = 2 * px, cy = 2 * py, cz = 2 * pz + h;   // the thread's first child in the brick
  auto origin = [&](int b, int &x0, int &y0, int &z0b) {
    const int bz = b / (nbx * nby), rem = b - bz * nbx * nby, by = rem / nbx;
    x0 = (rem - by * nbx) * BRX;
    y0 = by * BRY;
    z0b = bz * BRZ;
  };
  // the brick's chunks: their offsets, and the flags of their cells (one
  // load of four or two flag bytes each) to skip the all-solid ones
  auto stage = [&](int b) {
    int x0, y0, z0b;
    origin(b, x0, y0, z0b);
    unsigned off[NM];
    bool need[NM];
#pragma unroll
    for (int m = 0; m < NM; ++m) {
      const int c = m * BLOCK + tid;
      off[m] = brick_chunk<T>(G, c < BRCH<T> ? c : 0, x0, y0, z0b);
      if constexpr (BRCW<T> == 4) need[m] = (ldo((const uint32_t *)flags, off[m]) & 0x40404040u) != 0x40404040u;
      else need[m] = (ldo((const uint16_t *)flags, off[m]) & 0x4040u) != 0x4040u;
    }
    brick_stage<T>(r0, sr, off, need);
    brick_stage<T>(q, sq, off, need);
    brick_stage<T>(invD, si, off, need);
    brick_stage<T>(rAU, sa, off, need);
  };
  if (wk.first < wk.end) stage(wk.first);
  if (done) {   // uniform; no LDS transfer may outlive the workgroup
    __builtin_amdgcn_s_waitcnt(0);
    return false;
  }
  // the previous launch's <d,q> while the first brick loads
  T al = (T)0;
  if (upd) {
    Partials<1> pt;
    prefetch_totals(s, CH_DQ, pt);
    double v[1];
    finish_totals(pt, v);
    al = (T)(st->gam[it & 1] / v[0]);
    if (lb == 0 && tid == 0) {
      st->it = it + 1;
      st->total_it = st->total_it + 1;
    }
  }
  for (int b = wk.first; b < wk.end; b += wk.stride) {
    int x0, y0, z0b;
    origin(b, x0, y0, z0b);
    // the thread's own cells: two x pairs (rows y and y + 1)
    const int gi = x0 + cx, gj = y0 + cy, gk = z0b + cz;
    const int P0 = gi + G.nx * (gj + G.ny * gk), P1 = P0 + G.nx;
    const unsigned fl0 = (unsigned)ldo((const uint16_t *)flags, (unsigned)P0);
    const unsigned fl1 = (unsigned)ldo((const uint16_t *)flags, (unsigned)P1);
    constexpr unsigned WB = (unsigned)sizeof(T);
    const P2 d0 = ldo((const P2 *)d, (unsigned)P0 * WB), d1 = ldo((const P2 *)d, (unsigned)P1 * WB);
    const P2 xo0 = ldo((const P2 *)xv, (unsigned)P0 * WB), xo1 = ldo((const P2 *)xv, (unsigned)P1 * WB);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    T tv[2][2];
#pragma unroll
    for (int yk = 0; yk < 2; ++yk) {
      T zz[2], rnv[2], xn2[2];
      bool fl[2];
#pragma unroll
      for (int xk = 0; xk < 2; ++xk) {
        const uint8_t f8 = (uint8_t)((yk ? fl1 : fl0) >> (8 * xk));
        fl[xk] = !(f8 & 0x40);
        tv[yk][xk] = (T)0;
        zz[xk] = rnv[xk] = xn2[xk] = (T)0;
        if (!fl[xk]) continue;
        const int L = ((cz + 1) * (BRY + 2) + (cy + yk + 1)) * BRP + (cx + xk + 4);
        const int off[6] = {-1, 1, -BRP, BRP, -(BRY + 2) * BRP, (BRY + 2) * BRP};
        const T rn = sr[L] - al * sq[L];
        const T zc = w * (si[L] * rn);
        T xn[6], ran[6];
#pragma unroll
        for (int f = 0; f < 6; ++f) {
          const int Lf = L + off[f];
          xn[f] = w * (si[Lf] * (sr[Lf] - al * sq[Lf]));
          ran[f] = sa[Lf];
        }
        Cell c;
        c.P = (yk ? P1 : P0) + xk;
        c.i = gi + xk;
        c.j = gj + yk;
        c.k = gk;
        c.row = c.j + G.ny * c.k;
        c.valid = true;
        const T Az = matvec_pre<T>(G, c, f8, zc, sa[L], xn, ran);
        zz[xk] = zc;
        rnv[xk] = rn;
        const P2 dd = yk ? d1 : d0;
        const P2 xo = yk ? xo1 : xo0;
        xn2[xk] = (xk ? xo.y : xo.x) + al * (xk ? dd.y : dd.x);
        tv[yk][xk] = rn - Az;
      }
      const unsigned o = (unsigned)(yk ? P1 : P0) * WB;
      if (upd) {
        sto_pair<T>(xv, o, fl[0], fl[1], xn2[0], xn2[1]);
        sto_pair<T>(r1, o, fl[0], fl[1], rnv[0], rnv[1]);
      }
      sto_pair<T>(z0, o, fl[0], fl[1], zz[0], zz[1]);
    }
    // children of the parent: x pairs, then y, then z across the lane pair
    T v = (tv[0][0] + tv[0][1]) + (tv[1][0] + tv[1][1]);
    v = v + lane_move(v, lane_x1);
    if (h == 0) b1[(gi >> 1) + cnx * ((gj >> 1) + cny * (gk >> 1))] = v;
    __syncthreads();   // every wavefront is done with the LDS: stage the next brick
    if (b + wk.stride < wk.end) stage(b + wk.stride);
  }
  return true;
}

// (FP32: four wavefronts per SIMD, 128 registers, the LDS of four
// workgroups fits; FP64: the 77 KB of two workgroups per CU)
template <typename T>
__global__ void __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 2)))
k_mg_fine_down_brick(const Slot S, int it, int mode, unsigned long long *ts) {
  OSCAR_PRIME("s"(ts), "s"(S.st), "s"(S.flags), "s"(S.part), "s"(S.rAU), "s"(S.invD), "s"(S.cr[0]), "s"(S.cr[1]),
              "s"(S.cs[0]), "s"(S.cs[1]), "s"(S.cp), "s"(S.cw[1]), "s"(S.e), "s"(S.nblocks), "s"(S.nx), "s"(S.ny));
  OSCAR_PRIME("s"(S.nz), "s"(S.nxy), "s"(S.outlet), "s"(S.Sh), "s"(S.S2h), "s"(S.mg.lv[1].nx), "s"(S.mg.lv[1].ny),
              "s"(S.mg.lv[1].b), "s"(it));
  Stamp stamp(ts);
  const int lb = xcd_block(blockIdx.x, S.nblocks);
  if (lb < 0) return;
  if (mg_fine_down_brick<T>(S, lb, it, mode)) stamp.done();
}

template <typename R, int NB>
__global__ void __launch_bounds__(BLOCK) k_mg_fine_down(const Slot S, int it, int mode, unsigned long long *ts) {
  OSCAR_PRIME("s"(ts), "s"(S.st), "s"(S.flags), "s"(S.part), "s"(S.rAU), "s"(S.invD), "s"(S.cr[0]), "s"(S.cr[1]),
              "s"(S.cs[0]), "s"(S.cs[1]), "s"(S.cp), "s"(S.cw[1]), "s"(S.e), "s"(S.nblocks), "s"(S.dim), "s"(S.nx));
  OSCAR_PRIME("s"(S.ny), "s"(S.nz), "s"(S.nxy), "s"(S.nc), "s"(S.outlet), "s"(S.Sh), "s"(S.S2h), "s"(S.mg.lv[1].nx),
              "s"(S.mg.lv[1].ny), "s"(S.mg.lv[1].nz), "s"(S.mg.lv[1].b), "s"(it));
  Stamp stamp(ts);
  const int lb = xcd_block(blockIdx.x, S.nblocks);
  if (lb < 0) return;
  if (mg_fine_down_body<R, NB>(S, lb, it, mode, true)) stamp.done();
}

template <typename R, int NB>
__global__ void __launch_bounds__(BLOCK) k_mg_fine_down_b(const Slot *slots, const int2 *btab, int it) {
  const int2 t = btab[blockIdx.x];
  const Slot &s = slots[t.x];
  if (t.y < 0 || s.st->done) return;
  mg_fine_down_body<R, NB>(s, t.y, it, s.ctl->mode);
}

// Last step of the cycle: z' = z0 + P x1, z = z' + w D^-1 (r - A z'); the
// reduction <r,z>, |r|^2 for the next search direction.
template <typename R, int NB>
__device__ __forceinline__ bool mg_fine_up_body(const Slot &s, int lb, int it, bool gate = false) {
  using T = R;
  const Grid G = grid_of(s);
  const uint8_t *flags = s.flags;
  const R *rAU = (const R *)s.rAU;
  const T *invD = (const T *)s.invD;
  const T *r = (it & 1) ? (const T *)s.cr[0] : (const T *)s.cr[1];
  const T *z0 = (const T *)s.cw[1];
  T *z = (T *)s.cw[0];
  const int cnx = s.mg.lv[1].nx, cnxy = s.mg.lv[1].nxy;
  const T *xc = (const T *)s.mg.lv[1].t;
  const T w = (T)MG_OMEGA_FINE;
  struct Op {
    Cell c;
    uint8_t fl;
    T z0[7], xc[7];   // z0 and the parent's correction across faces 0..5, then at the cell
    R ra[7];          // rAU likewise
    T r, iD;
  };
  double red[2] = {0.0, 0.0};
  const int done = gate ? s.st->done : 0;   // converged before this launch (tested with the first loads)
  const Walk wk = cell_walk(G, lb);
  batched<NB, Op>(
      wk.first, wk.stride, wk.end,
      [&](Op &o, int t) {
        o.fl = 0x40;
        if (t < wk.end) {
          const int g = walk_at(wk, t);
          o.c = cell_at(G, g);
          o.fl = flags[g];
        }
      },
      [&](Op &o) {
        if (o.fl & 0x40) return;
        const Cell &c = o.c;
        const int pP = (c.i >> 1) + cnx * (c.j >> 1) + cnxy * (c.k >> 1);
        const int q[3] = {c.i, c.j, c.k};
        const int cst[3] = {1, cnx, cnxy};
        unsigned oP, on[6];
        nb_offsets(G, (unsigned)c.P, o.fl, sizeof(T), oP, on);
        const unsigned opP = (unsigned)pP * sizeof(T);
        o.z0[6] = ldo(z0, oP);
        o.xc[6] = ldo(xc, opP);
        o.ra[6] = ldo(rAU, oP);
        o.r = ldo(r, oP);
        o.iD = ldo(invD, oP);
#pragma unroll
        for (int f = 0; f < 6; ++f) {
          const bool in = (o.fl >> f) & 1u;
          // parent of the neighbour: it changes across the face iff the face is a parent's face
          const int pn = in ? pP + parent_shift(q[f >> 1], (f & 1) ? 1 : -1, cst[f >> 1]) : pP;
          o.z0[f] = ldo(z0, on[f]);
          o.xc[f] = ldo(xc, (unsigned)pn * sizeof(T));
          o.ra[f] = ldo(rAU, on[f]);
        }
      },
      [&]() { return !done; },
      [&](Op &o) {
        if (o.fl & 0x40) return;
        auto zp = [&](int m) -> T { return o.z0[m] + o.xc[m]; };
        const T zP = zp(6);
        T xn[6], rn[6];
#pragma unroll
        for (int f = 0; f < 6; ++f) {
          xn[f] = zp(f);
          rn[f] = (T)o.ra[f];
        }
        const T Az = matvec_pre<T>(G, o.c, o.fl, zP, (T)o.ra[6], xn, rn);
        const T rr = o.r;
        const T zn = zP + w * (o.iD * (rr - Az));
        sto(z, (unsigned)o.c.P * sizeof(T), zn);
        red[0] = red[0] + (double)(rr * zn);
        red[1] = red[1] + (double)(rr * rr);
      });
  if (done) return false;   // uniform
  put_partials<0u>(s, lb, CH_CG0 + (it & 1), red);
  return true;
}

template <typename R, int NB>
__global__ void __launch_bounds__(BLOCK) k_mg_fine_up(const Slot S, int it, unsigned long long *ts) {
  OSCAR_PRIME("s"(ts), "s"(S.st), "s"(S.flags), "s"(S.part), "s"(S.rAU), "s"(S.invD), "s"(S.cr[0]), "s"(S.cr[1]),
              "s"(S.cw[0]), "s"(S.cw[1]), "s"(S.nblocks), "s"(S.dim), "s"(S.nx), "s"(S.ny), "s"(S.nz), "s"(S.nxy));
  OSCAR_PRIME("s"(S.nc), "s"(S.outlet), "s"(S.Sh), "s"(S.S2h), "s"(S.mg.lv[1].nx), "s"(S.mg.lv[1].nxy),
              "s"(S.mg.lv[1].t), "s"(it));
  Stamp stamp(ts);
  const int lb = xcd_block(blockIdx.x, S.nblocks);
  if (lb < 0) return;
  if (mg_fine_up_body<R, NB>(S, lb, it, true)) stamp.done();
}

template <typename R, int NB>
__global__ void __launch_bounds__(BLOCK) k_mg_fine_up_b(const Slot *slots, const int2 *btab, int it) {
  const int2 t = btab[blockIdx.x];
  const Slot &s = slots[t.x];
  if (t.y < 0 || s.st->done) return;
  mg_fine_up_body<R, NB>(s, t.y, it);
}

// ---------------------------------------------------------------------------
// persistent pressure solve
// ---------------------------------------------------------------------------
// One launch runs the whole pressure solve -- every CG iteration, V-cycle
// and FP64 refinement step -- of every slot of a batch.  A slot's solve is a
// chain of phases, the steps the grid-wide path launches as kernels; a phase
// is made of tiles: the slot's fine blocks, the blocks of a coarse level, or
// one tile (the tail, the refinement's finaliser).  A tile runs the body of
// the grid-wide kernel on the same block, so the results are bitwise those of
// the grid-wide path.
//
// Work queue: each slot publishes its open phase in one 64-bit word of its
// state (generation, tiles, tiles claimed).  A workgroup finds a slot with an
// unclaimed tile (one wavefront polls 64 slots at once), claims the tile with
// an atomic add on that word, runs it, and counts it complete; the workgroup
// that completes the last tile of a phase decides the next phase from the
// slot's state and publishes it.  Slots advance independently of each other
// and no host round trip separates their steps.
//
// Ordering: a tile's stores are released (agent scope) by every thread before
// its completion is counted; the deciding workgroup acquires before it reads
// the slot's state, and releases the next phase before its word; a claimer
// acquires before it reads the phase.  No workgroup waits for another except
// to find work, so any number of resident workgroups makes progress; the
// launch ends when every slot's solve has finished, or when no phase has
// completed for idle_ticks of the wall clock (g->err: the host reports it).
enum : int { PQ_FD = 0, PQ_SM, PQ_TAIL, PQ_UP, PQ_FU, PQ_DIR, PQ_CGI, PQ_CG, PQ_RX, PQ_RR, PQ_RF, PQ_FIN };

struct PQPhase {
  int ph, it, l;   // kind, CG iteration, coarse level
};

__device__ __forceinline__ unsigned long long pq_pack(unsigned gen, int tiles) {
  return ((unsigned long long)gen << 32) | ((unsigned long long)(unsigned)tiles << 16);
}
__device__ __forceinline__ unsigned pq_gen(unsigned long long w) { return (unsigned)(w >> 32); }
__device__ __forceinline__ int pq_ntiles(unsigned long long w) { return (int)((w >> 16) & 0xffffu); }
// claims past the tiles stay below 2^16: a workgroup adds only after it saw
// an unclaimed tile, so the excess is at most the launch's workgroups
__device__ __forceinline__ int pq_claimed(unsigned long long w) { return (int)(w & 0xffffu); }

__device__ inline int pq_tiles(const Slot &s, const PQPhase &p) {
  switch (p.ph) {
    case PQ_SM: return smooth_blocks(s.mg, p.l, s.dim);
    case PQ_UP: return up_blocks(s.mg, p.l);
    case PQ_TAIL:
    case PQ_RF: return 1;
    case PQ_FIN: return 0;
    default: return s.nblocks;
  }
}

// first phase of a solve whose set-up has run: none if the set-up found the
// equation solved (zero right-hand side, or an initial residual within the
// tolerance), else the cycle of r_0 (multigrid) or w_0 = A D^-1 r_0 (Jacobi)
__device__ inline PQPhase pq_first(const Slot &s) {
  if (s.st->done) return PQPhase{PQ_FIN, 0, 0};
  return s.mg_pc ? PQPhase{PQ_FD, -1, 0} : PQPhase{PQ_CGI, 0, 0};
}

// The phase after p, once all of p's tiles have completed: the launch order
// of the grid-wide path (cycle: fine down, the coarse levels down, the tail,
// the coarse levels up, fine up; then the search direction of the next
// iteration, which holds the convergence test), and after a finished inner
// solve the refinement when it is due; after the refinement, the end if it
// met the tolerance or stalled, else a new inner solve.
__device__ inline PQPhase pq_next(const Slot &s, const PQPhase &p) {
  const int tail = s.mg.tail;
  const SlotState *st = s.st;
  auto after_inner = [&]() -> PQPhase { return refine_due(s, *s.ctl) ? PQPhase{PQ_RX, 0, 0} : PQPhase{PQ_FIN, 0, 0}; };
  switch (p.ph) {
    case PQ_FD: return tail > 1 ? PQPhase{PQ_SM, p.it, 1} : PQPhase{PQ_TAIL, p.it, 0};
    case PQ_SM: return p.l + 1 < tail ? PQPhase{PQ_SM, p.it, p.l + 1} : PQPhase{PQ_TAIL, p.it, 0};
    case PQ_TAIL: return tail > 1 ? PQPhase{PQ_UP, p.it, tail - 1} : PQPhase{PQ_FU, p.it, 0};
    case PQ_UP: return p.l > 1 ? PQPhase{PQ_UP, p.it, p.l - 1} : PQPhase{PQ_FU, p.it, 0};
    case PQ_FU: return PQPhase{PQ_DIR, p.it + 1, 0};
    case PQ_DIR: return st->done ? after_inner() : PQPhase{PQ_FD, p.it, 0};
    case PQ_CGI: return PQPhase{PQ_CG, 0, 0};
    case PQ_CG: return st->done ? after_inner() : PQPhase{PQ_CG, p.it + 1, 0};
    case PQ_RX: return PQPhase{PQ_RR, 0, 0};
    case PQ_RR: return PQPhase{PQ_RF, 0, 0};
    case PQ_RF:
      if (st->done) return PQPhase{PQ_FIN, 0, 0};
      return s.mg_pc ? PQPhase{PQ_FD, -1, 0} : PQPhase{PQ_CGI, 0, 0};
    default: return PQPhase{PQ_FIN, 0, 0};
  }
}

template <int DIM, typename T>
__device__ __forceinline__ void pq_coarse(const Slot &s, const PQPhase &p, int t, uint4 *lds, int lds_bytes) {
  const int tid = (int)threadIdx.x;
  const bool two = (s.mg.nu2 >> p.l) & 1;
  if (p.ph == PQ_SM) {
    const unsigned nb = (unsigned)smooth_blocks(s.mg, p.l, DIM);
    const unsigned start = (unsigned)t * BLOCK + (unsigned)tid, stride = nb * BLOCK;
    if (two) mg_smooth_body<DIM, T, 2>(s, p.l, start, stride);
    else mg_smooth_body<DIM, T, 1>(s, p.l, start, stride);
  } else if (p.ph == PQ_UP) {
    const int nb = up_blocks(s.mg, p.l);
    if (two) mg_up_body<DIM, T, 2>(s, p.l, t * BLOCK + tid, nb * BLOCK);
    else mg_up_body<DIM, T, 1>(s, p.l, t * BLOCK + tid, nb * BLOCK);
  } else {
    if (s.mg.tail_bytes <= lds_bytes) mg_tail_body<DIM, T, true>(s, lds, tid, BLOCK);
    else mg_tail_body<DIM, T, false>(s, nullptr, tid, BLOCK);
  }
}

// tile t of phase p of slot s
template <typename R>
__device__ __forceinline__ void pq_tile(const Slot &s, const PQPhase &p, int t, uint4 *lds, int lds_bytes) {
  constexpr int NB = FINE_NB<R>;
  switch (p.ph) {
    case PQ_FD: mg_fine_down_body<R, NB>(s, t, p.it, s.ctl->mode); break;
    case PQ_SM:
    case PQ_TAIL:
    case PQ_UP:
      if (s.dim == 3) pq_coarse<3, R>(s, p, t, lds, lds_bytes);
      else pq_coarse<2, R>(s, p, t, lds, lds_bytes);
      break;
    case PQ_FU: mg_fine_up_body<R, NB>(s, t, p.it); break;
    case PQ_DIR: (void)mgcg_dir_body<R, NB>(s, t, p.it); break;
    case PQ_CGI: cg_init_body<R>(s, t); break;
    case PQ_CG: (void)cg_iter_body<R>(s, t, p.it); break;
    case PQ_RX: refine_x_body<R>(s, *s.ctl, t); break;
    case PQ_RR: refine_res_body<R>(s, *s.ctl, t); break;
    case PQ_RF: refine_fin_body(s); break;
    default: break;
  }
}

__device__ __forceinline__ const Slot &pq_slot(const Slot *slots, const int *list, int k) {
  return slots[list ? list[k] : k];
}

// one workgroup: every listed slot's first phase and the batch words
__global__ void __launch_bounds__(BLOCK) k_pq_init(const Slot *slots, const int *list, int n, PQGlobal *g) {
  int open = 0;
  for (int k = (int)threadIdx.x; k < n; k += BLOCK) {
    const Slot &s = pq_slot(slots, list, k);
    SlotState *st = s.st;
    const PQPhase p = pq_first(s);
    st->pq_phase = p.ph;
    st->pq_it = p.it;
    st->pq_lvl = p.l;
    st->pq_done = 0;
    st->pq_word = pq_pack(0u, pq_tiles(s, p));
    st->solve_base = st->total_it;
    open += p.ph != PQ_FIN;
  }
  __shared__ int sh[BLOCK / 64];
  for (int off = 32; off > 0; off >>= 1) open += __shfl_down(open, off, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = open;
  __syncthreads();
  if (threadIdx.x == 0) {
    int tot = 0;
    for (int w = 0; w < BLOCK / 64; ++w) tot += sh[w];
    g->remaining = tot;
    g->err = 0;
    g->progress = 0u;
  }
}

// a chunk of a slot list, passed by value (no host buffer outlives the call)
struct PQListChunk {
  static constexpr int MAXN = 256;
  int32_t off, n;
  int32_t v[MAXN];
};
__global__ void __launch_bounds__(BLOCK) k_pq_list(int *dst, const PQListChunk c) {
  if ((int)threadIdx.x < c.n) dst[c.off + (int)threadIdx.x] = c.v[threadIdx.x];
}

// (three wavefronts per SIMD: 168 registers, enough for the radius-2 3D
// coarse sweeps with little spilling)
template <typename R>
__global__ void __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(3)))
k_pq_solve(const Slot *slots, const int *list, int n, PQGlobal *g, int lds_bytes, long long idle_ticks) {
  extern __shared__ uint4 pq_lds[];
  // the claimed tile: list index, phase, iteration, level, tile, tiles of the
  // phase, whether the phase is new to this workgroup (phase < 0: exit)
  __shared__ int task[7];
  const int tid = (int)threadIdx.x, lane = tid & 63;
  // wavefront 0 finds the work; these stay uniform over its lanes
  int rot = (int)(blockIdx.x % (unsigned)n);   // where the next scan starts
  int cur = -1;                                // slot and generation of the last tile
  unsigned cur_gen = 0u;
  for (;;) {
    if (tid < 64) {
      int k = -1, tile = 0, ntiles = 0;
      unsigned gen = 0u, prog = 0u;
      long long t_idle = -1;
      bool quit = false;
      for (;;) {
        for (int base = 0; base < n && k < 0; base += 64) {
          int kk = -1;
          bool open = false;
          if (base + lane < n) {
            kk = base + lane + rot;
            if (kk >= n) kk -= n;
            const unsigned long long w = __hip_atomic_load(&pq_slot(slots, list, kk).st->pq_word, __ATOMIC_RELAXED,
                                                           __HIP_MEMORY_SCOPE_AGENT);
            open = pq_claimed(w) < pq_ntiles(w);
          }
          unsigned long long m = __ballot(open);
          while (m && k < 0) {
            const int src = __ffsll((long long)m) - 1;
            m &= m - 1;
            const int cand = __shfl(kk, src, 64);
            unsigned long long old = 0ull;
            if (lane == 0)
              old = __hip_atomic_fetch_add(&pq_slot(slots, list, cand).st->pq_word, 1ull, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
            const unsigned lo = __shfl((unsigned)old, 0, 64), hi = __shfl((unsigned)(old >> 32), 0, 64);
            old = ((unsigned long long)hi << 32) | lo;
            if (pq_claimed(old) < pq_ntiles(old)) {
              k = cand;
              tile = pq_claimed(old);
              ntiles = pq_ntiles(old);
              gen = pq_gen(old);
            }
          }
        }
        if (k >= 0) break;
        // nothing open: every solve finished, the launch gave up, or a
        // phase is closing
        if (__hip_atomic_load(&g->remaining, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0 ||
            __hip_atomic_load(&g->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
          quit = true;
          break;
        }
        const unsigned pr = __hip_atomic_load(&g->progress, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const long long now = (long long)wall_clock64();
        if (t_idle < 0 || pr != prog) {
          prog = pr;
          t_idle = now;
        } else if (now - t_idle > idle_ticks) {
          if (lane == 0) __hip_atomic_store(&g->err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          quit = true;
          break;
        }
        __builtin_amdgcn_s_sleep(32);
      }
      if (lane == 0) {
        if (quit) {
          task[1] = -1;
        } else {
          // the phase's publication, and all the stores released before it
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
          const SlotState *st = pq_slot(slots, list, k).st;
          task[0] = k;
          task[1] = st->pq_phase;
          task[2] = st->pq_it;
          task[3] = st->pq_lvl;
          task[4] = tile;
          task[5] = ntiles;
          task[6] = k != cur || gen != cur_gen;
        }
      }
      if (!quit) {
        cur = k;
        cur_gen = gen;
        rot = k;   // stay with this slot while it has tiles
      }
    }
    __syncthreads();
    const int ph = task[1];
    if (ph < 0) break;
    const int k = task[0], tile = task[4], ntiles = task[5];
    const PQPhase p = {ph, task[2], task[3]};
    if (task[6]) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    const Slot &s = pq_slot(slots, list, k);
    pq_tile<R>(s, p, tile, pq_lds, lds_bytes);
    // the tile's stores: every wavefront's complete, then one release
    // (agent scope) before the tile counts as complete
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (tid == 0) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      SlotState *st = s.st;
      const int c = __hip_atomic_fetch_add(&st->pq_done, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (c + 1 == ntiles) {   // the phase's last tile: decide the next phase and publish it
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        const PQPhase nx = pq_next(s, p);
        st->pq_phase = nx.ph;
        st->pq_it = nx.it;
        st->pq_lvl = nx.l;
        __hip_atomic_store(&st->pq_done, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const unsigned long long w = __hip_atomic_load(&st->pq_word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&st->pq_word, pq_pack(pq_gen(w) + 1u, pq_tiles(s, nx)), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
        if (nx.ph == PQ_FIN) __hip_atomic_fetch_add(&g->remaining, -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(&g->progress, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// host launchers (one slot: its record hs passed by value)
// ---------------------------------------------------------------------------

static unsigned lvl_grid(int nc) {
  int n = (nc + BLOCK - 1) / BLOCK;
  return (unsigned)(n < 1024 ? (n > 0 ? n : 1) : 1024);
}


template <typename R>
void launch_mg_setup(const Slot &hs, hipStream_t stream) {
  for (int l = 1; l <= hs.mg.L; ++l)
    hipLaunchKernelGGL((k_mg_setup<R, R>), dim3(lvl_grid(hs.mg.lv[l].nc)), dim3(BLOCK), 0, stream, hs, l);
  hipLaunchKernelGGL(k_mg_coarse_inv<R>, dim3(1), dim3(MG_INV_THREADS), 0, stream, hs);
}

template <typename R>
void launch_mg_dir(const Slot &hs, const Launch &L, int it, unsigned long long *ts) {
  hipLaunchKernelGGL((k_mgcg_dir<R, DIR_NB<R>>), dim3((unsigned)L.nblocks), dim3(BLOCK), 0, L.stream, hs, it, ts);
}

template <int DIM, typename R>
static void vcycle_levels(const Slot &hs, const Launch &L, unsigned long long *ts) {
  const int tl = hs.mg.tail;
  int m = 0;   // launch index within the part: its stamp region
  auto next = [&]() -> unsigned long long * { return ts ? ts + (size_t)TS_WORDS * m++ : nullptr; };
  // the split levels' first post-sweep goes to z of the fine grid, which
  // no launch reads between the fine pre-smoothing and fine up (fine up
  // writes it)
  R *tmp = (R *)hs.cw[0];
  for (int l = 1; l < tl; ++l) {
    const MGLevel &C = hs.mg.lv[l + 1];
    const dim3 g(lvl_grid((int)kid_total(DIM, C.nx, C.ny, C.nz)));
    if (mg_split(hs, l)) {
      hipLaunchKernelGGL((k_mg_split_smooth<DIM, R>), dim3(lvl_grid(hs.mg.lv[l].nc)), dim3(BLOCK), 0, L.stream, hs.st,
                         hs.mg.lv[l], C, next());
      hipLaunchKernelGGL((k_mg_split_restrict<DIM, R>), g, dim3(BLOCK), 0, L.stream, hs.st, hs.mg.lv[l], C, next());
    } else if ((hs.mg.nu2 >> l) & 1)
      hipLaunchKernelGGL((k_mg_smooth<DIM, R, 2>), g, dim3(BLOCK), 0, L.stream, hs.st, hs.mg.lv[l], C, next());
    else hipLaunchKernelGGL((k_mg_smooth<DIM, R, 1>), g, dim3(BLOCK), 0, L.stream, hs.st, hs.mg.lv[l], C, next());
  }
  hipLaunchKernelGGL((k_mg_tail<DIM, R>), dim3(1), dim3(MG_TAIL_THREADS), (size_t)hs.mg.tail_bytes, L.stream, hs,
                     next());
  for (int l = tl - 1; l >= 1; --l) {
    const dim3 g(lvl_grid(hs.mg.lv[l].nc));
    if (mg_split(hs, l)) {
      hipLaunchKernelGGL((k_mg_split_up1<DIM, R>), g, dim3(BLOCK), 0, L.stream, hs.st, hs.mg.lv[l], hs.mg.lv[l + 1], tmp,
                         next());
      hipLaunchKernelGGL((k_mg_split_up2<DIM, R>), g, dim3(BLOCK), 0, L.stream, hs.st, hs.mg.lv[l], hs.mg.lv[l + 1],
                         (const R *)tmp, next());
    } else if ((hs.mg.nu2 >> l) & 1)
      hipLaunchKernelGGL((k_mg_up<DIM, R, 2>), g, dim3(BLOCK), 0, L.stream, hs.st, hs.mg.lv[l], hs.mg.lv[l + 1],
                         next());
    else hipLaunchKernelGGL((k_mg_up<DIM, R, 1>), g, dim3(BLOCK), 0, L.stream, hs.st, hs.mg.lv[l], hs.mg.lv[l + 1],
                            next());
  }
}

// part of the cycle of iteration it (it = -1: the cycle of the initial residual)
template <typename R>
void launch_mg_cycle_part(const Slot &hs, const Launch &L, int it, int part, int mode, unsigned long long *ts) {
  const dim3 fg((unsigned)L.nblocks), fb(BLOCK);
  if (part == 0) {
    if (brick_ok(hs.dim, hs.nx, hs.ny, hs.nz))
      hipLaunchKernelGGL(k_mg_fine_down_brick<R>, fg, fb, 0, L.stream, hs, it, mode, ts);
    else hipLaunchKernelGGL((k_mg_fine_down<R, FINE_NB<R>>), fg, fb, 0, L.stream, hs, it, mode, ts);
  } else if (part == 1) {
    if (hs.dim == 3) vcycle_levels<3, R>(hs, L, ts);
    else vcycle_levels<2, R>(hs, L, ts);
  } else {
    hipLaunchKernelGGL((k_mg_fine_up<R, FINE_NB<R>>), fg, fb, 0, L.stream, hs, it, ts);
  }
}

// ---------------------------------------------------------------------------
// batched launchers (serving engine)
// ---------------------------------------------------------------------------

void mg_batch_levels(MGBatch::Dim &d, const Slot *const *hs, int n, int dim) {
  d.n = n;
  d.maxL = 0;
  d.maxtail = 0;
  d.tail_bytes = 0;
  for (int l = 0; l <= MG_MAXL; ++l) d.setup_b[l] = d.smooth_b[l] = d.up_b[l] = 0;
  for (int x = 0; x < n; ++x) {
    const MGInfo &mg = hs[x]->mg;
    d.maxL = mg.L > d.maxL ? mg.L : d.maxL;
    d.maxtail = mg.tail > d.maxtail ? mg.tail : d.maxtail;
    d.tail_bytes = mg.tail_bytes > d.tail_bytes ? mg.tail_bytes : d.tail_bytes;
    for (int l = 1; l <= mg.L; ++l) {
      const int b = lvl_blocks(mg.lv[l].nc);
      d.setup_b[l] = b > d.setup_b[l] ? b : d.setup_b[l];
    }
    for (int l = 1; l < mg.tail; ++l) {
      const int bs = smooth_blocks(mg, l, dim), bu = up_blocks(mg, l);
      d.smooth_b[l] = bs > d.smooth_b[l] ? bs : d.smooth_b[l];
      d.up_b[l] = bu > d.up_b[l] ? bu : d.up_b[l];
    }
  }
}

template <typename R>
void launch_mg_setup_b(const MGBatch &B) {
  for (int di = 0; di < 2; ++di) {
    const MGBatch::Dim &d = B.dim[di];
    if (!d.n) continue;
    for (int l = 1; l <= d.maxL; ++l)
      hipLaunchKernelGGL((k_mg_setup_b<R, R>), dim3((unsigned)(d.n * d.setup_b[l])), dim3(BLOCK), 0, B.stream, B.slots,
                         d.act, d.setup_b[l], l);
    hipLaunchKernelGGL(k_mg_coarse_inv_b<R>, dim3((unsigned)d.n), dim3(MG_INV_THREADS), 0, B.stream, B.slots, d.act);
  }
}

template <typename R>
void launch_mg_dir_b(const MGBatch &B, int it) {
  hipLaunchKernelGGL((k_mgcg_dir_b<R, FINE_NB<R>>), dim3((unsigned)B.nblocks), dim3(BLOCK), 0, B.stream, B.slots,
                     B.btab, it);
}

template <int DIM, typename R>
static void vcycle_levels_b(const MGBatch &B, const MGBatch::Dim &d) {
  for (int l = 1; l < d.maxtail; ++l)
    if (d.smooth_b[l])
      hipLaunchKernelGGL((k_mg_smooth_b<DIM, R>), dim3((unsigned)(d.n * d.smooth_b[l])), dim3(BLOCK), 0, B.stream,
                         B.slots, d.act, d.smooth_b[l], l);
  hipLaunchKernelGGL((k_mg_tail_b<DIM, R>), dim3((unsigned)d.n), dim3(MG_TAIL_THREADS), (size_t)d.tail_bytes, B.stream,
                     B.slots, d.act);
  for (int l = d.maxtail - 1; l >= 1; --l)
    if (d.up_b[l])
      hipLaunchKernelGGL((k_mg_up_b<DIM, R>), dim3((unsigned)(d.n * d.up_b[l])), dim3(BLOCK), 0, B.stream, B.slots,
                         d.act, d.up_b[l], l);
}

template <typename R>
void launch_mg_cycle_part_b(const MGBatch &B, int it, int part) {
  const dim3 fg((unsigned)B.nblocks), fb(BLOCK);
  if (part == 0) {
    hipLaunchKernelGGL((k_mg_fine_down_b<R, FINE_NB<R>>), fg, fb, 0, B.stream, B.slots, B.btab, it);
  } else if (part == 1) {
    if (B.dim[0].n) vcycle_levels_b<2, R>(B, B.dim[0]);
    if (B.dim[1].n) vcycle_levels_b<3, R>(B, B.dim[1]);
  } else {
    hipLaunchKernelGGL((k_mg_fine_up_b<R, FINE_NB<R>>), fg, fb, 0, B.stream, B.slots, B.btab, it);
  }
}

void launch_pq_list(int *dst, const int *host, int n, hipStream_t stream) {
  for (int off = 0; off < n; off += PQListChunk::MAXN) {
    PQListChunk c;
    c.off = off;
    c.n = n - off < PQListChunk::MAXN ? n - off : PQListChunk::MAXN;
    for (int i = 0; i < c.n; ++i) c.v[i] = host[off + i];
    hipLaunchKernelGGL(k_pq_list, dim3(1), dim3(BLOCK), 0, stream, dst, c);
  }
}

void launch_pq_init(const Slot *slots, const int *list, int n, PQGlobal *g, hipStream_t stream) {
  hipLaunchKernelGGL(k_pq_init, dim3(1), dim3(BLOCK), 0, stream, slots, list, n, g);
}

template <typename R>
void launch_pq_solve(const Slot *slots, const int *list, int n, PQGlobal *g, int wgs, int lds, long long idle_ticks,
                     hipStream_t stream) {
  hipLaunchKernelGGL(k_pq_solve<R>, dim3((unsigned)wgs), dim3(BLOCK), (size_t)lds, stream, slots, list, n, g, lds,
                     idle_ticks);
}

template <typename R> int pq_resident_wgs(int lds) {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_pq_solve<R>, BLOCK, (size_t)lds) != hipSuccess) return 0;
  return per * cus;
}

template void launch_pq_solve<double>(const Slot *, const int *, int, PQGlobal *, int, int, long long, hipStream_t);
template void launch_pq_solve<float>(const Slot *, const int *, int, PQGlobal *, int, int, long long, hipStream_t);
template int pq_resident_wgs<double>(int);
template int pq_resident_wgs<float>(int);

template void launch_mg_setup_b<double>(const MGBatch &);
template void launch_mg_setup_b<float>(const MGBatch &);
template void launch_mg_dir_b<double>(const MGBatch &, int);
template void launch_mg_dir_b<float>(const MGBatch &, int);
template void launch_mg_cycle_part_b<double>(const MGBatch &, int, int);
template void launch_mg_cycle_part_b<float>(const MGBatch &, int, int);

template void launch_mg_setup<double>(const Slot &, hipStream_t);
template void launch_mg_setup<float>(const Slot &, hipStream_t);
template void launch_mg_dir<double>(const Slot &, const Launch &, int, unsigned long long *);
template void launch_mg_dir<float>(const Slot &, const Launch &, int, unsigned long long *);
template void launch_mg_cycle_part<double>(const Slot &, const Launch &, int, int, int, unsigned long long *);
template void launch_mg_cycle_part<float>(const Slot &, const Launch &, int, int, int, unsigned long long *);

}  // namespace oscar
