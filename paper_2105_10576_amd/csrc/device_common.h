// Device helpers shared by the OSCAR kernels: indexing and boundary
// classification of a slot's voxel grid, deterministic block/slot
// reductions, mixture properties, and the matrix-free pressure operator.
#pragma once
#include "oscar_internal.h"

namespace oscar {

struct Cell {
  int P;
  int i, j, k, row;   // row = j + ny*k
  bool valid;
};

// A kernel's register copy of a slot's grid constants, read once at kernel
// start: stores through the field pointers may alias the slot record, so
// reading the record inside a loop would force a memory round trip per use.
struct Grid {
  int dim, nx, ny, nz, nxy, nc, nblocks;
  uint32_t outlet;   // bit f: box side f is an outlet
  double Sh, S2h;
};

__device__ __forceinline__ Grid grid_of(const Slot &s) {
  Grid g;
  g.dim = s.dim;
  g.nx = s.nx;
  g.ny = s.ny;
  g.nz = s.nz;
  g.nxy = s.nxy;
  g.nc = s.nc;
  g.nblocks = s.nblocks;
  g.outlet = s.outlet;
  g.Sh = s.Sh;
  g.S2h = s.S2h;
  return g;
}

struct Block {
  const Slot *s;
  const SlotCtl *ctl;
  SlotState *st;
  int lb;
};

// cell coordinates from the linear index (32-bit unsigned arithmetic)
__device__ __forceinline__ Cell cell_at(const Slot &s, int g) {
  Cell c;
  c.valid = true;
  c.P = g;
  unsigned ug = (unsigned)g, nx = (unsigned)s.nx, ny = (unsigned)s.ny;
  unsigned row = ug / nx;
  c.i = (int)(ug - row * nx);
  c.row = (int)row;
  unsigned k = row / ny;
  c.j = (int)(row - k * ny);
  c.k = (int)k;
  return c;
}

// grid-stride loop over the cells of the slot handled by block lb
template <class Fn>
__device__ __forceinline__ void for_cells(const Slot &s, int lb, Fn &&fn) {
  const int stride = s.nblocks * BLOCK, nc = s.nc;
  for (int g = lb * BLOCK + (int)threadIdx.x; g < nc; g += stride) fn(cell_at(s, g));
}

__device__ __forceinline__ Cell cell_at(const Grid &G, int g) {
  Cell c;
  c.valid = true;
  c.P = g;
  unsigned ug = (unsigned)g, nx = (unsigned)G.nx, ny = (unsigned)G.ny;
  unsigned row = ug / nx;
  c.i = (int)(ug - row * nx);
  c.row = (int)row;
  unsigned k = row / ny;
  c.j = (int)(row - k * ny);
  c.k = (int)k;
  return c;
}

template <class Fn>
__device__ __forceinline__ void for_cells(const Grid &G, int lb, Fn &&fn) {
  const int stride = G.nblocks * BLOCK;
  for (int g = lb * BLOCK + (int)threadIdx.x; g < G.nc; g += stride) fn(cell_at(G, g));
}

// Walk of a grid-wide launch over an index space of `planes` planes, each of
// `rows` rows of `rowlen` indices (cells, or the wave tiles of the
// restriction order).  The launch's blocks are grouped as the XCD deal
// groups them (group x: the contiguous run of blocks that runs on XCD x),
// and group x walks its own contiguous slab of planes in row blocks of about
// WALK_BLOCK indices: the first row block through every plane of the slab,
// then the next, grid-stride over the group's threads.  The planes a stencil
// reads above and below its own were then read by the same XCD a moment
// before and are still in its 4 MB L2.  Used in 3D with at least 8 blocks,
// 8 planes and WALK_MIN elements (below that the arrays of a launch fit the
// 256 MB last-level cache and the index arithmetic costs more than the
// walk saves); otherwise the plain grid-stride walk over the whole space.
// The walk is a function of the block's index within the slot and the
// slot's block count alone, so a batched launch (block table) walks exactly
// as a single-slot launch.
constexpr int WALK_BLOCK = 16384;
constexpr int WALK_MIN = 1 << 22;

struct Walk {
  int first, stride, end;   // local index range [first, end) in steps of stride
  bool slabbed;
  int base;                 // plain walk: index of the first element
  int z0, nzs, per_plane;   // slab: first plane, planes, indices per plane
  int pb, pbl, tfull;       // indices per row block (the last one: pbl) and before the last row block
  int nrb;                  // row blocks per plane
};

__device__ __forceinline__ Walk slab_walk(int lb, int nblocks, int planes, int rows, int rowlen, bool slabs,
                                          int min_elems = WALK_MIN) {
  Walk w;
  w.slabbed = slabs && nblocks >= 8 && planes >= 8 && planes * rows * rowlen >= min_elems;
  if (!w.slabbed) {
    w.first = lb * BLOCK + (int)threadIdx.x;
    w.stride = nblocks * BLOCK;
    w.end = planes * rows * rowlen;
    w.base = 0;
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
  w.z0 = (int)(((long long)x * planes) / X);
  const int z1 = (int)(((long long)(x + 1) * planes) / X);
  w.nzs = z1 - w.z0;
  w.per_plane = rows * rowlen;
  int yb = WALK_BLOCK / rowlen;
  yb = yb < 1 ? 1 : (yb > rows ? rows : yb);
  w.nrb = (rows + yb - 1) / yb;
  w.pb = yb * rowlen;
  w.pbl = (rows - (w.nrb - 1) * yb) * rowlen;
  w.tfull = (w.nrb - 1) * w.nzs * w.pb;
  w.first = (lb - l0) * BLOCK + (int)threadIdx.x;
  w.stride = cnt * BLOCK;
  w.end = w.tfull + w.nzs * w.pbl;
  w.base = 0;
  return w;
}

// the element at local index t (t < end) of a walk
__device__ __forceinline__ int walk_at(const Walk &w, int t) {
  if (!w.slabbed) return w.base + t;
  unsigned rb, z, c;
  if (t < w.tfull) {
    const unsigned qq = (unsigned)t / (unsigned)w.pb;
    c = (unsigned)t - qq * (unsigned)w.pb;
    rb = qq / (unsigned)w.nzs;
    z = qq - rb * (unsigned)w.nzs;
  } else {
    const unsigned r = (unsigned)(t - w.tfull);
    z = r / (unsigned)w.pbl;
    c = r - z * (unsigned)w.pbl;
    rb = (unsigned)w.nrb - 1u;
  }
  return (int)(((unsigned)w.z0 + z) * (unsigned)w.per_plane + rb * (unsigned)w.pb + c);
}

__device__ __forceinline__ Walk cell_walk(const Grid &G, int lb) {
  return slab_walk(lb, G.nblocks, G.nz, G.ny, G.nx, G.dim == 3);
}

__device__ __forceinline__ int cidx(const Slot &s, int i, int j, int k) { return i + s.nx * (j + s.ny * k); }

__device__ __forceinline__ int fidx(const Slot &s, int e, int i, int j, int k) {
  if (e == 0) return i + (s.nx + 1) * (j + s.ny * k);
  if (e == 1) return s.nf0 + i + s.nx * (j + (s.ny + 1) * k);
  return s.nf0 + s.nf1 + i + s.nx * (j + s.ny * k);
}

__device__ __forceinline__ bool solid_at(const Slot &s, int P) { return (s.flags[P] & 0x40) != 0; }

// offset between a cell and its neighbour across face f
__device__ __forceinline__ int nb_step(const Slot &s, int f) {
  int e = f >> 1;
  int st = e == 0 ? 1 : (e == 1 ? s.nx : s.nxy);
  return (f & 1) ? st : -st;
}

// face f of the cell lies on the box side (no neighbour inside the box)
__device__ __forceinline__ bool on_edge(const Slot &s, const Cell &c, int f) {
  int e = f >> 1;
  if (e == 0) return (f & 1) ? c.i == s.nx - 1 : c.i == 0;
  if (e == 1) return (f & 1) ? c.j == s.ny - 1 : c.j == 0;
  return (f & 1) ? c.k == s.nz - 1 : c.k == 0;
}

// face f (0..5 = x-,x+,y-,y+,z-,z+) of a fluid cell
struct CFace {
  int type;
  int nb, fi;
};

__device__ __forceinline__ CFace cell_face(const Slot &s, uint8_t fl, const Cell &c, int f) {
  CFace r;
  int e = f >> 1, hi = f & 1;
  r.nb = -1;
  r.fi = -1;
  if (e >= s.dim) { r.type = F_NONE; return r; }
  if (e == 0) r.fi = c.P + c.row + hi;
  else if (e == 1) r.fi = s.nf0 + c.P + s.nx * c.k + (hi ? s.nx : 0);
  else r.fi = s.nf0 + s.nf1 + c.P + (hi ? s.nxy : 0);
  if (fl & (1u << f)) { r.type = F_INT; r.nb = c.P + nb_step(s, f); return r; }
  r.type = on_edge(s, c, f) ? s.bcf[f] : F_WALL;
  return r;
}

// face of direction e whose high-side cell is (i,j,k) (coordinate along e in [0, n_e])
struct FView {
  int type;
  int lo, hi, P;
  double sf;   // orientation sign seen from the fluid cell (WALL / INLET / OUTLET)
};

__device__ __forceinline__ FView face_view(const Slot &s, int e, int i, int j, int k) {
  FView v;
  int li = i - (e == 0), lj = j - (e == 1), lk = k - (e == 2);
  bool loin = (e == 0 ? li >= 0 : (e == 1 ? lj >= 0 : lk >= 0));
  bool hiin = (e == 0 ? i < s.nx : (e == 1 ? j < s.ny : k < s.nz));
  v.lo = loin ? cidx(s, li, lj, lk) : -1;
  v.hi = hiin ? cidx(s, i, j, k) : -1;
  bool lof = loin && !solid_at(s, v.lo);
  bool hif = hiin && !solid_at(s, v.hi);
  v.type = F_NONE;
  v.P = -1;
  v.sf = 0.0;
  if (lof && hif) { v.type = F_INT; return v; }
  if (!lof && !hif) return v;
  if (lof) { v.P = v.lo; v.sf = 1.0; } else { v.P = v.hi; v.sf = -1.0; }
  if (loin && hiin) { v.type = F_WALL; return v; }
  v.type = s.bcf[2 * e + (lof ? 1 : 0)];
  return v;
}

// visit the faces owned by the thread of cell c: (e, fi, view)
template <class Fn>
__device__ __forceinline__ void for_owned_faces(const Slot &s, const Cell &c, Fn &&fn) {
  for (int e = 0; e < s.dim; ++e) {
    fn(e, fidx(s, e, c.i, c.j, c.k), face_view(s, e, c.i, c.j, c.k));
    bool last = e == 0 ? c.i == s.nx - 1 : (e == 1 ? c.j == s.ny - 1 : c.k == s.nz - 1);
    if (last) {
      int i = c.i + (e == 0), j = c.j + (e == 1), k = c.k + (e == 2);
      fn(e, fidx(s, e, i, j, k), face_view(s, e, i, j, k));
    }
  }
}

// Measurement only: with a non-null ts, workgroup b of the launch writes its
// start and end on the device's constant-rate wall clock to ts[2b], ts[2b+1]
// (plain stores: no contention between workgroups).
// Kernel entry.  A kernel's record arrives by value in its argument
// segment, and the compiler reads each field in the basic block that first
// uses it, waiting before each branch: the entry code of a kernel (timing
// stamp, block mapping, converged-solve test) chained several round trips
// to the segment before the first data load.  OSCAR_PRIME("s"(field), ...)
// asks for the fields together at entry (one batch of scalar loads, one
// wait); later reads of the same fields reuse the registers.
#define OSCAR_PRIME(...) asm volatile("" ::__VA_ARGS__)

// v exists at this point: the loads it was computed from cannot sink past a
// branch that follows (a converged-solve test taken after the first data
// loads, before the first store, so that its own load overlaps them)
template <typename T>
__device__ __forceinline__ void keep_live(const T &v) {
  asm volatile("" ::"v"(v));
}
// v as read at this point and no earlier (a uniform test of a loaded value
// would otherwise wait for it where the compiler moves it to scalar
// registers, ahead of the loads that follow)
__device__ __forceinline__ int read_late(int v) {
  asm volatile("" : "+v"(v));
  return v;
}

struct Stamp {
  unsigned long long *ts;
  unsigned long long t0;
  __device__ __forceinline__ explicit Stamp(unsigned long long *p) : ts(p), t0(p ? wall_clock64() : 0ull) {}
  __device__ __forceinline__ void done() {
    if (!ts) return;
    __syncthreads();
    if (threadIdx.x == 0) {
      ts[2 * blockIdx.x] = t0;
      ts[2 * blockIdx.x + 1] = (unsigned long long)wall_clock64();
    }
  }
};

// ---------------------------------------------------------------------------
// deterministic per-slot reductions
// ---------------------------------------------------------------------------

// Lane exchanges within a wavefront whose lanes are all active, as VALU
// operations rather than round trips through the LDS crossbar
// (ds_bpermute): a DPP quad permutation (lane l ^ 1), DPP row shifts (lane
// l + n of l's 16-lane row, 0 past the row's end) and the gfx950 swaps of
// odd with even rows (lane l ^ 16) and of the two halves (lane l ^ 32).
__device__ __forceinline__ unsigned lane_x1(unsigned u) {
  return (unsigned)__builtin_amdgcn_mov_dpp((int)u, 0xB1, 0xF, 0xF, true);   // quad_perm [1, 0, 3, 2]
}
__device__ __forceinline__ unsigned lane_x16(unsigned u) {
  const auto s = __builtin_amdgcn_permlane16_swap(u, u, false, false);
  return (__lane_id() & 16u) ? s[0] : s[1];
}
__device__ __forceinline__ unsigned lane_x32(unsigned u) {
  const auto s = __builtin_amdgcn_permlane32_swap(u, u, false, false);
  return (__lane_id() & 32u) ? s[0] : s[1];
}
template <int N>
__device__ __forceinline__ unsigned lane_shl(unsigned u) {
  return (unsigned)__builtin_amdgcn_update_dpp(0, (int)u, 0x100 + N, 0xF, 0xF, true);   // row_shl:N
}
// one of the exchanges above applied to a float or a double (by halves)
template <class F>
__device__ __forceinline__ float lane_move(float v, F &&f) {
  return __uint_as_float(f(__float_as_uint(v)));
}
template <class F>
__device__ __forceinline__ double lane_move(double v, F &&f) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = f((unsigned)b), hi = f((unsigned)(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
// the value of lane l + off for the lanes l < off that a reduction tree
// uses next (off = 32, 16: the partner l ^ off; 8, 4, 2, 1: the row shift)
template <int OFF, typename T>
__device__ __forceinline__ T lane_down(T v) {
  if constexpr (OFF == 32) return lane_move(v, lane_x32);
  else if constexpr (OFF == 16) return lane_move(v, lane_x16);
  else return lane_move(v, lane_shl<OFF>);
}

// Wavefront reduction: lane 0 receives the total of the tree that adds lanes
// l and l + off for off = 32, 16, ..., 1 (max for the MAXMASK values).
template <unsigned MAXMASK, int M>
__device__ __forceinline__ void wave_reduce(double (&v)[M]) {
#pragma unroll
  for (int m = 0; m < M; ++m) {
    auto step = [&](double o) {
      if ((MAXMASK >> m) & 1u) v[m] = o > v[m] ? o : v[m];
      else v[m] = v[m] + o;
    };
    step(lane_down<32>(v[m]));
    step(lane_down<16>(v[m]));
    step(lane_down<8>(v[m]));
    step(lane_down<4>(v[m]));
    step(lane_down<2>(v[m]));
    step(lane_down<1>(v[m]));
  }
}

// Block-level reduction of v (fixed order); every thread receives the totals.
template <unsigned MAXMASK, int M>
__device__ __forceinline__ void block_reduce(double (&v)[M]) {
  __shared__ double sh[M][BLOCK / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  wave_reduce<MAXMASK>(v);
  __syncthreads();
  if (lane == 0)
#pragma unroll
    for (int m = 0; m < M; ++m) sh[m][w] = v[m];
  __syncthreads();
#pragma unroll
  for (int m = 0; m < M; ++m) {
    double t = sh[m][0];
    for (int x = 1; x < BLOCK / 64; ++x) t = ((MAXMASK >> m) & 1u) ? (sh[m][x] > t ? sh[m][x] : t) : t + sh[m][x];
    v[m] = t;
  }
}

// publish this block's partials of channel ch
template <unsigned MAXMASK, int M>
__device__ __forceinline__ void put_partials(const Slot &s, int lb, int ch, double (&v)[M]) {
  block_reduce<MAXMASK>(v);
  if (threadIdx.x == 0)
#pragma unroll
    for (int m = 0; m < M; ++m) s.part[(int)(ch * NVAL + m) * s.nblocks + lb] = v[m];
}

// totals of channel ch over the slot's blocks, in every thread (fixed
// order: each thread sums blocks tid, tid + BLOCK, ... in turn; the loads of
// four strides are issued together)
template <unsigned MAXMASK, int M>
__device__ __forceinline__ void get_totals(const Slot &s, int ch, double (&v)[M]) {
  const int nb = s.nblocks;
  const double *base = s.part + (int)(ch * NVAL) * nb;
  double t[M];
#pragma unroll
  for (int m = 0; m < M; ++m) t[m] = 0.0;
  int b = threadIdx.x;
  for (; b + 3 * BLOCK < nb; b += 4 * BLOCK) {
    double x[M][4];
#pragma unroll
    for (int m = 0; m < M; ++m)
#pragma unroll
      for (int u = 0; u < 4; ++u) x[m][u] = base[m * nb + b + u * BLOCK];
#pragma unroll
    for (int m = 0; m < M; ++m)
#pragma unroll
      for (int u = 0; u < 4; ++u) t[m] = ((MAXMASK >> m) & 1u) ? (x[m][u] > t[m] ? x[m][u] : t[m]) : t[m] + x[m][u];
  }
  for (; b < nb; b += BLOCK)
#pragma unroll
    for (int m = 0; m < M; ++m) {
      double x = base[m * nb + b];
      t[m] = ((MAXMASK >> m) & 1u) ? (x > t[m] ? x : t[m]) : t[m] + x;
    }
#pragma unroll
  for (int m = 0; m < M; ++m) v[m] = t[m];
  block_reduce<MAXMASK>(v);
}

// The same totals in two steps, so that their loads can be issued ahead of
// other work: prefetch_totals loads a thread's partials (a slot has at most
// 4 x BLOCK blocks), finish_totals sums them in the order get_totals uses
// and reduces over the block.  A thread's missing partials read as zero
// (adding +0 leaves its sum unchanged).
template <int M>
struct Partials {
  double x[M][4];
};
template <int M>
__device__ __forceinline__ void prefetch_totals(const Slot &s, int ch, Partials<M> &p) {
  const int nb = s.nblocks;
  const double *base = s.part + (int)(ch * NVAL) * nb;
#pragma unroll
  for (int m = 0; m < M; ++m)
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int b = (int)threadIdx.x + u * BLOCK;
      const double v = base[m * nb + (b < nb ? b : 0)];
      p.x[m][u] = b < nb ? v : 0.0;
    }
}
template <int M>
__device__ __forceinline__ void finish_totals(const Partials<M> &p, double (&v)[M]) {
#pragma unroll
  for (int m = 0; m < M; ++m) {
    double t = 0.0;
#pragma unroll
    for (int u = 0; u < 4; ++u) t = t + p.x[m][u];
    v[m] = t;
  }
  block_reduce<0u>(v);
}

// ---------------------------------------------------------------------------
// mixture properties
// ---------------------------------------------------------------------------

template <typename R>
__device__ __forceinline__ R rho_of(const Slot &s, R a) {
  return a * (R)s.rho1 + ((R)1 - a) * (R)s.rho2;
}
template <typename R>
__device__ __forceinline__ R mu_of(const Slot &s, R a) {
  return a * (R)s.mu1 + ((R)1 - a) * (R)s.mu2;
}

template <typename R>
__device__ __forceinline__ R vnorm(const R *v, int d) {
  R t = v[0] * v[0] + v[1] * v[1];
  if (d == 3) t = t + v[2] * v[2];
  return sqrt(t);
}

// surface-tension face term sigma*kappa_f*(alpha_hi - alpha_lo)/h, in FP64
// (it is balanced against the pressure gradient on the same face)
template <typename R>
__device__ __forceinline__ double st_face(const Slot &s, const R *kap, const R *a, int lo, int hi) {
  return (s.sigma * (0.5 * ((double)kap[lo] + (double)kap[hi]))) * (((double)a[hi] - (double)a[lo]) / s.h);
}

// pressure coefficient of face f of fluid cell P in precision X
template <typename X, typename R>
__device__ __forceinline__ X pcoef(const Slot &s, const R *rAU, int P, const CFace &cf) {
  if (cf.type == F_INT) return ((X)0.5 * ((X)rAU[P] + (X)rAU[cf.nb])) * (X)s.Sh;
  if (cf.type == F_OUTLET) return (X)rAU[P] * (X)s.S2h;
  return (X)0;
}

// face f of cell c lies on the box side
__device__ __forceinline__ bool on_edge(const Grid &G, const Cell &c, int f) {
  int e = f >> 1;
  if (e == 0) return (f & 1) ? c.i == G.nx - 1 : c.i == 0;
  if (e == 1) return (f & 1) ? c.j == G.ny - 1 : c.j == 0;
  return (f & 1) ? c.k == G.nz - 1 : c.k == 0;
}

// (M x)_P in precision X from preloaded operands: x and rAU at the cell
// (xP, rP) and across each face f (xn[f], rn[f]; any value where face f is
// not interior: it is not used).  The sum is taken face by face in the order
// x-, x+, y-, y+, z-, z+, adding only interior and outlet terms, which is
// the operation order of the sequential reference.
template <typename X>
__device__ __forceinline__ X matvec_pre(const Grid &G, const Cell &c, uint8_t fl, X xP, X rP, const X (&xn)[6],
                                        const X (&rn)[6]) {
  X acc = (X)0;
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    if ((fl >> f) & 1u) acc = acc + (((X)0.5 * (rP + rn[f])) * (X)G.Sh) * (xP - xn[f]);
    else if (((G.outlet >> f) & 1u) && on_edge(G, c, f)) acc = acc + (rP * (X)G.S2h) * xP;
  }
  return acc;
}

// neighbour of cell P across face f where the face is interior (flag bit
// f), else P itself: every index is a valid load address
__device__ __forceinline__ int nb_at(const Grid &G, int P, uint8_t fl, int f) {
  const int st = (f >> 1) == 0 ? 1 : ((f >> 1) == 1 ? G.nx : G.nxy);
  return ((fl >> f) & 1u) ? ((f & 1) ? P + st : P - st) : P;
}

// (M x)_P in precision X, with x read through xf(index, f): f = -1 for the
// cell itself, else the face across which the (interior) neighbour lies.
// All six faces are unrolled and every neighbour value is read
// unconditionally, at the cell itself where the face is not interior (faces
// 4 and 5 in 2D), so the loads issue together.
template <typename X, typename R, class XF>
__device__ __forceinline__ X matvec_row_f(const Grid &G, const R *rAU, const Cell &c, uint8_t fl, XF &&xf) {
  const int P = c.P;
  const X xP = xf(P, -1);
  const X rP = (X)rAU[P];
  X xn[6], rn[6];
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    const int n = nb_at(G, P, fl, f);
    xn[f] = xf(n, ((fl >> f) & 1u) ? f : -1);
    rn[f] = (X)rAU[n];
  }
  return matvec_pre<X>(G, c, fl, xP, rP, xn, rn);
}

// Element at a 32-bit byte offset from a base pointer: with the base in
// scalar registers the load takes the offset as its only per-lane address
// operand, and one offset serves every array of the same element size.
// (The accesses name the global address space: a pointer read from the
// slot table in memory is otherwise a generic one, accessed with flat
// instructions.)
#define OSCAR_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ T ldo(const T *base, unsigned off) {
  return *(const OSCAR_GLOBAL T *)((const char *)base + off);
}
template <typename T>
__device__ __forceinline__ void sto(T *base, unsigned off, T v) {
  *(OSCAR_GLOBAL T *)((char *)base + off) = v;
}

// element idx of a field known to live in device global memory
template <typename T>
__device__ __forceinline__ T gld(const T *base, int idx) {
  return ((const OSCAR_GLOBAL T *)base)[idx];
}
template <typename T>
__device__ __forceinline__ void gst(T *base, int idx, T v) {
  ((OSCAR_GLOBAL T *)base)[idx] = v;
}

// Per-cell operand indices of the six faces of a cell, every one valid: the
// neighbour across face f where that face is interior and the cell itself
// otherwise, and the face index (0 beyond dim), so the operands of all faces
// can be loaded ahead of the arithmetic without a branch.
struct Hood {
  int nb[6], fi[6];
};
__device__ __forceinline__ Hood hood_of(const Slot &s, uint8_t fl, const Cell &c) {
  Hood h;
  const int st[3] = {1, s.nx, s.nxy};
  const int fb[3] = {c.P + c.row, s.nf0 + c.P + s.nx * c.k, s.nf0 + s.nf1 + c.P};
  const int fs[3] = {1, s.nx, s.nxy};
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    const int e = f >> 1;
    h.nb[f] = ((fl >> f) & 1u) ? ((f & 1) ? c.P + st[e] : c.P - st[e]) : c.P;
    h.fi[f] = e < s.dim ? fb[e] + ((f & 1) ? fs[e] : 0) : 0;
  }
  return h;
}

// The low face of direction e of a cell as the face_view classification
// sees it, from the cell's flags fl and those of the cell below it, flo
// (ignored when edge: the face lies on the box side).  side: the fluid cell
// of a boundary face, 1 = the cell itself (orientation sign -1 seen from
// it), 0 = the cell below (sign +1).
__device__ __forceinline__ int low_face_type(const Slot &s, uint8_t fl, uint8_t flo, bool edge, int e, int &side) {
  const bool hif = !(fl & 0x40);
  side = 1;
  if (edge) return hif ? s.bcf[2 * e] : F_NONE;
  const bool lof = !(flo & 0x40);
  if (lof && hif) return F_INT;
  if (!lof && !hif) return F_NONE;
  side = hif ? 1 : 0;
  return F_WALL;
}

// byte offsets of cell P (element size w) and of its neighbours across
// faces 0..5 where the face is interior (flag bit f), else of P itself
__device__ __forceinline__ void nb_offsets(const Grid &G, unsigned P, uint8_t fl, unsigned w, unsigned &oP,
                                           unsigned (&on)[6]) {
  oP = P * w;
  const unsigned sx = w, sy = (unsigned)G.nx * w, sz = (unsigned)G.nxy * w;
  const unsigned st[3] = {sx, sy, sz};
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    const unsigned n = (f & 1) ? oP + st[f >> 1] : oP - st[f >> 1];
    on[f] = ((fl >> f) & 1u) ? n : oP;
  }
}

// Grid-stride loop over index range [first, end) in steps of `stride`, NB
// indices per thread at a time: per batch, flag(o, g) for each index (it
// reads what decides which operands a cell needs; g may lie past the end),
// then data(o) for each (the operand loads, all in flight together), then,
// on the first batch only, pre() (every thread of the block reaches it, so
// it may hold a block reduction; its loads overlap the batch's; false ends
// the loop), then use(o) in index order.
template <int NB, class O, class F, class D, class Pre, class U>
__device__ __forceinline__ void batched(int first, int stride, int end, F &&flag, D &&data, Pre &&pre, U &&use) {
  O o[NB];
  int g = first;
  bool once = true;
  do {
#pragma unroll
    for (int m = 0; m < NB; ++m) flag(o[m], g + m * stride);
#pragma unroll
    for (int m = 0; m < NB; ++m) data(o[m]);
    if (once) {
      if (!pre()) return;
      once = false;
    }
#pragma unroll
    for (int m = 0; m < NB; ++m) use(o[m]);
    g += NB * stride;
  } while (g < end);
}

template <typename X, typename R, class XV>
__device__ __forceinline__ X matvec_row(const Grid &G, const R *rAU, const Cell &c, uint8_t fl, XV &&xv) {
  return matvec_row_f<X, R>(G, rAU, c, fl, [&](int n, int) { return xv(n); });
}

}  // namespace oscar
