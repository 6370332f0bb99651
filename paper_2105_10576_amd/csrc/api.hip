// Host side of the OSCAR library: descriptor validation, workspace layout,
// the stream-ordered orchestration of the viscous step and of the capillary
// relaxation (arXiv 2105.10576, Section 3), and the C ABI of include/oscar.h.
//
// Control flow stays on the device where it decides the arithmetic: the
// conjugate-gradient convergence test and the iteration count live in the
// per-slot device state, and every CG kernel returns at once when its slot
// is converged, so the host enqueues CG iterations in chunks and reads one
// small status block per chunk instead of one scalar per iteration.
#include "oscar_internal.h"
#include "../../include/oscar.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

using namespace oscar;

namespace {

thread_local std::string g_err = "no error";

constexpr uint64_t ALIGN = 256;

uint64_t up(uint64_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

struct Dims {
  int d;
  int64_t nc, nf0, nf1, nf2, nft;
  int nblocks;
};

Dims dims_of(const oscar_desc &D) {
  Dims g;
  g.d = D.dim;
  g.nc = (int64_t)D.nx * D.ny * D.nz;
  g.nf0 = (int64_t)(D.nx + 1) * D.ny * D.nz;
  g.nf1 = (int64_t)D.nx * (D.ny + 1) * D.nz;
  g.nf2 = D.dim == 3 ? (int64_t)D.nx * D.ny * (D.nz + 1) : 0;
  g.nft = g.nf0 + g.nf1 + g.nf2;
  g.nblocks = blocks_for(g.nc, D.max_blocks);
  return g;
}

// Carve a workspace: every array on its own 256-byte boundary.
struct Carver {
  uint64_t off = 0;
  char *base = nullptr;
  void *take(uint64_t bytes) {
    void *p = base ? base + off : nullptr;
    off += up(bytes ? bytes : 1);
    return p;
  }
};

// The multigrid hierarchy (a preconditioner: the CG solves the current
// operator whatever it was built from) is rebuilt from the current 1/a_P at
// every viscous step and every MG_REBUILD-th capillary sub-step of a
// relaxation, starting with the first; the sub-steps between reuse it.
// Measured on the 128 x 64 x 64 channel (12 sub-steps): 724 CG iterations
// per step whether it is rebuilt every sub-step or once per relaxation.
constexpr int MG_REBUILD = 4;
inline bool mg_rebuild(bool capillary, int substep) { return !capillary || substep % MG_REBUILD == 0; }

// Multigrid hierarchy: halve every dimension (rounding up) until a level
// has at most MG_COARSEST cells (at most MG_MAXL levels); the tail (run by
// one workgroup out of LDS) starts at the first level of at most
// MG_TAIL_CELLS cells whose block fits MG_TAIL_LDS bytes.
void mg_levels(const oscar_desc &D, MGInfo &mg) {
  int nx = D.nx, ny = D.ny, nz = D.nz;
  mg.L = 0;
  do {
    nx = (nx + 1) / 2;
    ny = (ny + 1) / 2;
    nz = D.dim == 3 ? (nz + 1) / 2 : 1;
    MGLevel &v = mg.lv[++mg.L];
    v.nx = nx;
    v.ny = ny;
    v.nz = nz;
    v.nxy = nx * ny;
    v.nc = nx * ny * nz;
    v.nblocks = 0;
  } while (mg.lv[mg.L].nc > MG_COARSEST && mg.L < MG_MAXL);
  const int w = D.precision == OSCAR_MIXED ? 4 : 8;
  mg.tail = mg.L;
  for (int l = 1; l < mg.L; ++l)
    if (mg.lv[l].nc <= MG_TAIL_CELLS && mg_tail_bytes(mg, l, D.dim, w) <= MG_TAIL_LDS) {
      mg.tail = l;
      break;
    }
  mg.tail_bytes = (int32_t)mg_tail_bytes(mg, mg.tail, D.dim, w);
  // Smoothing sweeps of the grid-wide coarse levels: two in 3D, one in 2D.
  // A second sweep cuts the CG iterations but makes these latency-bound
  // kernels slower; in 3D it pays on every level, in 2D on none.  The
  // descriptor's mg_sweeps2 mask replaces the rule.
  mg.nu2 = 0;
  if (D.dim == 3)
    for (int l = 1; l < mg.tail; ++l) mg.nu2 |= 1 << l;
  if (D.mg_sweeps2 > 0) mg.nu2 = D.mg_sweeps2;
  else if (D.mg_sweeps2 < 0) mg.nu2 = 0;
  mg.nu2 &= ((1 << mg.tail) - 1) & ~1;
}

// Lay out one slot's arrays (and, with `ctl_block`, its table entries).
void layout(const oscar_desc &D, Carver &cv, Slot *s, bool ctl_block) {
  Dims g = dims_of(D);
  uint64_t w = D.precision == OSCAR_MIXED ? 4 : 8;
  const int64_t nc = g.nc, d = g.d, nf = g.nft;
  s->flags = (const uint8_t *)cv.take(nc);
  void **cell1[] = {&s->alpha, &s->alpha_old, &s->kappa, &s->aP, &s->rAU, &s->Rp, &s->Rm, &s->invD,
                    &s->cr[0], &s->cr[1], &s->cw[0], &s->cw[1], &s->cs[0], &s->cs[1], &s->cp, &s->e};
  for (void **p : cell1) *p = cv.take(w * nc);
  void **celld[] = {&s->U_vd, &s->U_cr, &s->U_sum, &s->U, &s->grad, &s->HbyA, &s->b};
  for (void **p : celld) *p = cv.take(w * nc * d);
  s->gradU = cv.take(w * nc * d * d);
  void **face[] = {&s->phi_vd, &s->phi_prev, &s->phi_cr, &s->nhatf, &s->Fm, &s->FL, &s->Af};
  for (void **p : face) *p = cv.take(w * nf);
  s->Af2 = D.mules_iter > 1 ? cv.take(w * nf) : nullptr;
  s->phiH = (double *)cv.take(8 * nf);
  double **dbl[] = {&s->p_vd, &s->p_cr, &s->p, &s->rhs, &s->Mp};
  for (double **p : dbl) *p = (double *)cv.take(8 * nc);
  s->r64 = nullptr;
  memset(&s->mg, 0, sizeof s->mg);
  if (D.precond == OSCAR_PC_MG) {
    mg_levels(D, s->mg);
    MGInfo &mg = s->mg;
    for (int l = 1; l < mg.tail; ++l) {
      MGLevel &v = mg.lv[l];
      for (int e = 0; e < d; ++e) v.cf[e] = cv.take(w * v.nc);
      void **arr[] = {&v.cout, &v.invD, &v.b, &v.x, &v.t};
      for (void **p : arr) *p = cv.take(w * v.nc);
    }
    // the tail block, packed, with the arrays the tail reads before writing
    // first (the part copied into LDS, tail_load bytes), then the rest
    char *tb = (char *)cv.take((uint64_t)mg.tail_bytes);
    uint64_t at = 0;
    auto part = [&](uint64_t n) -> void * {
      void *p = tb ? tb + at : nullptr;
      at += w * n;
      return p;
    };
    mg.tail_base = tb;
    const uint64_t ncl = (uint64_t)mg.lv[mg.L].nc;
    mg.Ainv = part(ncl * ncl);
    for (int l = mg.tail; l <= mg.L; ++l) {
      MGLevel &v = mg.lv[l];
      for (int e = 0; e < d; ++e) v.cf[e] = part(v.nc);
      v.cout = part(v.nc);
      v.invD = part(v.nc);
    }
    mg.lv[mg.tail].b = part(mg.lv[mg.tail].nc);
    mg.tail_load = (int32_t)((at + 15) / 16 * 16);
    for (int l = mg.tail; l <= mg.L; ++l) {
      MGLevel &v = mg.lv[l];
      if (l > mg.tail) v.b = part(v.nc);
      v.x = part(v.nc);
      v.t = part(v.nc);
    }
  }
  s->part = (double *)cv.take(8ull * NCH * NVAL * g.nblocks);
  s->st = (SlotState *)cv.take(sizeof(SlotState));
  s->ctl = (SlotCtl *)cv.take(sizeof(SlotCtl));
  (void)ctl_block;
}

int check_desc(const oscar_desc *D, std::string &why) {
  if (!D) { why = "descriptor is NULL"; return OSCAR_E_ARG; }
  if (D->dim != 2 && D->dim != 3) { why = "dim must be 2 or 3"; return OSCAR_E_ARG; }
  if (D->nx < 1 || D->ny < 1 || D->nz < 1) { why = "grid sizes must be >= 1"; return OSCAR_E_ARG; }
  if (D->dim == 2 && D->nz != 1) { why = "nz must be 1 when dim = 2"; return OSCAR_E_ARG; }
  {
    // 32-bit indexing in the kernels: face arrays and the velocity gradient
    // (dim^2 components per cell) must stay below 2^31 entries
    int64_t nc = (int64_t)D->nx * D->ny * D->nz;
    int64_t nft = (int64_t)(D->nx + 1) * D->ny * D->nz + (int64_t)D->nx * (D->ny + 1) * D->nz +
                  (int64_t)D->nx * D->ny * (D->nz + 1);
    if (nft >= ((int64_t)1 << 31) || 9 * nc >= ((int64_t)1 << 31)) { why = "grid too large"; return OSCAR_E_ARG; }
  }
  if (!(D->h > 0.0) || !std::isfinite(D->h)) { why = "h must be > 0"; return OSCAR_E_ARG; }
  if (!(D->rho1 > 0) || !(D->rho2 > 0) || !(D->mu1 > 0) || !(D->mu2 > 0)) { why = "densities and viscosities must be > 0"; return OSCAR_E_ARG; }
  if (!(D->sigma >= 0) || !std::isfinite(D->sigma)) { why = "sigma must be >= 0"; return OSCAR_E_ARG; }
  if (!std::isfinite(D->theta_deg) || !std::isfinite(D->u_inlet)) { why = "theta and u_inlet must be finite"; return OSCAR_E_ARG; }
  if (D->precision != OSCAR_FP64 && D->precision != OSCAR_MIXED) { why = "unknown precision"; return OSCAR_E_ARG; }
  if (D->precond != OSCAR_PC_JACOBI && D->precond != OSCAR_PC_MG) { why = "unknown preconditioner"; return OSCAR_E_ARG; }
  if (D->precond == OSCAR_PC_MG) {
    MGInfo mg;
    mg_levels(*D, mg);
    if (mg.lv[mg.L].nc > MG_DENSE_MAX) { why = "grid too large for the multigrid hierarchy"; return OSCAR_E_ARG; }
  }
  if (D->mules_iter < 0 || D->mules_iter > 8) { why = "mules_iter must be in [0, 8]"; return OSCAR_E_ARG; }
  if (D->n_corr < 1 || D->n_corr > 64) { why = "n_corr must be in [1, 64]"; return OSCAR_E_ARG; }
  if (!(D->pcg_rtol > 0) || D->pcg_max_it < 1) { why = "pcg_rtol must be > 0 and pcg_max_it >= 1"; return OSCAR_E_ARG; }
  if (D->max_blocks < 0 || D->max_blocks > MAX_BLOCKS) { why = "max_blocks must be in [0, 1024]"; return OSCAR_E_ARG; }
  if (!(D->inner_rtol >= 0.0 && D->inner_rtol < 1.0)) { why = "inner_rtol must be in [0, 1)"; return OSCAR_E_ARG; }
  if (D->solve_mode < OSCAR_SOLVE_DEFAULT || D->solve_mode > OSCAR_SOLVE_PERSISTENT || D->reserved != 0) {
    why = "unknown solve_mode (or reserved not 0)";
    return OSCAR_E_ARG;
  }
  for (int f = 0; f < 2 * D->dim; ++f)
    if (D->bc[f] < OSCAR_BC_WALL || D->bc[f] > OSCAR_BC_OUTLET) { why = "unknown boundary type"; return OSCAR_E_ARG; }
  return OSCAR_OK;
}

// Persistent solves: the multigrid tail runs out of LDS when its block fits
// PQ_LDS_MAX bytes (more LDS per workgroup would cut the resident
// workgroups of the whole launch), else from global memory; a launch gives up
// after PQ_IDLE_S seconds without a completed phase.
constexpr int PQ_LDS_MAX = 40 * 1024;
constexpr double PQ_IDLE_S = 2.0;
static int pq_lds_for(const Slot &s) { return s.mg_pc && s.mg.tail_bytes <= PQ_LDS_MAX ? s.mg.tail_bytes : 0; }

// bit f set when box side f (f < 2*dim) is an outlet
uint32_t outlet_mask(const Slot &s) {
  uint32_t m = 0;
  for (int f = 0; f < 2 * s.dim; ++f)
    if (s.bcf[f] == F_OUTLET) m |= 1u << f;
  return m;
}

// per-cell face flags (bit f: neighbour across face f is fluid and inside the
// box; bit 6: solid) and the outlet-connectivity check
int build_flags(const oscar_desc &D, std::vector<uint8_t> &fl, int64_t &n_fluid, std::string &why) {
  const int64_t nx = D.nx, ny = D.ny, nz = D.nz, nc = nx * ny * nz;
  fl.assign(nc, 0);
  n_fluid = 0;
  auto id = [&](int64_t i, int64_t j, int64_t k) { return i + nx * (j + ny * k); };
  for (int64_t k = 0; k < nz; ++k)
    for (int64_t j = 0; j < ny; ++j)
      for (int64_t i = 0; i < nx; ++i) {
        int64_t P = id(i, j, k);
        if (D.mask[P]) { fl[P] = 0x40; continue; }
        n_fluid++;
        uint8_t b = 0;
        int64_t c[3] = {i, j, k}, n[3] = {nx, ny, nz};
        for (int f = 0; f < 2 * D.dim; ++f) {
          int e = f >> 1;
          int64_t q[3] = {c[0], c[1], c[2]};
          q[e] += (f & 1) ? 1 : -1;
          if (q[e] < 0 || q[e] >= n[e]) continue;
          if (!D.mask[id(q[0], q[1], q[2])]) b |= (uint8_t)(1u << f);
        }
        fl[P] = b;
      }
  if (n_fluid == 0) { why = "the mask has no fluid cell"; return OSCAR_E_MASK; }
  // flood fill from every fluid cell that owns an outlet face
  std::vector<uint8_t> seen(nc, 0);
  std::vector<int64_t> stack;
  for (int64_t k = 0; k < nz; ++k)
    for (int64_t j = 0; j < ny; ++j)
      for (int64_t i = 0; i < nx; ++i) {
        int64_t P = id(i, j, k);
        if (fl[P] & 0x40) continue;
        int64_t c[3] = {i, j, k}, n[3] = {nx, ny, nz};
        bool out = false;
        for (int f = 0; f < 2 * D.dim; ++f) {
          int e = f >> 1;
          bool edge = (f & 1) ? c[e] == n[e] - 1 : c[e] == 0;
          if (edge && D.bc[f] == OSCAR_BC_OUTLET) out = true;
        }
        if (out) { seen[P] = 1; stack.push_back(P); }
      }
  while (!stack.empty()) {
    int64_t P = stack.back();
    stack.pop_back();
    int64_t i = P % nx, j = (P / nx) % ny, k = P / (nx * ny);
    for (int f = 0; f < 2 * D.dim; ++f) {
      if (!(fl[P] & (1u << f))) continue;
      int64_t q[3] = {i, j, k};
      q[f >> 1] += (f & 1) ? 1 : -1;
      int64_t N = id(q[0], q[1], q[2]);
      if (!seen[N]) { seen[N] = 1; stack.push_back(N); }
    }
  }
  for (int64_t P = 0; P < nc; ++P)
    if (!(fl[P] & 0x40) && !seen[P]) {
      char buf[160];
      snprintf(buf, sizeof buf, "fluid cell %lld (i=%lld j=%lld k=%lld) cannot reach an outlet", (long long)P,
               (long long)(P % nx), (long long)((P / nx) % ny), (long long)(P / (nx * ny)));
      why = buf;
      return OSCAR_E_MASK;
    }
  return OSCAR_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------

struct oscar_ctx {
  oscar_desc D;
  Dims g;
  Slot s;                  // host copy of the slot (device pointers)
  Slot *d_slot = nullptr;  // device copy
  int2 *d_btab = nullptr;
  int btab_len = 0;
  hipStream_t stream = nullptr;
  SlotState *h_state = nullptr;   // pinned readback (the static-workspace variant: h_state_own)
  SlotState h_state_own;          // pageable readback of a context in the static workspace
  int static_dev = -1;            // device whose static workspace this context holds, or -1
  std::string err = "no error";
  int64_t n_fluid = 0;
  // host bookkeeping
  std::vector<double> Ehist;
  int k_f = 0;
  double last_E = 0.0, last_res = 0.0;
  int last_pcg = 0, pcg_call = 0, refine_call = 0, maxit_hits = 0;
  // Predicted CG iterations of the next solve of each kind: [viscous step,
  // capillary sub-step, stand-alone solve][corrector][first / later inner
  // solve of the mixed refinement].  A chunk of work ends with the
  // search-direction launch that holds a convergence test; the first chunk
  // of a solve runs the predicted iterations plus PRED_MARGIN and ends with
  // the test of the next one, so an exact prediction launches nothing past
  // convergence; later chunks add PRED_STEP iterations.  A launch past
  // convergence costs its early exit (about 2.4 us); one chunk too few costs
  // a host round trip (about 13 us) and the relaunch latency.
  static constexpr int PRED_MARGIN = 0;
  static constexpr int PRED_STEP = 2;
  int pred[3][64][2];
  bool refine_stall = false;  // an outer refinement stopped short of its tolerance
  bool mg_stale = true;       // the multigrid hierarchy predates the current 1/a_P
  int ctl_mode = 0;           // mode of the control block last set (0 viscous, 1 capillary)
  int total_seen = 0;   // device total_it at the last state read (0 after a state reset)
  // persistent solves (OSCAR_SOLVE_PERSISTENT): one launch per pressure solve
  bool pq = false;
  PQGlobal *d_pq = nullptr;   // the launch's batch words (device)
  PQGlobal h_pq;              // read back with the state
  int pq_wgs = 0, pq_lds = 0; // workgroups and LDS bytes of the launch
  long long pq_idle = 0;      // wall-clock ticks without a completed phase before the launch gives up
  // optional timing of sampled conjugate-gradient iterations: every
  // t_period-th iteration of a solve gives each of its launches a region of
  // per-workgroup wall-clock stamps in a small device buffer
  static constexpr int NT = 5;   // whole iteration, search direction, fine down, coarse levels, fine up
  static constexpr int TS_CAP = 64;       // stamp slots (each ts_reg regions of TS_WORDS words)
  static_assert(TS_CAP <= 64, "the span launch flags slots in one 64-bit mask");
  static constexpr int TS_BATCH = TS_CAP / 4;   // samples per span reduction; also per chunk of iterations
  int ts_reg = 0;                       // stamp regions per sample: the launches of one iteration
  bool timing = false;
  int t_period = 1;
  unsigned long long *d_ts = nullptr;   // TS_CAP x ts_reg regions of TS_WORDS words (device)
  unsigned long long *d_span = nullptr; // TS_CAP x ts_reg spans (device)
  unsigned long long *h_span = nullptr; // pinned copy of the spans
  double wall_hz = 0.0;                 // wall-clock rate
  enum { S_OPEN, S_RUN, S_DONE, S_COPIED };
  struct Sample {
    int g;        // the iteration's index among the call's iterations (device total_it when it ran)
    int slot;     // stamp slot
    int stage;    // S_OPEN: search direction enqueued, rest of the iteration not yet; S_RUN: all
                  // enqueued; S_DONE: ran and did work; S_COPIED: span copy enqueued
    bool split;   // a host read fell between its search direction and the rest
  };
  std::vector<Sample> samples;   // not yet folded
  std::vector<int> ts_free;      // free stamp slots
  std::vector<char> ts_zero;     // per stamp slot: its regions are known to be zero (no clearing before use)
  double t_ms[NT] = {0.0, 0.0, 0.0, 0.0, 0.0};
  int64_t t_cnt[NT] = {0, 0, 0, 0, 0};
  Launch L() const {
    Launch l;
    l.slots = d_slot;
    l.btab = d_btab;
    l.nblocks = btab_len;
    l.nslots = 1;
    l.stream = stream;
    return l;
  }
  bool mixed() const { return D.precision == OSCAR_MIXED; }
};

static int hip_fail(oscar_ctx *c, hipError_t e, const char *what) {
  char buf[256];
  snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString(e));
  if (c) c->err = buf;
  else g_err = buf;
  return OSCAR_E_HIP;
}

#define HIPCHK(c, x)                                       \
  do {                                                     \
    hipError_t _e = (x);                                   \
    if (_e != hipSuccess) return hip_fail((c), _e, #x);   \
  } while (0)

static int set_ctl(oscar_ctx *c, const SlotCtl &ctl) {
  CtlUpdate u;
  memset(&u, 0, sizeof u);
  u.n = 1;
  u.slot[0] = 0;
  u.ctl[0] = ctl;
  c->ctl_mode = ctl.mode;
  launch_ctl_update(c->L(), u);
  HIPCHK(c, hipGetLastError());
  return OSCAR_OK;
}

// Timing samples after a synchronisation of the stream: spans whose copy
// was enqueued earlier are folded into the totals; the other samples have
// run, and count when their iteration did work (g below the device's
// iteration count: launches enqueued past the convergence test exit at
// once).  Once TS_BATCH samples (or, with `flush`, any) await their spans,
// the spans of every stamp region are reduced and copied to the host in one
// launch and one copy, stream-ordered, to be folded after the next
// synchronisation.
static int settle_samples(oscar_ctx *c, bool flush) {
  const bool mg = c->D.precond == OSCAR_PC_MG;
  const int ncoarse = mg ? mg_part_launches(c->s, 1) : 0;
  // parts as ranges of stamp regions: search direction, fine down, coarse levels, fine up
  const int p0[4] = {0, 1, 2, 2 + ncoarse}, p1[4] = {1, 2, 2 + ncoarse, 3 + ncoarse};
  const int parts = mg ? 4 : 1;
  const int total = c->h_state->total_it;
  std::vector<oscar_ctx::Sample> keep;
  int waiting = 0;
  for (oscar_ctx::Sample x : c->samples) {
    if (x.stage == oscar_ctx::S_OPEN) {   // the rest of its iteration is still to be enqueued
      keep.push_back(x);
      continue;
    }
    if (x.stage == oscar_ctx::S_RUN) {
      if (x.g >= total) {   // its launches exited without work
        c->ts_free.push_back(x.slot);
        continue;
      }
      x.stage = oscar_ctx::S_DONE;
    }
    if (x.stage == oscar_ctx::S_DONE) {
      ++waiting;
      keep.push_back(x);
      continue;
    }
    c->ts_free.push_back(x.slot);
    c->ts_zero[x.slot] = 1;   // the span launch that copied it cleared its regions
    const unsigned long long *t = c->h_span + 2 * (size_t)c->ts_reg * x.slot;
    // first and last stamp of the search direction (part 0) and of the rest
    unsigned long long first[2] = {~0ull, ~0ull}, last[2] = {0ull, 0ull};
    for (int k = 0; k < parts; ++k) {
      unsigned long long lo = ~0ull, hi = 0ull;
      for (int r = p0[k]; r < p1[k]; ++r) {
        lo = t[2 * r] < lo ? t[2 * r] : lo;
        hi = t[2 * r + 1] > hi ? t[2 * r + 1] : hi;
      }
      if (hi <= lo) continue;   // a part that stamped nothing
      c->t_ms[1 + k] += 1e3 * (double)(hi - lo) / c->wall_hz;
      c->t_cnt[1 + k] += 1;
      const int h = k > 0;
      first[h] = lo < first[h] ? lo : first[h];
      last[h] = hi > last[h] ? hi : last[h];
    }
    // whole iteration: first to last stamp; when a host read fell between
    // the search direction and the rest, the two spans without the gap
    const unsigned long long f0 = first[0] < first[1] ? first[0] : first[1];
    const unsigned long long l0 = last[0] > last[1] ? last[0] : last[1];
    double whole = l0 > f0 ? (double)(l0 - f0) : 0.0;
    if (x.split && last[0] > first[0] && last[1] > first[1])
      whole = (double)(last[0] - first[0]) + (double)(last[1] - first[1]);
    if (whole > 0.0) {
      c->t_ms[0] += 1e3 * whole / c->wall_hz;
      c->t_cnt[0] += 1;
    }
  }
  c->samples.swap(keep);
  if (waiting == 0 || (waiting < oscar_ctx::TS_BATCH && !flush)) return OSCAR_OK;
  const int nreg = oscar_ctx::TS_CAP * c->ts_reg;
  unsigned long long clear = 0ull;   // slots whose spans this launch takes: zeroed for their next use
  for (const oscar_ctx::Sample &x : c->samples)
    if (x.stage == oscar_ctx::S_DONE) clear |= 1ull << x.slot;
  launch_ts_span(c->d_ts, nreg, c->d_span, c->ts_reg, clear, c->stream);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipMemcpyAsync(c->h_span, c->d_span, sizeof(unsigned long long) * 2 * nreg, hipMemcpyDeviceToHost,
                           c->stream));
  for (oscar_ctx::Sample &x : c->samples)
    if (x.stage == oscar_ctx::S_DONE) x.stage = oscar_ctx::S_COPIED;
  return OSCAR_OK;
}

// an inner solve ended: search-direction launches whose iteration was never
// completed (they found convergence) leave their samples
static void drop_open_samples(oscar_ctx *c) {
  std::vector<oscar_ctx::Sample> keep;
  for (const oscar_ctx::Sample &x : c->samples)
    if (x.stage == oscar_ctx::S_OPEN) c->ts_free.push_back(x.slot);
    else keep.push_back(x);
  c->samples.swap(keep);
}

// synchronisation: the device state into h_state
static int read_state(oscar_ctx *c) {
  HIPCHK(c, hipMemcpyAsync(c->h_state, c->s.st, sizeof(SlotState), hipMemcpyDeviceToHost, c->stream));
  if (c->pq) HIPCHK(c, hipMemcpyAsync(&c->h_pq, c->d_pq, sizeof(PQGlobal), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (c->pq && c->h_pq.err) {
    c->err = "persistent pressure solve: no phase completed within its time limit";
    return OSCAR_E_HIP;
  }
  c->total_seen = c->h_state->total_it;
  return c->samples.empty() ? OSCAR_OK : settle_samples(c, false);
}

// every pending sample folded into the totals
static int drain_samples(oscar_ctx *c) {
  for (int round = 0; round < 3 && !c->samples.empty(); ++round) {
    int rc = read_state(c);
    if (!rc && !c->samples.empty()) rc = settle_samples(c, true);
    if (rc) return rc;
  }
  return OSCAR_OK;
}

// a state reset (iteration counts to zero) is enqueued: samples still
// pending belong to the previous count and are dropped
static void state_reset(oscar_ctx *c, const Launch &L) {
  launch_state_reset(L, 1);
  c->total_seen = 0;
  for (const oscar_ctx::Sample &x : c->samples) c->ts_free.push_back(x.slot);
  c->samples.clear();
}

// Position in the launch sequence of an inner solve after its initial
// cycle: iteration it is its search-direction launch D(it), which holds the
// convergence test, and with multigrid the rest of the iteration T(it): fine
// down, the coarse levels, fine up.  Chunks end right after a D launch.
struct CgPos {
  int base = 0;        // iterations of the call before this inner solve
  int next = 0;        // iteration of the next D launch
  bool tail = false;   // T(next - 1) is due
  int tail_slot = -1;  // its stamp slot (-1: not sampled)
};

// n more D launches, each preceded by the due T launch (with timing on,
// every t_period-th iteration gets a free stamp slot, zeroed first)
template <typename R>
static int enqueue_chunk(oscar_ctx *c, CgPos &q, int n) {
  Launch L = c->L();
  const bool mg = c->D.precond == OSCAR_PC_MG;
  const size_t slot_words = (size_t)TS_WORDS * c->ts_reg;
  const int ncoarse = mg ? mg_part_launches(c->s, 1) : 0;
  auto region = [&](int slot, int r) -> unsigned long long * {
    return slot < 0 ? nullptr : c->d_ts + slot_words * slot + (size_t)TS_WORDS * r;
  };
  for (int x = 0; x < n; ++x) {
    if (q.tail) {
      const int it = q.next - 1;
      if (q.tail_slot >= 0)
        for (oscar_ctx::Sample &smp : c->samples)
          if (smp.slot == q.tail_slot && smp.stage == oscar_ctx::S_OPEN) {
            smp.stage = oscar_ctx::S_RUN;
            smp.split = x == 0;   // its D launch ended the previous chunk
          }
      launch_mg_cycle_part<R>(c->s, L, it, 0, c->ctl_mode, region(q.tail_slot, 1));
      launch_mg_cycle_part<R>(c->s, L, it, 1, c->ctl_mode, region(q.tail_slot, 2));
      launch_mg_cycle_part<R>(c->s, L, it, 2, c->ctl_mode, region(q.tail_slot, 2 + ncoarse));
      q.tail = false;
    }
    const int it = q.next++;
    int slot = -1;
    if (c->timing && it % c->t_period == 0 && !c->ts_free.empty()) {
      slot = c->ts_free.back();
      c->ts_free.pop_back();
      if (!c->ts_zero[slot])
        HIPCHK(c, hipMemsetAsync(c->d_ts + slot_words * slot, 0, sizeof(unsigned long long) * slot_words, c->stream));
      c->ts_zero[slot] = 0;
      c->samples.push_back({q.base + it, slot, mg ? oscar_ctx::S_OPEN : oscar_ctx::S_RUN, false});
    }
    if (mg) {
      launch_mg_dir<R>(c->s, L, it, region(slot, 0));
      q.tail = true;
      q.tail_slot = slot;
    } else {
      launch_cg_iters<R>(L, it, 1, region(slot, 0));
    }
  }
  HIPCHK(c, hipGetLastError());
  return OSCAR_OK;
}

// Block-table segment of one slot: workgroups are dealt round-robin to the
// 8 XCDs (each with its own L2), so position p of a segment that starts on a
// multiple of 8 runs on XCD p % 8.  Each XCD gets a contiguous run of the
// slot's blocks (neighbouring cells share its L2); the segment is padded to
// a multiple of 8 with entries (slot, -1) that kernels skip.
static void append_segment(std::vector<int2> &bt, int slot, int nb) {
  const int X = 8;
  while (bt.size() % X) bt.push_back(make_int2(slot, -1));
  int q = nb / X, rem = nb % X;
  int padded = (nb + X - 1) / X * X;
  for (int p = 0; p < padded; ++p) {
    int x = p % X, i = p / X;
    int cnt = q + (x < rem ? 1 : 0);
    int start = x * q + (x < rem ? x : rem);
    bt.push_back(make_int2(slot, i < cnt ? start + i : -1));
  }
}

// smallest relative residual reduction asked of one FP32 inner solve of the
// mixed-precision path (each inner solve otherwise stops at the residual the
// FP64 test needs)
static double inner_rtol(const oscar_desc &D) { return D.inner_rtol > 0.0 ? D.inner_rtol : 1e-6; }

int oscar::blocks_for(int64_t nc, int cap) {
  if (cap < 1 || cap > MAX_BLOCKS) cap = MAX_BLOCKS;
  int64_t n = (nc + BLOCK - 1) / BLOCK;
  return (int)(n < cap ? n : cap);
}

extern "C" double oscar_dt_brackbill(double rho1, double rho2, double h, double sigma) {
  const double pi = 3.14159265358979323846;
  double rbar = 0.5 * (rho1 + rho2);
  return std::sqrt(rbar * h * h * h / (2.0 * pi * sigma));
}

extern "C" int32_t oscar_workspace_size(const oscar_desc *desc, uint64_t *bytes) {
  std::string why;
  if (!bytes) { g_err = "bytes is NULL"; return OSCAR_E_ARG; }
  int rc = check_desc(desc, why);
  if (rc) { g_err = why; return rc; }
  Carver cv;
  Slot s;
  layout(*desc, cv, &s, true);
  cv.take(sizeof(Slot));
  cv.take(sizeof(int2) * (uint64_t)(dims_of(*desc).nblocks + 8));
  cv.take(sizeof(PQGlobal));
  *bytes = cv.off;
  return OSCAR_OK;
}

// static_dev >= 0: the workspace is that device's static array and the
// state readback goes through pageable host memory inside the context, so
// nothing is allocated by HIP.
static int32_t create_impl(const oscar_desc *desc, void *ws, uint64_t bytes, void *hip_stream, oscar_ctx **out,
                           int static_dev) {
  if (!out) { g_err = "out is NULL"; return OSCAR_E_ARG; }
  *out = nullptr;
  std::string why;
  int rc = check_desc(desc, why);
  if (rc) { g_err = why; return rc; }
  if (!desc->mask || !desc->alpha0) { g_err = "mask and alpha0 must be non-NULL"; return OSCAR_E_ARG; }
  uint64_t need = 0;
  oscar_workspace_size(desc, &need);
  if (!ws || bytes < need || ((uintptr_t)ws % ALIGN) != 0) {
    char buf[160];
    snprintf(buf, sizeof buf, "workspace %p of %llu bytes; need %llu bytes, 256-byte aligned", ws,
             (unsigned long long)bytes, (unsigned long long)need);
    g_err = buf;
    return OSCAR_E_WORKSPACE;
  }
  std::vector<uint8_t> fl;
  int64_t n_fluid = 0;
  rc = build_flags(*desc, fl, n_fluid, why);
  if (rc) { g_err = why; return rc; }
  const int64_t nc = (int64_t)desc->nx * desc->ny * desc->nz;
  for (int64_t P = 0; P < nc; ++P)
    if (!desc->mask[P] && !std::isfinite(desc->alpha0[P])) { g_err = "alpha0 has a non-finite value"; return OSCAR_E_ARG; }

  if (desc->precond == OSCAR_PC_MG) {   // the multigrid tail runs out of LDS
    MGInfo mg;
    mg_levels(*desc, mg);
    int dev = 0, lds = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (e != hipSuccess) return hip_fail(nullptr, e, "hipDeviceGetAttribute");
    if (lds < mg.tail_bytes) {
      char buf[160];
      snprintf(buf, sizeof buf, "the multigrid tail needs %d bytes of LDS per workgroup; the device has %d",
               (int)mg.tail_bytes, lds);
      g_err = buf;
      return OSCAR_E_ARG;
    }
  }
  oscar_ctx *c = new oscar_ctx();
  for (auto &kind : c->pred)
    for (auto &corr : kind) corr[0] = corr[1] = 16;
  c->D = *desc;
  c->D.mask = nullptr;
  c->D.alpha0 = nullptr;
  c->g = dims_of(*desc);
  c->stream = (hipStream_t)hip_stream;
  c->n_fluid = n_fluid;
  Carver cv;
  cv.base = (char *)ws;
  Slot &s = c->s;
  memset(&s, 0, sizeof s);
  layout(*desc, cv, &s, true);
  c->d_slot = (Slot *)cv.take(sizeof(Slot));
  c->d_btab = (int2 *)cv.take(sizeof(int2) * (uint64_t)(c->g.nblocks + 8));
  c->d_pq = (PQGlobal *)cv.take(sizeof(PQGlobal));
  s.dim = desc->dim;
  s.nx = desc->nx;
  s.ny = desc->ny;
  s.nz = desc->nz;
  s.nc = (int32_t)c->g.nc;
  s.nf0 = (int32_t)c->g.nf0;
  s.nf1 = (int32_t)c->g.nf1;
  s.nf2 = (int32_t)c->g.nf2;
  s.nftot = (int32_t)c->g.nft;
  s.nxy = desc->nx * desc->ny;
  s.block0 = 0;
  s.nblocks = c->g.nblocks;
  s.n_fluid = (int32_t)n_fluid;
  s.precision = desc->precision;
  s.mules_iter = desc->mules_iter > 1 ? desc->mules_iter : 1;
  s.mg_pc = desc->precond == OSCAR_PC_MG;
  for (int f = 0; f < 6; ++f)
    s.bcf[f] = desc->bc[f] == OSCAR_BC_INLET ? F_INLET : (desc->bc[f] == OSCAR_BC_OUTLET ? F_OUTLET : F_WALL);
  s.outlet = outlet_mask(s);
  const double h = desc->h;
  s.h = h;
  s.V = desc->dim == 3 ? h * h * h : h * h;
  s.S = desc->dim == 3 ? h * h : h;
  s.Sh = s.S / h;
  s.hh = 0.5 * h;
  s.S2h = s.S / s.hh;
  s.delta = 1e-8 / h;
  // cos and sin of theta from the complementary angle, exact at 90 degrees
  const double pi = 3.14159265358979323846;
  double comp = (90.0 - desc->theta_deg) * (pi / 180.0);
  s.cos_t = std::sin(comp);
  s.sin_t = std::cos(comp);
  s.rho1 = desc->rho1;
  s.mu1 = desc->mu1;
  s.rho2 = desc->rho2;
  s.mu2 = desc->mu2;
  s.sigma = desc->sigma;
  s.u_inlet = desc->u_inlet;

  auto fail = [&](hipError_t e, const char *what) {
    hip_fail(nullptr, e, what);
    if (c->h_state && c->static_dev < 0) (void)hipHostFree(c->h_state);
    delete c;
    return OSCAR_E_HIP;
  };
  hipError_t e;
  c->static_dev = static_dev;
  if (static_dev >= 0) c->h_state = &c->h_state_own;
  else if ((e = hipHostMalloc((void **)&c->h_state, sizeof(SlotState), hipHostMallocDefault)) != hipSuccess)
    return fail(e, "hipHostMalloc");
  if (desc->solve_mode == OSCAR_SOLVE_PERSISTENT) {
    int dev = 0, khz = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return fail(e, "hipGetDevice");
    if ((e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev)) != hipSuccess)
      return fail(e, "hipDeviceGetAttribute");
    c->pq_lds = pq_lds_for(s);
    const int res = desc->precision == OSCAR_MIXED ? pq_resident_wgs<float>(c->pq_lds)
                                                   : pq_resident_wgs<double>(c->pq_lds);
    if (khz <= 0 || res < 1) return fail(hipErrorInvalidValue, "sizing the persistent solve");
    c->pq_idle = (long long)(PQ_IDLE_S * 1e3 * (double)khz);
    c->pq_wgs = res < c->g.nblocks ? res : c->g.nblocks;
    c->pq = true;
  }
  if ((e = hipMemsetAsync(ws, 0, cv.off, c->stream)) != hipSuccess) return fail(e, "hipMemsetAsync");
  if ((e = hipMemcpyAsync((void *)s.flags, fl.data(), nc, hipMemcpyHostToDevice, c->stream)) != hipSuccess)
    return fail(e, "upload mask");
  std::vector<int2> bt;
  append_segment(bt, 0, c->g.nblocks);
  c->btab_len = (int)bt.size();
  if ((e = hipMemcpyAsync(c->d_btab, bt.data(), sizeof(int2) * bt.size(), hipMemcpyHostToDevice, c->stream)) != hipSuccess)
    return fail(e, "upload block table");
  if ((e = hipMemcpyAsync(c->d_slot, &s, sizeof(Slot), hipMemcpyHostToDevice, c->stream)) != hipSuccess)
    return fail(e, "upload slot");
  if (desc->precision == OSCAR_MIXED) {
    std::vector<float> a(nc);
    for (int64_t P = 0; P < nc; ++P) a[P] = desc->mask[P] ? 0.f : (float)desc->alpha0[P];
    e = hipMemcpyAsync(s.alpha, a.data(), 4 * nc, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  } else {
    std::vector<double> a(nc);
    for (int64_t P = 0; P < nc; ++P) a[P] = desc->mask[P] ? 0.0 : desc->alpha0[P];
    e = hipMemcpyAsync(s.alpha, a.data(), 8 * nc, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  }
  if (e != hipSuccess) return fail(e, "upload alpha0");
  *out = c;
  return OSCAR_OK;
}

extern "C" int32_t oscar_create(const oscar_desc *desc, void *ws, uint64_t bytes, void *hip_stream,
                                oscar_ctx **out) {
  return create_impl(desc, ws, bytes, hip_stream, out, -1);
}

// ---------------------------------------------------------------------------
// the allocation-free variant: the workspace is a static device array
// ---------------------------------------------------------------------------

namespace {

// The workspace of oscar_create_static.  In host code `scratch` names a
// host-side stand-in; its device address on each device comes from
// hipGetSymbolAddress and is the only handle used.
constexpr uint64_t STATIC_WS_BYTES = OSCAR_STATIC_WORKSPACE_BYTES;
static __device__ __align__(256) unsigned char scratch[STATIC_WS_BYTES];

constexpr int STATIC_MAX_DEV = 64;
struct StaticWs {
  void *ptr = nullptr;   // device address of `scratch` on this device (0: not looked up yet)
  bool busy = false;     // a live context holds it
};
StaticWs g_static[STATIC_MAX_DEV];
std::mutex g_static_mu;

}  // namespace

extern "C" int32_t oscar_create_static(const oscar_desc *desc, void *hip_stream, oscar_ctx **out) {
  if (!out) { g_err = "out is NULL"; return OSCAR_E_ARG; }
  *out = nullptr;
  uint64_t need = 0;
  int rc = oscar_workspace_size(desc, &need);
  if (rc) return rc;
  if (need > STATIC_WS_BYTES) {
    char buf[200];
    snprintf(buf, sizeof buf, "the descriptor needs %llu bytes of workspace; the static workspace holds %llu",
             (unsigned long long)need, (unsigned long long)STATIC_WS_BYTES);
    g_err = buf;
    return OSCAR_E_WORKSPACE;
  }
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(nullptr, e, "hipGetDevice");
  if (dev < 0 || dev >= STATIC_MAX_DEV) { g_err = "device ordinal out of range"; return OSCAR_E_ARG; }
  void *ws = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_static_mu);
    StaticWs &w = g_static[dev];
    if (!w.ptr) {   // once per device, with that device current
      void *p = nullptr;
      e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (e != hipSuccess) return hip_fail(nullptr, e, "hipGetSymbolAddress(scratch)");
      if (!p) { g_err = "hipGetSymbolAddress(scratch) returned NULL"; return OSCAR_E_HIP; }
      w.ptr = p;
    }
    if (w.busy) { g_err = "the static workspace of this device is held by another context"; return OSCAR_E_CAPACITY; }
    w.busy = true;
    ws = w.ptr;
  }
  rc = create_impl(desc, ws, STATIC_WS_BYTES, hip_stream, out, dev);
  if (rc) {
    std::lock_guard<std::mutex> lock(g_static_mu);
    g_static[dev].busy = false;
  }
  return rc;
}

extern "C" void oscar_destroy(oscar_ctx *c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  if (c->d_ts) (void)hipFree(c->d_ts);
  if (c->d_span) (void)hipFree(c->d_span);
  if (c->h_span) (void)hipHostFree(c->h_span);
  if (c->static_dev >= 0) {
    std::lock_guard<std::mutex> lock(g_static_mu);
    g_static[c->static_dev].busy = false;
  } else if (c->h_state) {
    (void)hipHostFree(c->h_state);
  }
  delete c;
}

extern "C" const char *oscar_last_error(const oscar_ctx *c) { return c ? c->err.c_str() : g_err.c_str(); }

// ---------------------------------------------------------------------------
// orchestration
// ---------------------------------------------------------------------------

// Solve the assembled pressure equation of the current corrector on the
// device: chunks of CG iterations until the slot's done flag is set; in mixed
// precision, FP32 inner solves wrapped in FP64 refinement.
//
// The host reads the device state once per chunk.  The first chunk of an
// inner solve is the iteration count of the same equation (kind, corrector,
// first or later inner solve) at the previous call plus a margin, so most
// solves need a single read; in mixed precision the refinement step is
// enqueued behind every chunk and acts only if the chunk finished the inner
// solve, so one read also decides the outer step.
// Persistent mode: the whole solve as one launch (after the multigrid
// coarse operators, when they are stale); nothing is read back here.
template <typename R>
static int enqueue_solve_pq(oscar_ctx *c) {
  if (c->D.precond == OSCAR_PC_MG && c->mg_stale) {
    launch_mg_setup<R>(c->s, c->stream);
    c->mg_stale = false;
  }
  launch_pq_init(c->d_slot, nullptr, 1, c->d_pq, c->stream);
  launch_pq_solve<R>(c->d_slot, nullptr, 1, c->d_pq, c->pq_wgs, c->pq_lds, c->pq_idle, c->stream);
  HIPCHK(c, hipGetLastError());
  return OSCAR_OK;
}

template <typename R>
static int solve_pressure(oscar_ctx *c, int &iters, int kind, int corr) {
  c->refine_stall = false;
  if (c->pq) {
    int rc = enqueue_solve_pq<R>(c);
    if (!rc) rc = read_state(c);
    if (rc) return rc;
    iters = c->h_state->total_it - c->h_state->solve_base;
    c->total_seen = c->h_state->total_it;
    c->refine_stall = c->h_state->stalled != 0;
    c->refine_call += c->h_state->ref_solve;
    return OSCAR_OK;
  }
  const int start_total = c->total_seen;   // no iterations ran since the last state read
  const int max_it = c->D.pcg_max_it;
  const bool mg = c->D.precond == OSCAR_PC_MG;
  const bool mixed = c->mixed();
  if (mg && c->mg_stale) {   // coarse operators of the coefficients (1/a_P of the current assembly)
    launch_mg_setup<R>(c->s, c->stream);
    HIPCHK(c, hipGetLastError());
    c->mg_stale = false;
  }
  int (&pr)[2] = c->pred[kind][corr < 63 ? corr : 63];
  int outer = 0;   // refinement steps taken
  for (;;) {
    // one inner solve: w_0 = A D^-1 r_0 (Jacobi) or the V-cycle of r_0 (MG),
    // then chunks of iterations from index 0 until the device flags it done
    CgPos q;
    q.base = c->total_seen;
    const int base = q.base;
    if (mg)   // z_0 = B r_0
      for (int part = 0; part < 3; ++part) launch_mg_cycle_part<R>(c->s, c->L(), -1, part, c->ctl_mode);
    else launch_cg_init<R>(c->L());
    HIPCHK(c, hipGetLastError());
    int &pred = pr[outer > 0 ? 1 : 0];
    // the predicted iterations, and the convergence test after them
    int chunk = pred + 1 + oscar_ctx::PRED_MARGIN;
    for (;;) {
      if (q.next > max_it + 1) { c->err = "conjugate gradient did not terminate"; return OSCAR_E_HIP; }
      // with timing on, a chunk holds at most TS_BATCH samples
      const int cap = oscar_ctx::TS_BATCH * c->t_period;
      const int n = c->timing && chunk > cap ? cap : chunk;
      int r = enqueue_chunk<R>(c, q, n);
      if (r) return r;
      if (mixed) {
        launch_refine<R>(c->L());
        HIPCHK(c, hipGetLastError());
      }
      r = read_state(c);
      if (r) return r;
      // finished: done (FP64), or the refinement ran (it back to 0) or had
      // nothing to refine (mixed)
      if (mixed ? c->h_state->it == 0 : c->h_state->done != 0) break;
      chunk = oscar_ctx::PRED_STEP;
    }
    if (!c->samples.empty()) drop_open_samples(c);
    const int used = c->h_state->total_it - base;
    if (used > 0) pred = used;
    if (!mixed || used == 0) break;   // FP64, or the equation was solved before any iteration
    ++outer;
    // the refinement met the tolerance, or stalled (an outer step no longer
    // halved the FP64 residual, or REFINE_MAX steps: decided on the device)
    if (c->h_state->stalled) c->refine_stall = true;
    if (c->h_state->done) break;
    if (outer > REFINE_MAX) { c->err = "refinement did not terminate"; return OSCAR_E_HIP; }
  }
  c->refine_call += outer;
  iters = c->total_seen - start_total;
  return OSCAR_OK;
}

template <typename R>
static int run_correctors(oscar_ctx *c, bool cr, double &E, int &warn) {
  Launch L = c->L();
  if (c->pq) {   // every corrector enqueued, one state read at the end
    for (int j = 0; j < c->D.n_corr; ++j) {
      launch_predictor<R>(L);
      launch_pressure_setup<R>(L, cr && j == 0);
      HIPCHK(c, hipGetLastError());
      int rc = enqueue_solve_pq<R>(c);
      if (rc) return rc;
      launch_correct<R>(L, j);
      HIPCHK(c, hipGetLastError());
    }
    int rc = read_state(c);
    if (rc) return rc;
    const SlotState &st = *c->h_state;
    if (cr) E = st.E;
    c->last_pcg = st.total_it - st.solve_base;
    c->pcg_call = st.total_it;   // the call's state reset zeroed the count
    c->total_seen = st.total_it;
    c->refine_call = st.refine_steps;
    if (st.maxit_hit) warn = OSCAR_W_PCG_MAXIT;
    else if (st.stall_hits && warn == OSCAR_OK) warn = OSCAR_W_REFINE_STALL;
    return OSCAR_OK;
  }
  for (int j = 0; j < c->D.n_corr; ++j) {
    launch_predictor<R>(L);
    launch_pressure_setup<R>(L, cr && j == 0);
    HIPCHK(c, hipGetLastError());
    int it = 0;
    int rc = solve_pressure<R>(c, it, cr ? 1 : 0, j);
    if (rc) return rc;
    if (cr && j == 0) E = c->h_state->E;
    c->last_pcg = it;
    c->pcg_call += it;
    if (c->h_state->maxit_hit) warn = OSCAR_W_PCG_MAXIT;
    else if (c->refine_stall && warn == OSCAR_OK) warn = OSCAR_W_REFINE_STALL;
    launch_correct<R>(L, j);
    HIPCHK(c, hipGetLastError());
  }
  return OSCAR_OK;
}

static SlotCtl make_ctl(const oscar_ctx *c, int mode, double dt, int n_sub) {
  SlotCtl k;
  memset(&k, 0, sizeof k);
  k.active = 1;
  k.mode = mode;
  k.dt = dt;
  k.ub = mode ? 0.0 : c->D.u_inlet;
  k.with_st = mode;
  k.rtol = c->D.pcg_rtol;
  k.rtol_inner = inner_rtol(c->D);
  k.max_it = c->D.pcg_max_it;
  k.last_corr = c->D.n_corr - 1;
  k.n_sub = n_sub;
  return k;
}

static int finish_call(oscar_ctx *c, int warn) {
  int rc = read_state(c);
  if (rc) return rc;
  const SlotState &st = *c->h_state;
  c->maxit_hits += st.maxit_hit;
  c->last_res = c->mixed() ? (st.bn64 > 0 ? st.rn64 / st.bn64 : 0.0) : (st.bn > 0 ? st.rn / st.bn : 0.0);
  if (st.nonfinite) { c->err = "non-finite velocity"; return OSCAR_E_NONFINITE; }
  if (st.unstable) { c->err = "transport Courant number above 1"; return OSCAR_E_UNSTABLE; }
  return warn;
}

template <typename R>
static int viscous_step_t(oscar_ctx *c, double dt) {
  Launch L = c->L();
  int rc = set_ctl(c, make_ctl(c, 0, dt, 1));
  if (rc) return rc;
  state_reset(c, L);
  c->pcg_call = 0;
  c->refine_call = 0;
  launch_copy_phi_prev<R>(L);
  launch_normals<R>(L, false);
  launch_advect<R>(L, c->s.mules_iter);
  launch_assemble<R>(L);
  c->mg_stale = true;
  HIPCHK(c, hipGetLastError());
  double E = 0.0;
  int warn = OSCAR_OK;
  rc = run_correctors<R>(c, false, E, warn);
  if (rc) return rc;
  return finish_call(c, warn);
}

template <typename R>
static int relax_t(oscar_ctx *c, double dt_vd, int n_sub, int max_iters, double tol) {
  Launch L = c->L();
  double dt = dt_vd / (double)n_sub;
  int rc = set_ctl(c, make_ctl(c, 1, dt, n_sub));
  if (rc) return rc;
  state_reset(c, L);
  launch_zero_usum<R>(L);
  HIPCHK(c, hipGetLastError());
  c->pcg_call = 0;
  c->refine_call = 0;
  c->Ehist.clear();
  int warn = OSCAR_OK;
  int kf = max_iters;
  for (int k = 0; k < max_iters; ++k) {
    launch_normals<R>(L, false);
    launch_advect<R>(L, c->s.mules_iter);
    launch_normals<R>(L, true);
    launch_assemble<R>(L);
    if (mg_rebuild(true, k)) c->mg_stale = true;
    HIPCHK(c, hipGetLastError());
    double E = 0.0;
    rc = run_correctors<R>(c, true, E, warn);
    if (rc) return rc;
    c->Ehist.push_back(E);
    c->last_E = E;
    if (c->h_state->nonfinite) break;
    if (E < tol) { kf = k + 1; break; }
  }
  c->k_f = kf;
  launch_finalize<R>(L);
  HIPCHK(c, hipGetLastError());
  return finish_call(c, warn);
}

extern "C" int32_t oscar_viscous_step(oscar_ctx *c, double dt_vd) {
  if (!c) { g_err = "ctx is NULL"; return OSCAR_E_ARG; }
  if (!(dt_vd > 0.0) || !std::isfinite(dt_vd)) { c->err = "dt_vd must be > 0"; return OSCAR_E_ARG; }
  return c->mixed() ? viscous_step_t<float>(c, dt_vd) : viscous_step_t<double>(c, dt_vd);
}

extern "C" int32_t oscar_capillary_relax(oscar_ctx *c, double dt_vd, int32_t n_sub, int32_t max_iters, double tol,
                                         int32_t *k_f, double *E_last) {
  if (!c) { g_err = "ctx is NULL"; return OSCAR_E_ARG; }
  if (!(dt_vd > 0.0) || !std::isfinite(dt_vd) || n_sub < 1 || max_iters < 1 || max_iters > n_sub || !(tol >= 0.0)) {
    c->err = "need dt_vd > 0, n_sub >= 1, 1 <= max_iters <= n_sub, tol >= 0";
    return OSCAR_E_ARG;
  }
  double dt = dt_vd / (double)n_sub;
  if (c->D.sigma > 0.0 && !(dt < oscar_dt_brackbill(c->D.rho1, c->D.rho2, c->D.h, c->D.sigma))) {
    char buf[160];
    snprintf(buf, sizeof buf, "dt_vd/n_sub = %.4g s is not below the Brackbill limit %.4g s", dt,
             oscar_dt_brackbill(c->D.rho1, c->D.rho2, c->D.h, c->D.sigma));
    c->err = buf;
    return OSCAR_E_UNSTABLE;
  }
  int rc = c->mixed() ? relax_t<float>(c, dt_vd, n_sub, max_iters, tol) : relax_t<double>(c, dt_vd, n_sub, max_iters, tol);
  if (k_f) *k_f = c->k_f;
  if (E_last) *E_last = c->last_E;
  return rc;
}

extern "C" int32_t oscar_relax_history(const oscar_ctx *c, double *E, int32_t cap, int32_t *n) {
  if (!c || (!E && cap > 0)) return OSCAR_E_ARG;
  int m = (int)c->Ehist.size() < cap ? (int)c->Ehist.size() : cap;
  for (int x = 0; x < m; ++x) E[x] = c->Ehist[x];
  if (n) *n = m;
  return OSCAR_OK;
}

template <typename R>
static int pressure_solve_t(oscar_ctx *c, int which, double dt, double rtol, int max_it, int *iters, double *res) {
  Launch L = c->L();
  SlotCtl k = make_ctl(c, which, dt, 1);
  k.rtol = rtol;
  k.max_it = max_it;
  int rc = set_ctl(c, k);
  if (rc) return rc;
  state_reset(c, L);
  // alpha_old = alpha (no transport), then curvature, momentum, predictor, solve
  int saved_max = c->D.pcg_max_it;
  c->D.pcg_max_it = max_it;
  if (which == 0) launch_copy_phi_prev<R>(L);
  hipError_t e = hipMemcpyAsync(c->s.alpha_old, c->s.alpha, (c->mixed() ? 4 : 8) * c->g.nc, hipMemcpyDeviceToDevice, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "copy alpha");
  if (which) launch_normals<R>(L, true);
  launch_assemble<R>(L);
  c->mg_stale = true;
  launch_predictor<R>(L);
  launch_pressure_setup<R>(L, false);
  HIPCHK(c, hipGetLastError());
  int it = 0;
  rc = solve_pressure<R>(c, it, 2, 0);
  c->D.pcg_max_it = saved_max;
  if (rc) return rc;
  int warn = c->h_state->maxit_hit ? OSCAR_W_PCG_MAXIT : (c->refine_stall ? OSCAR_W_REFINE_STALL : OSCAR_OK);
  if (iters) *iters = it;
  if (res) {
    // FP64 relative residual of the final pressure
    SlotCtl k2 = k;
    (void)k2;
    const SlotState &st = *c->h_state;
    if (c->mixed()) *res = st.bn64 > 0 ? st.rn64 / st.bn64 : 0.0;
    else {
      // recompute ||b - M p|| in FP64 with the setup kernel (it also refreshes rhs)
      launch_pressure_setup<R>(L, false);
      rc = read_state(c);
      if (rc) return rc;
      *res = st.bn > 0 ? st.rn / st.bn : 0.0;
    }
  }
  return warn;
}

extern "C" int32_t oscar_pressure_solve(oscar_ctx *c, int32_t which, double dt, double rtol, int32_t max_it,
                                        int32_t *iters, double *rel_residual_fp64) {
  if (!c) { g_err = "ctx is NULL"; return OSCAR_E_ARG; }
  if ((which != 0 && which != 1) || !(dt > 0.0) || !(rtol > 0.0) || max_it < 1) {
    c->err = "need which in {0,1}, dt > 0, rtol > 0, max_it >= 1";
    return OSCAR_E_ARG;
  }
  int it = 0;
  double res = 0.0;
  int rc = c->mixed() ? pressure_solve_t<float>(c, which, dt, rtol, max_it, &it, &res)
                      : pressure_solve_t<double>(c, which, dt, rtol, max_it, &it, &res);
  if (iters) *iters = it;
  if (rel_residual_fp64) *rel_residual_fp64 = res;
  return rc;
}

// ---------------------------------------------------------------------------
// fields and statistics
// ---------------------------------------------------------------------------

static void *field_ptr(oscar_ctx *c, int id, int64_t &len, bool &dbl) {
  const Slot &s = c->s;
  const int64_t nc = c->g.nc, dn = c->g.d * c->g.nc, nf = c->g.nft;
  dbl = false;
  switch (id) {
    case OSCAR_FIELD_ALPHA: len = nc; return s.alpha;
    case OSCAR_FIELD_U: len = dn; return s.U;
    case OSCAR_FIELD_P: len = nc; dbl = true; return s.p;
    case OSCAR_FIELD_U_VD: len = dn; return s.U_vd;
    case OSCAR_FIELD_P_VD: len = nc; dbl = true; return s.p_vd;
    case OSCAR_FIELD_U_CR: len = dn; return s.U_cr;
    case OSCAR_FIELD_P_CR: len = nc; dbl = true; return s.p_cr;
    case OSCAR_FIELD_PHI_VD: len = nf; return s.phi_vd;
    case OSCAR_FIELD_PHI_VD_PREV: len = nf; return s.phi_prev;
    case OSCAR_FIELD_PHI_CR: len = nf; return s.phi_cr;
    case OSCAR_FIELD_KAPPA: len = nc; return s.kappa;
    case OSCAR_FIELD_RAU: len = nc; return s.rAU;
    case OSCAR_FIELD_RHS: len = nc; dbl = true; return s.rhs;
    case OSCAR_FIELD_U_SUM: len = dn; return s.U_sum;
    case OSCAR_FIELD_HBYA: len = dn; return s.HbyA;
    case OSCAR_FIELD_NHATF: len = nf; return s.nhatf;
    default: len = -1; return nullptr;
  }
}

extern "C" int64_t oscar_field_len(const oscar_ctx *c, int32_t id) {
  if (!c) return -1;
  int64_t len;
  bool dbl;
  field_ptr(const_cast<oscar_ctx *>(c), id, len, dbl);
  return len;
}

extern "C" int32_t oscar_get_field(oscar_ctx *c, int32_t id, double *dst) {
  if (!c) { g_err = "ctx is NULL"; return OSCAR_E_ARG; }
  int64_t len;
  bool dbl;
  void *src = field_ptr(c, id, len, dbl);
  if (!src || !dst) { c->err = "unknown field or NULL destination"; return OSCAR_E_ARG; }
  if (dbl || !c->mixed()) {
    HIPCHK(c, hipMemcpyAsync(dst, src, 8 * len, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  } else {
    std::vector<float> t(len);
    HIPCHK(c, hipMemcpyAsync(t.data(), src, 4 * len, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int64_t x = 0; x < len; ++x) dst[x] = t[x];
  }
  return OSCAR_OK;
}

extern "C" int32_t oscar_set_field(oscar_ctx *c, int32_t id, const double *src) {
  if (!c) { g_err = "ctx is NULL"; return OSCAR_E_ARG; }
  int64_t len;
  bool dbl;
  void *dst = field_ptr(c, id, len, dbl);
  if (!dst || !src) { c->err = "unknown field or NULL source"; return OSCAR_E_ARG; }
  c->mg_stale = true;
  for (int64_t x = 0; x < len; ++x)
    if (!std::isfinite(src[x])) { c->err = "non-finite value in the field"; return OSCAR_E_NONFINITE; }
  if (dbl || !c->mixed()) {
    HIPCHK(c, hipMemcpyAsync(dst, src, 8 * len, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  } else {
    std::vector<float> t(len);
    for (int64_t x = 0; x < len; ++x) t[x] = (float)src[x];
    HIPCHK(c, hipMemcpyAsync(dst, t.data(), 4 * len, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  return OSCAR_OK;
}

extern "C" int32_t oscar_stats(oscar_ctx *c, oscar_stats_t *o) {
  if (!c || !o) return OSCAR_E_ARG;
  int rc = read_state(c);
  if (rc) return rc;
  const SlotState &st = *c->h_state;
  memset(o, 0, sizeof *o);
  o->mass_phase1 = st.mass1;
  o->max_courant = st.comax;
  o->mass_defect = st.mass_defect;
  o->last_E = c->last_E;
  o->last_res = c->last_res;
  o->last_pcg_iters = c->last_pcg;
  o->pcg_iters_call = c->pcg_call;
  o->refine_steps_call = c->refine_call;
  o->k_f = c->k_f;
  o->n_fluid = (int32_t)c->n_fluid;
  o->pcg_maxit_hits = c->maxit_hits;
  return OSCAR_OK;
}

extern "C" int32_t oscar_timing(oscar_ctx *c, int32_t period) {
  if (!c || period < 0) return OSCAR_E_ARG;
  int rc = drain_samples(c);
  if (rc) return rc;
  if (period && c->btab_len > TS_WORDS / 2) {
    c->err = "timing supports at most 1040 workgroups per launch";
    return OSCAR_E_ARG;
  }
  if (period && !c->d_ts) {   // measurement buffers, kept until oscar_destroy
    int dev = 0, khz = 0;
    HIPCHK(c, hipGetDevice(&dev));
    HIPCHK(c, hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    if (khz <= 0) {
      c->err = "device reports no wall-clock rate";
      return OSCAR_E_HIP;
    }
    c->wall_hz = 1e3 * (double)khz;
    c->ts_reg = c->D.precond == OSCAR_PC_MG ? 3 + mg_part_launches(c->s, 1) : 1;
    const size_t regions = (size_t)oscar_ctx::TS_CAP * c->ts_reg;
    HIPCHK(c, hipMalloc((void **)&c->d_ts, sizeof(unsigned long long) * TS_WORDS * regions));
    HIPCHK(c, hipMalloc((void **)&c->d_span, sizeof(unsigned long long) * 2 * regions));
    HIPCHK(c, hipHostMalloc((void **)&c->h_span, sizeof(unsigned long long) * 2 * regions, hipHostMallocDefault));
    for (int k = oscar_ctx::TS_CAP - 1; k >= 0; --k) c->ts_free.push_back(k);
    c->ts_zero.assign(oscar_ctx::TS_CAP, 0);
  }
  c->timing = period != 0;
  if (c->timing) {
    c->t_period = period;
    for (int k = 0; k < oscar_ctx::NT; ++k) {
      c->t_ms[k] = 0.0;
      c->t_cnt[k] = 0;
    }
  }
  return OSCAR_OK;
}

extern "C" int32_t oscar_timing_read(oscar_ctx *c, int32_t kernel, double *total_ms, int64_t *launches) {
  if (!c || kernel < 0 || kernel >= oscar_ctx::NT) return OSCAR_E_ARG;
  int rc = drain_samples(c);
  if (rc) return rc;
  if (total_ms) *total_ms = c->t_ms[kernel];
  if (launches) *launches = c->t_cnt[kernel];
  return OSCAR_OK;
}

// ---------------------------------------------------------------------------
// Serving engine: continuous batching of independent OSCAR requests.
//
// A request (descriptor + dt_vd, N, max_iters, tol) is admitted into a free
// slot when its workspace footprint fits a free region of the engine's
// workspace; its fields stay resident until released.  Each tick advances
// every resident request by one step in lockstep launches: a viscous step
// for a new request, a capillary sub-step otherwise.  Conjugate-gradient
// convergence, refinement and the E_k stop rule are per slot; a request that
// finishes is finalised (U, p) and waits for fetch/release while the others
// keep running.  Every per-slot quantity depends only on that slot's data and
// size, so a request's results are the same alone and in any mix.
// ---------------------------------------------------------------------------

namespace {

enum { ES_FREE = 0, ES_VD = 1, ES_CR = 2, ES_DONE = 3 };

struct EngSlot {
  int state = ES_FREE;
  oscar_desc D;
  Dims g;
  Slot s;
  uint64_t off = 0, bytes = 0;
  double dt_vd = 0.0, tol = 0.0;
  int n_sub = 1, max_iters = 1, k = 0, k_f = 0, status = OSCAR_OK;
  double last_E = 0.0;
  int64_t n_fluid = 0;
  int pred = 32, pred_inner = 16;
  bool stalled = false;   // a refinement of this tick stopped short of its tolerance
};

struct Region {
  uint64_t off, bytes;
};

}  // namespace

struct oscar_engine {
  int max_slots = 0, precision = OSCAR_FP64;
  char *ws = nullptr;
  uint64_t bytes = 0, heap_off = 0;
  hipStream_t stream = nullptr;
  Slot *d_slots = nullptr;
  int2 *d_btab = nullptr, *d_btab2 = nullptr;
  int2 *d_btab_j = nullptr, *d_btab_m = nullptr;   // block tables of the Jacobi and the multigrid slots
  int2 *d_btab_live = nullptr;     // block table of the multigrid slots still iterating in an inner solve
  int *d_act = nullptr;            // multigrid slot lists by dimension, then those whose hierarchy is
                                   // rebuilt this tick, then those still iterating (6 x max_slots)
  SlotState *d_states = nullptr;   // gathered copy of the slots' states
  // persistent solves (OSCAR_SOLVE_PERSISTENT): the list of the slots a
  // launch solves, its batch words and their host copy
  int solve_mode = OSCAR_SOLVE_LAUNCHES;
  int *d_pq_list = nullptr;
  PQGlobal *d_pq = nullptr;
  PQGlobal h_pq;
  long long pq_idle = 0;
  std::vector<std::pair<int, int>> pq_res;   // resident workgroups by LDS bytes (looked up once each)
  int btab_cap = 0;
  SlotState *h_states = nullptr;
  std::vector<EngSlot> slots;
  std::vector<Region> free_list;
  std::vector<int2> bt, bt2, bt_j, bt_m, bt_live;
  std::vector<int> act_m, act_live;
  std::string err = "no error";
  int64_t ticks = 0, cg_iters = 0;
};

static int eng_fail(oscar_engine *e, hipError_t x, const char *what) {
  char buf[256];
  snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString(x));
  if (e) e->err = buf;
  g_err = buf;
  return OSCAR_E_HIP;
}

#define EHIP(e, x)                                        \
  do {                                                    \
    hipError_t _x = (x);                                  \
    if (_x != hipSuccess) return eng_fail((e), _x, #x);   \
  } while (0)

static uint64_t eng_table_bytes(int max_slots, int btab_cap) {
  return up(sizeof(Slot) * (uint64_t)max_slots) + 5 * up(sizeof(int2) * (uint64_t)btab_cap) +
         up(sizeof(int) * 6 * (uint64_t)max_slots) + up(sizeof(SlotState) * (uint64_t)max_slots) +
         up(sizeof(int) * (uint64_t)max_slots) + up(sizeof(PQGlobal));
}

extern "C" int32_t oscar_engine_table_bytes(int32_t max_slots, uint64_t *bytes) {
  if (max_slots < 1 || max_slots > 4096 || !bytes) { g_err = "need 1 <= max_slots <= 4096"; return OSCAR_E_ARG; }
  *bytes = eng_table_bytes(max_slots, max_slots * (MAX_BLOCKS + 16));
  return OSCAR_OK;
}

extern "C" int32_t oscar_engine_create(int32_t max_slots, int32_t precision, void *ws, uint64_t bytes,
                                       void *hip_stream, oscar_engine **out) {
  if (!out) { g_err = "out is NULL"; return OSCAR_E_ARG; }
  *out = nullptr;
  if (max_slots < 1 || max_slots > 4096 || (precision != OSCAR_FP64 && precision != OSCAR_MIXED)) {
    g_err = "need 1 <= max_slots <= 4096 and a known precision";
    return OSCAR_E_ARG;
  }
  const int btab_cap = max_slots * (MAX_BLOCKS + 16);
  uint64_t tb = eng_table_bytes(max_slots, btab_cap);
  if (!ws || ((uintptr_t)ws % ALIGN) != 0 || bytes < tb) {
    g_err = "engine workspace too small or not 256-byte aligned";
    return OSCAR_E_WORKSPACE;
  }
  oscar_engine *e = new oscar_engine();
  e->max_slots = max_slots;
  e->precision = precision;
  e->ws = (char *)ws;
  e->bytes = bytes;
  e->stream = (hipStream_t)hip_stream;
  e->btab_cap = btab_cap;
  e->d_slots = (Slot *)ws;
  e->d_btab = (int2 *)(e->ws + up(sizeof(Slot) * (uint64_t)max_slots));
  e->d_btab2 = (int2 *)((char *)e->d_btab + up(sizeof(int2) * (uint64_t)btab_cap));
  e->d_btab_j = (int2 *)((char *)e->d_btab2 + up(sizeof(int2) * (uint64_t)btab_cap));
  e->d_btab_m = (int2 *)((char *)e->d_btab_j + up(sizeof(int2) * (uint64_t)btab_cap));
  e->d_btab_live = (int2 *)((char *)e->d_btab_m + up(sizeof(int2) * (uint64_t)btab_cap));
  e->d_act = (int *)((char *)e->d_btab_live + up(sizeof(int2) * (uint64_t)btab_cap));
  e->d_states = (SlotState *)((char *)e->d_act + up(sizeof(int) * 6 * (uint64_t)max_slots));
  e->d_pq_list = (int *)((char *)e->d_states + up(sizeof(SlotState) * (uint64_t)max_slots));
  e->d_pq = (PQGlobal *)((char *)e->d_pq_list + up(sizeof(int) * (uint64_t)max_slots));
  e->heap_off = tb;
  e->slots.resize(max_slots);
  e->free_list.push_back(Region{tb, bytes - tb});
  hipError_t x = hipHostMalloc((void **)&e->h_states, sizeof(SlotState) * max_slots, hipHostMallocDefault);
  if (x != hipSuccess) { eng_fail(nullptr, x, "hipHostMalloc"); delete e; return OSCAR_E_HIP; }
  // every table entry starts inactive: point each slot's ctl at a zeroed word
  x = hipMemsetAsync(ws, 0, tb, e->stream);
  if (x == hipSuccess) x = hipStreamSynchronize(e->stream);
  if (x != hipSuccess) { eng_fail(nullptr, x, "engine init"); (void)hipHostFree(e->h_states); delete e; return OSCAR_E_HIP; }
  *out = e;
  return OSCAR_OK;
}

extern "C" int32_t oscar_engine_set_solve_mode(oscar_engine *e, int32_t mode) {
  if (!e) { g_err = "engine is NULL"; return OSCAR_E_ARG; }
  if (mode < OSCAR_SOLVE_DEFAULT || mode > OSCAR_SOLVE_PERSISTENT) { e->err = "unknown solve mode"; return OSCAR_E_ARG; }
  e->solve_mode = mode == OSCAR_SOLVE_DEFAULT ? OSCAR_SOLVE_LAUNCHES : mode;
  return OSCAR_OK;
}

extern "C" void oscar_engine_destroy(oscar_engine *e) {
  if (!e) return;
  if (e->stream) (void)hipStreamSynchronize(e->stream);
  if (e->h_states) (void)hipHostFree(e->h_states);
  delete e;
}

extern "C" const char *oscar_engine_last_error(const oscar_engine *e) { return e ? e->err.c_str() : g_err.c_str(); }

static bool eng_alloc(oscar_engine *e, uint64_t need, uint64_t &off) {
  for (size_t i = 0; i < e->free_list.size(); ++i) {
    Region &r = e->free_list[i];
    if (r.bytes >= need) {
      off = r.off;
      r.off += need;
      r.bytes -= need;
      if (r.bytes == 0) e->free_list.erase(e->free_list.begin() + i);
      return true;
    }
  }
  return false;
}

static void eng_free(oscar_engine *e, uint64_t off, uint64_t bytes) {
  e->free_list.push_back(Region{off, bytes});
  std::sort(e->free_list.begin(), e->free_list.end(), [](const Region &a, const Region &b) { return a.off < b.off; });
  std::vector<Region> merged;
  for (const Region &r : e->free_list) {
    if (!merged.empty() && merged.back().off + merged.back().bytes == r.off) merged.back().bytes += r.bytes;
    else merged.push_back(r);
  }
  e->free_list.swap(merged);
}

extern "C" int32_t oscar_engine_free_bytes(const oscar_engine *e, uint64_t *largest, int32_t *free_slots) {
  if (!e) return OSCAR_E_ARG;
  uint64_t m = 0;
  for (const Region &r : e->free_list) m = r.bytes > m ? r.bytes : m;
  int f = 0;
  for (const EngSlot &s : e->slots) f += s.state == ES_FREE;
  if (largest) *largest = m;
  if (free_slots) *free_slots = f;
  return OSCAR_OK;
}

extern "C" int32_t oscar_engine_admit(oscar_engine *e, const oscar_desc *desc, double dt_vd, int32_t n_sub,
                                      int32_t max_iters, double tol, int32_t *slot_out) {
  if (!e) { g_err = "engine is NULL"; return OSCAR_E_ARG; }
  std::string why;
  int rc = check_desc(desc, why);
  if (rc) { e->err = why; return rc; }
  if (desc->precision != e->precision) { e->err = "descriptor precision differs from the engine's"; return OSCAR_E_ARG; }
  if (desc->precond == OSCAR_PC_MG) {   // the multigrid tail runs out of LDS
    MGInfo mg;
    mg_levels(*desc, mg);
    int dev = 0, lds = 0;
    hipError_t x = hipGetDevice(&dev);
    if (x == hipSuccess) x = hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (x != hipSuccess) return eng_fail(e, x, "hipDeviceGetAttribute");
    if (lds < mg.tail_bytes) { e->err = "the multigrid tail does not fit the device's LDS"; return OSCAR_E_ARG; }
  }
  if (!desc->mask || !desc->alpha0) { e->err = "mask and alpha0 must be non-NULL"; return OSCAR_E_ARG; }
  if (!(dt_vd > 0.0) || n_sub < 1 || max_iters < 1 || max_iters > n_sub || !(tol >= 0.0)) {
    e->err = "need dt_vd > 0, n_sub >= 1, 1 <= max_iters <= n_sub, tol >= 0";
    return OSCAR_E_ARG;
  }
  double dt = dt_vd / (double)n_sub;
  if (desc->sigma > 0.0 && !(dt < oscar_dt_brackbill(desc->rho1, desc->rho2, desc->h, desc->sigma))) {
    e->err = "dt_vd/n_sub is not below the Brackbill limit";
    return OSCAR_E_UNSTABLE;
  }
  std::vector<uint8_t> fl;
  int64_t n_fluid = 0;
  rc = build_flags(*desc, fl, n_fluid, why);
  if (rc) { e->err = why; return rc; }
  int idx = -1;
  for (int i = 0; i < e->max_slots; ++i)
    if (e->slots[i].state == ES_FREE) { idx = i; break; }
  Carver probe;
  Slot tmp;
  layout(*desc, probe, &tmp, true);
  uint64_t need = probe.off, off = 0;
  if (idx < 0 || !eng_alloc(e, need, off)) { e->err = "no free slot or workspace region"; return OSCAR_E_CAPACITY; }
  EngSlot &es = e->slots[idx];
  es = EngSlot();
  es.D = *desc;
  es.D.mask = nullptr;
  es.D.alpha0 = nullptr;
  es.g = dims_of(*desc);
  es.off = off;
  es.bytes = need;
  es.dt_vd = dt_vd;
  es.n_sub = n_sub;
  es.max_iters = max_iters;
  es.tol = tol;
  es.n_fluid = n_fluid;
  Carver cv;
  cv.base = e->ws + off;
  Slot &s = es.s;
  memset(&s, 0, sizeof s);
  layout(*desc, cv, &s, true);
  s.dim = desc->dim;
  s.nx = desc->nx;
  s.ny = desc->ny;
  s.nz = desc->nz;
  s.nc = (int32_t)es.g.nc;
  s.nf0 = (int32_t)es.g.nf0;
  s.nf1 = (int32_t)es.g.nf1;
  s.nf2 = (int32_t)es.g.nf2;
  s.nftot = (int32_t)es.g.nft;
  s.nxy = desc->nx * desc->ny;
  s.nblocks = es.g.nblocks;
  s.n_fluid = (int32_t)n_fluid;
  s.precision = desc->precision;
  s.mules_iter = desc->mules_iter > 1 ? desc->mules_iter : 1;
  s.mg_pc = desc->precond == OSCAR_PC_MG;
  for (int f = 0; f < 6; ++f)
    s.bcf[f] = desc->bc[f] == OSCAR_BC_INLET ? F_INLET : (desc->bc[f] == OSCAR_BC_OUTLET ? F_OUTLET : F_WALL);
  s.outlet = outlet_mask(s);
  const double h = desc->h;
  s.h = h;
  s.V = desc->dim == 3 ? h * h * h : h * h;
  s.S = desc->dim == 3 ? h * h : h;
  s.Sh = s.S / h;
  s.hh = 0.5 * h;
  s.S2h = s.S / s.hh;
  s.delta = 1e-8 / h;
  const double pi = 3.14159265358979323846;
  double comp = (90.0 - desc->theta_deg) * (pi / 180.0);
  s.cos_t = std::sin(comp);
  s.sin_t = std::cos(comp);
  s.rho1 = desc->rho1;
  s.mu1 = desc->mu1;
  s.rho2 = desc->rho2;
  s.mu2 = desc->mu2;
  s.sigma = desc->sigma;
  s.u_inlet = desc->u_inlet;
  const int64_t nc = es.g.nc;
  hipError_t x = hipMemsetAsync(e->ws + off, 0, need, e->stream);
  if (x == hipSuccess) x = hipMemcpyAsync((void *)s.flags, fl.data(), nc, hipMemcpyHostToDevice, e->stream);
  std::vector<double> a64;
  std::vector<float> a32;
  if (x == hipSuccess) {
    if (e->precision == OSCAR_MIXED) {
      a32.resize(nc);
      for (int64_t P = 0; P < nc; ++P) a32[P] = desc->mask[P] ? 0.f : (float)desc->alpha0[P];
      x = hipMemcpyAsync(s.alpha, a32.data(), 4 * nc, hipMemcpyHostToDevice, e->stream);
    } else {
      a64.resize(nc);
      for (int64_t P = 0; P < nc; ++P) a64[P] = desc->mask[P] ? 0.0 : desc->alpha0[P];
      x = hipMemcpyAsync(s.alpha, a64.data(), 8 * nc, hipMemcpyHostToDevice, e->stream);
    }
  }
  if (x == hipSuccess) x = hipMemcpyAsync(e->d_slots + idx, &s, sizeof(Slot), hipMemcpyHostToDevice, e->stream);
  if (x == hipSuccess) x = hipStreamSynchronize(e->stream);
  if (x != hipSuccess) {
    eng_free(e, off, need);
    es.state = ES_FREE;
    return eng_fail(e, x, "admit upload");
  }
  es.state = ES_VD;
  if (slot_out) *slot_out = idx;
  return OSCAR_OK;
}

static SlotCtl eng_ctl(const EngSlot &es, int mode, int precision) {
  SlotCtl k;
  memset(&k, 0, sizeof k);
  k.active = 1;
  k.mode = mode;
  k.dt = mode ? es.dt_vd / (double)es.n_sub : es.dt_vd;
  k.ub = mode ? 0.0 : es.D.u_inlet;
  k.with_st = mode;
  k.rtol = es.D.pcg_rtol;
  k.rtol_inner = inner_rtol(es.D);
  k.max_it = es.D.pcg_max_it;
  k.last_corr = es.D.n_corr - 1;
  k.n_sub = es.n_sub;
  k.substep = es.k;
  k.tol = es.tol;
  (void)precision;
  return k;
}

static int eng_set_ctl(oscar_engine *e, const std::vector<std::pair<int, SlotCtl>> &upd) {
  Launch L;
  L.slots = e->d_slots;
  L.btab = e->d_btab;
  L.nblocks = 0;
  L.nslots = e->max_slots;
  L.stream = e->stream;
  for (size_t i = 0; i < upd.size(); i += CtlUpdate::MAXN) {
    CtlUpdate u;
    memset(&u, 0, sizeof u);
    u.n = 0;
    for (size_t j = i; j < upd.size() && u.n < CtlUpdate::MAXN; ++j) {
      u.slot[u.n] = upd[j].first;
      u.ctl[u.n] = upd[j].second;
      u.n++;
    }
    launch_ctl_update(L, u);
    EHIP(e, hipGetLastError());
  }
  return OSCAR_OK;
}

static int eng_read_states(oscar_engine *e) {
  Launch L;
  L.slots = e->d_slots;
  L.btab = e->d_btab;
  L.nblocks = 0;
  L.nslots = e->max_slots;
  L.stream = e->stream;
  launch_gather_states(L, e->max_slots, e->d_states);
  EHIP(e, hipGetLastError());
  EHIP(e, hipMemcpyAsync(e->h_states, e->d_states, sizeof(SlotState) * e->max_slots, hipMemcpyDeviceToHost, e->stream));
  const bool pq = e->solve_mode == OSCAR_SOLVE_PERSISTENT;
  if (pq) EHIP(e, hipMemcpyAsync(&e->h_pq, e->d_pq, sizeof(PQGlobal), hipMemcpyDeviceToHost, e->stream));
  EHIP(e, hipStreamSynchronize(e->stream));
  if (pq && e->h_pq.err) {
    e->err = "persistent pressure solve: no phase completed within its time limit";
    return OSCAR_E_HIP;
  }
  return OSCAR_OK;
}

// One persistent launch for the pressure solves of the listed slots (their
// set-up enqueued before it).
template <typename R>
static int eng_enqueue_pq(oscar_engine *e, const std::vector<int> &list, std::vector<int> &uploaded) {
  if (list.empty()) return OSCAR_OK;
  if (e->pq_idle == 0) {
    int dev = 0, khz = 0;
    EHIP(e, hipGetDevice(&dev));
    EHIP(e, hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    if (khz <= 0) { e->err = "device reports no wall-clock rate"; return OSCAR_E_HIP; }
    e->pq_idle = (long long)(PQ_IDLE_S * 1e3 * (double)khz);
  }
  int lds = 0, tiles = 0;
  for (int i : list) {
    const int l = pq_lds_for(e->slots[i].s);
    lds = l > lds ? l : lds;
    tiles += e->slots[i].g.nblocks;
  }
  int res = -1;
  for (const auto &x : e->pq_res)
    if (x.first == lds) res = x.second;
  if (res < 0) {
    res = pq_resident_wgs<R>(lds);
    e->pq_res.push_back({lds, res});
  }
  if (res < 1) { e->err = "sizing the persistent solve"; return OSCAR_E_HIP; }
  if (list != uploaded) {
    launch_pq_list(e->d_pq_list, list.data(), (int)list.size(), e->stream);
    uploaded = list;
  }
  const int n = (int)list.size();
  launch_pq_init(e->d_slots, e->d_pq_list, n, e->d_pq, e->stream);
  launch_pq_solve<R>(e->d_slots, e->d_pq_list, n, e->d_pq, res < tiles ? res : tiles, lds, e->pq_idle, e->stream);
  EHIP(e, hipGetLastError());
  return OSCAR_OK;
}

template <typename R>
static int eng_tick(oscar_engine *e) {
  // active slots and their block table
  std::vector<int> act;
  e->bt.clear();
  for (int i = 0; i < e->max_slots; ++i) {
    EngSlot &es = e->slots[i];
    if (es.state != ES_VD && es.state != ES_CR) continue;
    act.push_back(i);
    append_segment(e->bt, i, es.g.nblocks);
  }
  if (act.empty()) return OSCAR_OK;
  if ((int)e->bt.size() > e->btab_cap) { e->err = "block table overflow"; return OSCAR_E_CAPACITY; }
  EHIP(e, hipMemcpyAsync(e->d_btab, e->bt.data(), sizeof(int2) * e->bt.size(), hipMemcpyHostToDevice, e->stream));
  std::vector<std::pair<int, SlotCtl>> upd;
  for (int i : act) upd.push_back({i, eng_ctl(e->slots[i], e->slots[i].state == ES_CR ? 1 : 0, e->precision)});
  int rc = eng_set_ctl(e, upd);
  if (rc) return rc;
  Launch L;
  L.slots = e->d_slots;
  L.btab = e->d_btab;
  L.nblocks = (int)e->bt.size();
  L.nslots = e->max_slots;
  L.stream = e->stream;
  launch_state_reset(L, e->max_slots);
  launch_zero_usum<R>(L);
  launch_copy_phi_prev<R>(L);
  launch_normals<R>(L, false);
  int npass = 1;
  for (int i : act) npass = std::max(npass, e->slots[i].s.mules_iter);
  launch_advect<R>(L, npass);
  launch_normals<R>(L, true);
  launch_assemble<R>(L);
  EHIP(e, hipGetLastError());
  const bool mixed = e->precision == OSCAR_MIXED;
  // correctors: each slot runs its own n_corr; a slot whose correctors are
  // done sits out the later ones (its control block inactive)
  int n_corr = 1;
  for (int i : act) n_corr = std::max(n_corr, (int)e->slots[i].D.n_corr);
  // The pressure solves run per preconditioner: the Jacobi slots and the
  // multigrid slots, each group with a block table of its own when both are
  // present (every other launch covers all active slots).
  std::vector<int> gj, gm;
  for (int i : act) (e->slots[i].D.precond == OSCAR_PC_MG ? gm : gj).push_back(i);
  Launch Lj = L, Lm = L;
  if (!gj.empty() && !gm.empty()) {
    e->bt_j.clear();
    e->bt_m.clear();
    for (int i : gj) append_segment(e->bt_j, i, e->slots[i].g.nblocks);
    for (int i : gm) append_segment(e->bt_m, i, e->slots[i].g.nblocks);
    EHIP(e, hipMemcpyAsync(e->d_btab_j, e->bt_j.data(), sizeof(int2) * e->bt_j.size(), hipMemcpyHostToDevice, e->stream));
    EHIP(e, hipMemcpyAsync(e->d_btab_m, e->bt_m.data(), sizeof(int2) * e->bt_m.size(), hipMemcpyHostToDevice, e->stream));
    Lj.btab = e->d_btab_j;
    Lj.nblocks = (int)e->bt_j.size();
    Lm.btab = e->d_btab_m;
    Lm.nblocks = (int)e->bt_m.size();
  }
  MGBatch B;
  if (!gm.empty()) {
    B.slots = e->d_slots;
    B.btab = Lm.btab;
    B.nblocks = Lm.nblocks;
    B.stream = e->stream;
    // the slots whose hierarchy is rebuilt this tick (the rule of a context)
    MGBatch Bs = B;
    e->act_m.assign(4 * (size_t)e->max_slots, 0);
    bool any_setup = false;
    for (int di = 0; di < 2; ++di) {
      std::vector<const Slot *> hs, hss;
      for (int i : gm)
        if (e->slots[i].D.dim == di + 2) {
          const EngSlot &es = e->slots[i];
          e->act_m[(size_t)di * e->max_slots + hs.size()] = i;
          hs.push_back(&es.s);
          if (mg_rebuild(es.state == ES_CR, es.k)) {
            e->act_m[(size_t)(2 + di) * e->max_slots + hss.size()] = i;
            hss.push_back(&es.s);
          }
        }
      B.dim[di].act = e->d_act + (size_t)di * e->max_slots;
      mg_batch_levels(B.dim[di], hs.data(), (int)hs.size(), di + 2);
      Bs.dim[di].act = e->d_act + (size_t)(2 + di) * e->max_slots;
      mg_batch_levels(Bs.dim[di], hss.data(), (int)hss.size(), di + 2);
      any_setup = any_setup || !hss.empty();
    }
    EHIP(e, hipMemcpyAsync(e->d_act, e->act_m.data(), sizeof(int) * e->act_m.size(), hipMemcpyHostToDevice, e->stream));
    if (any_setup) launch_mg_setup_b<R>(Bs);   // coarse operators of this assembly's coefficients
    EHIP(e, hipGetLastError());
  }
  auto group_done = [&](const std::vector<int> &g) {
    for (int i : g)
      if (!e->h_states[i].done) return false;
    return true;
  };
  auto group_max_it = [&](const std::vector<int> &g) {
    int m = 0;
    for (int i : g) m = e->slots[i].D.pcg_max_it > m ? e->slots[i].D.pcg_max_it : m;
    return m;
  };
  auto group_pred = [&](const std::vector<int> &g) {
    int m = 1;
    for (int i : g) {
      const int p = mixed ? e->slots[i].pred_inner : e->slots[i].pred;
      m = p > m ? p : m;
    }
    return m;
  };
  auto record_pred = [&](const std::vector<int> &g, int floor_it) {
    for (int i : g) {
      const int used = e->h_states[i].it;
      int &p = mixed ? e->slots[i].pred_inner : e->slots[i].pred;
      p = used > floor_it ? used : floor_it;
    }
  };
  // one inner solve of the Jacobi group: chunks of single-launch iterations
  auto inner_j = [&]() -> int {
    launch_cg_init<R>(Lj);
    EHIP(e, hipGetLastError());
    int it0 = 0, chunk = group_pred(gj);
    chunk = chunk > 2 ? chunk : 2;
    const int max_it = group_max_it(gj);
    while (!group_done(gj)) {
      if (it0 > max_it + 1) { e->err = "conjugate gradient did not terminate"; return OSCAR_E_HIP; }
      launch_cg_iters<R>(Lj, it0, chunk);
      EHIP(e, hipGetLastError());
      it0 += chunk;
      int r2 = eng_read_states(e);
      if (r2) return r2;
      chunk = 8;
    }
    record_pred(gj, 2);
    return OSCAR_OK;
  };
  // The batch of the multigrid slots whose solve has not converged at the
  // last state read: a converged slot's launches would only return at once,
  // so its workgroups are left out of the tables once any slot is done.
  int n_live = -1;
  auto live_batch = [&](MGBatch &Bl) -> int {
    std::vector<int> live;
    for (int i : gm)
      if (!e->h_states[i].done) live.push_back(i);
    if ((int)live.size() == n_live) return OSCAR_OK;   // the same slots as the current table
    n_live = (int)live.size();
    if (live.size() == gm.size() || live.empty()) {
      Bl = B;
      return OSCAR_OK;
    }
    e->bt_live.clear();
    for (int i : live) append_segment(e->bt_live, i, e->slots[i].g.nblocks);
    EHIP(e, hipMemcpyAsync(e->d_btab_live, e->bt_live.data(), sizeof(int2) * e->bt_live.size(),
                           hipMemcpyHostToDevice, e->stream));
    Bl = B;
    Bl.btab = e->d_btab_live;
    Bl.nblocks = (int)e->bt_live.size();
    e->act_live.assign(2 * (size_t)e->max_slots, 0);
    for (int di = 0; di < 2; ++di) {
      std::vector<const Slot *> hs;
      for (int i : live)
        if (e->slots[i].D.dim == di + 2) {
          e->act_live[(size_t)di * e->max_slots + hs.size()] = i;
          hs.push_back(&e->slots[i].s);
        }
      Bl.dim[di].act = e->d_act + (size_t)(4 + di) * e->max_slots;
      mg_batch_levels(Bl.dim[di], hs.data(), (int)hs.size(), di + 2);
    }
    EHIP(e, hipMemcpyAsync(e->d_act + (size_t)4 * e->max_slots, e->act_live.data(), sizeof(int) * e->act_live.size(),
                           hipMemcpyHostToDevice, e->stream));
    return OSCAR_OK;
  };
  // one inner solve of the multigrid group: the initial cycle, then chunks
  // ending with a search-direction launch (the convergence test)
  auto inner_m = [&]() -> int {
    MGBatch Bl = B;
    n_live = -1;
    int r2 = live_batch(Bl);
    if (r2) return r2;
    for (int part = 0; part < 3; ++part) launch_mg_cycle_part_b<R>(Bl, -1, part);
    EHIP(e, hipGetLastError());
    int next = 0;
    bool tail = false;
    int chunk = group_pred(gm) + 1;
    const int max_it = group_max_it(gm);
    while (!group_done(gm)) {
      if (next > max_it + 1) { e->err = "conjugate gradient did not terminate"; return OSCAR_E_HIP; }
      for (int x = 0; x < chunk; ++x) {
        if (tail)
          for (int part = 0; part < 3; ++part) launch_mg_cycle_part_b<R>(Bl, next - 1, part);
        launch_mg_dir_b<R>(Bl, next);
        ++next;
        tail = true;
      }
      EHIP(e, hipGetLastError());
      r2 = eng_read_states(e);
      if (r2) return r2;
      r2 = live_batch(Bl);
      if (r2) return r2;
      chunk = 2;
    }
    record_pred(gm, 1);
    return OSCAR_OK;
  };
  auto solve_group = [&](const std::vector<int> &g, const Launch &Lg, bool mg) -> int {
    if (g.empty()) return OSCAR_OK;
    if (!mixed) return mg ? inner_m() : inner_j();
    // FP32 inner solves wrapped in FP64 refinement; the refinement acts on
    // the slots whose inner solve finished, and marks a slot done when it
    // met its tolerance or stalled (the rule of a context, on the device)
    for (int outer = 0; !group_done(g); ++outer) {
      if (outer > REFINE_MAX) { e->err = "refinement did not terminate"; return OSCAR_E_HIP; }
      int r2 = mg ? inner_m() : inner_j();
      if (r2) return r2;
      launch_refine<R>(Lg);
      EHIP(e, hipGetLastError());
      r2 = eng_read_states(e);
      if (r2) return r2;
    }
    for (int i : g)
      if (e->h_states[i].stalled) e->slots[i].stalled = true;
    return OSCAR_OK;
  };
  std::vector<double> E(e->max_slots, 0.0);
  for (int i : act) e->slots[i].stalled = false;
  const bool pq = e->solve_mode == OSCAR_SOLVE_PERSISTENT;
  std::vector<int> pq_uploaded;
  const std::vector<int> gj_all = gj, gm_all = gm;
  bool parked = false;   // some slot's control block is inactive for the later correctors
  for (int j = 0; j < n_corr; ++j) {
    if (j > 0) {   // slots whose correctors are done sit out
      std::vector<std::pair<int, SlotCtl>> park;
      for (int i : act)
        if (e->slots[i].D.n_corr == j) {
          SlotCtl k = eng_ctl(e->slots[i], e->slots[i].state == ES_CR ? 1 : 0, e->precision);
          k.active = 0;
          park.push_back({i, k});
        }
      if (!park.empty()) {
        rc = eng_set_ctl(e, park);
        if (rc) return rc;
        parked = true;
        gj.clear();
        gm.clear();
        for (int i : gj_all)
          if (e->slots[i].D.n_corr > j) gj.push_back(i);
        for (int i : gm_all)
          if (e->slots[i].D.n_corr > j) gm.push_back(i);
      }
    }
    launch_predictor<R>(L);
    launch_pressure_setup<R>(L, j == 0);
    EHIP(e, hipGetLastError());
    if (pq) {   // every slot's solve in one launch; the state is read once, after the tick
      std::vector<int> list = gj;
      list.insert(list.end(), gm.begin(), gm.end());
      rc = eng_enqueue_pq<R>(e, list, pq_uploaded);
      if (rc) return rc;
    } else {
      rc = eng_read_states(e);
      if (rc) return rc;
      rc = solve_group(gj, Lj, false);
      if (rc) return rc;
      rc = solve_group(gm, Lm, true);
      if (rc) return rc;
      if (j == 0)
        for (int i : act) E[i] = e->h_states[i].E;
    }
    launch_correct<R>(L, j);
    EHIP(e, hipGetLastError());
  }
  if (parked) {   // active again for the finalisation
    rc = eng_set_ctl(e, upd);
    if (rc) return rc;
  }
  rc = eng_read_states(e);
  if (rc) return rc;
  if (pq)
    for (int i : act) {
      E[i] = e->h_states[i].E;
      e->slots[i].stalled = e->h_states[i].stall_hits != 0;
    }
  // state transitions; finishing relaxations are finalised with their own table
  e->bt2.clear();
  std::vector<std::pair<int, SlotCtl>> off;
  for (int i : act) {
    EngSlot &es = e->slots[i];
    const SlotState &st = e->h_states[i];
    e->cg_iters += st.total_it;
    if (st.nonfinite) es.status = OSCAR_E_NONFINITE;
    else if (st.unstable && es.status == OSCAR_OK) es.status = OSCAR_E_UNSTABLE;
    else if (st.maxit_hit && es.status == OSCAR_OK) es.status = OSCAR_W_PCG_MAXIT;
    else if (es.stalled && es.status == OSCAR_OK) es.status = OSCAR_W_REFINE_STALL;
    if (es.state == ES_VD) {
      es.state = ES_CR;
      es.k = 0;
      if (es.status < 0) {
        es.state = ES_DONE;
        off.push_back({i, SlotCtl()});
      }
      continue;
    }
    es.last_E = E[i];
    bool stop = E[i] < es.tol || es.k + 1 >= es.max_iters || es.status < 0;
    if (!stop) {
      es.k++;
      continue;
    }
    es.k_f = es.k + 1;
    es.state = ES_DONE;
    off.push_back({i, SlotCtl()});
    append_segment(e->bt2, i, es.g.nblocks);
  }
  if (!e->bt2.empty()) {
    EHIP(e, hipMemcpyAsync(e->d_btab2, e->bt2.data(), sizeof(int2) * e->bt2.size(), hipMemcpyHostToDevice, e->stream));
    Launch F = L;
    F.btab = e->d_btab2;
    F.nblocks = (int)e->bt2.size();
    launch_finalize<R>(F);
    EHIP(e, hipGetLastError());
  }
  if (!off.empty()) {
    rc = eng_set_ctl(e, off);
    if (rc) return rc;
  }
  EHIP(e, hipStreamSynchronize(e->stream));
  e->ticks++;
  return OSCAR_OK;
}

extern "C" int32_t oscar_engine_run(oscar_engine *e, int32_t ticks) {
  if (!e || ticks < 1) return OSCAR_E_ARG;
  for (int t = 0; t < ticks; ++t) {
    int rc = e->precision == OSCAR_MIXED ? eng_tick<float>(e) : eng_tick<double>(e);
    if (rc) return rc;
  }
  return OSCAR_OK;
}

extern "C" int32_t oscar_engine_poll(const oscar_engine *e, int32_t *done_slots, int32_t cap, int32_t *n_done,
                                     int32_t *n_active) {
  if (!e || (!done_slots && cap > 0)) return OSCAR_E_ARG;
  int n = 0, a = 0;
  for (int i = 0; i < e->max_slots; ++i) {
    int st = e->slots[i].state;
    if (st == ES_DONE && n < cap) done_slots[n++] = i;
    if (st == ES_VD || st == ES_CR) a++;
  }
  if (n_done) *n_done = n;
  if (n_active) *n_active = a;
  return OSCAR_OK;
}

extern "C" int32_t oscar_engine_fetch(oscar_engine *e, int32_t slot, double *alpha, double *p, double *U,
                                      int32_t *k_f, int32_t *status) {
  if (!e || slot < 0 || slot >= e->max_slots) return OSCAR_E_ARG;
  EngSlot &es = e->slots[slot];
  if (es.state != ES_DONE) { e->err = "slot has no finished request"; return OSCAR_E_ARG; }
  const int64_t nc = es.g.nc, dn = es.g.d * es.g.nc;
  const bool mixed = e->precision == OSCAR_MIXED;
  auto get = [&](void *src, double *dst, int64_t len, bool dbl) -> int {
    if (!dst) return OSCAR_OK;
    if (dbl || !mixed) {
      EHIP(e, hipMemcpyAsync(dst, src, 8 * len, hipMemcpyDeviceToHost, e->stream));
      EHIP(e, hipStreamSynchronize(e->stream));
    } else {
      std::vector<float> t(len);
      EHIP(e, hipMemcpyAsync(t.data(), src, 4 * len, hipMemcpyDeviceToHost, e->stream));
      EHIP(e, hipStreamSynchronize(e->stream));
      for (int64_t x = 0; x < len; ++x) dst[x] = t[x];
    }
    return OSCAR_OK;
  };
  int rc = get(es.s.alpha, alpha, nc, false);
  if (!rc) rc = get(es.s.p, p, nc, true);
  if (!rc) rc = get(es.s.U, U, dn, false);
  if (k_f) *k_f = es.k_f;
  if (status) *status = es.status;
  return rc;
}

extern "C" int32_t oscar_engine_release(oscar_engine *e, int32_t slot) {
  if (!e || slot < 0 || slot >= e->max_slots) return OSCAR_E_ARG;
  EngSlot &es = e->slots[slot];
  if (es.state == ES_FREE) return OSCAR_OK;
  if (es.state == ES_VD || es.state == ES_CR) {
    std::vector<std::pair<int, SlotCtl>> off{{slot, SlotCtl()}};
    int rc = eng_set_ctl(e, off);
    if (rc) return rc;
  }
  // clear the table entry (its pointers would reach into memory that the
  // next admission may reuse) before the region goes back to the free list
  EHIP(e, hipMemsetAsync(e->d_slots + slot, 0, sizeof(Slot), e->stream));
  EHIP(e, hipStreamSynchronize(e->stream));
  eng_free(e, es.off, es.bytes);
  es = EngSlot();
  return OSCAR_OK;
}

extern "C" int32_t oscar_engine_stats(const oscar_engine *e, int64_t *ticks, int64_t *cg_iters) {
  if (!e) return OSCAR_E_ARG;
  if (ticks) *ticks = e->ticks;
  if (cg_iters) *cg_iters = e->cg_iters;
  return OSCAR_OK;
}
