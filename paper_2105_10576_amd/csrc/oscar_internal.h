// Internal declarations of the OSCAR HIP library (gfx950).
//
// One "slot" is one OSCAR instance (one grid, its fields and its solver
// state).  Every kernel takes the device array of slots of a batch plus a
// block table that maps each workgroup to (slot, block within the slot), so a
// single launch advances every slot of a batch; a single instance is a batch
// of one.  All per-slot reductions go through per-block partials summed
// in a fixed order, so a slot's results do not depend on which other slots
// share the launch.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace oscar {

enum : int { F_NONE = 0, F_INT = 1, F_WALL = 2, F_INLET = 3, F_OUTLET = 4 };

constexpr int BLOCK = 256;   // threads per workgroup
constexpr int NVAL = 4;      // values per reduction channel

// Reduction channels: a producing kernel writes one partial per block and
// value at part[(ch*NVAL + m)*nblocks + block]; the consumer (the next
// kernel that needs the total, or a one-block-per-slot finaliser) sums the
// partials of its slot in a fixed order.  No atomics, no cache flushes.
// CH_CG0/CH_CG1: the CG reduction of iteration it goes to CH_CG0 + (it & 1)
// and is read by iteration it + 1, so no launch reads a channel it writes.
enum : int { CH_ADV1 = 0, CH_ADV2 = 1, CH_SETUP = 2, CH_NORM = 3, CH_CG0 = 4, CH_CG1 = 5, CH_REF = 6, CH_DQ = 7, NCH = 8 };

// Per-slot scalars written by one block (block 0 of a kernel, or a
// finaliser) and read by later kernels.
struct SlotState {
  double bn, rn, gam[2], alp[2];           // conjugate gradient (iteration-parity buffers)
  double pbar, E;                          // normalised residual
  double comax, mass0, mass1, bflux;       // transport
  double rn64, bn64, rn64_prev;            // refinement (mixed precision); rn64 before the last refinement
  double tgt;                              // absolute residual target of the FP32 inner solve
  double mass_defect;
  int32_t it, done, zero_rhs, total_it;
  int32_t nonfinite, unstable, maxit_hit, refine_steps;
  int32_t ref_solve;   // refinement steps of the current solve (reset by its set-up)
  int32_t stalled;     // the current solve's refinement stopped short of its tolerance
  int32_t stall_hits;  // solves whose refinement stalled since the last state reset
  int32_t solve_base;  // total_it when the current persistent solve started
  // persistent solve: the slot's open phase (generation << 32 | tiles << 16 |
  // tiles claimed), its kind, iteration and level, and its completed tiles
  unsigned long long pq_word;
  int32_t pq_phase, pq_it, pq_lvl, pq_done;
};

// Batch-wide words of one persistent solve launch.
struct PQGlobal {
  int32_t remaining;   // slots whose solve has not finished
  int32_t err;         // 1: no phase completed within the idle limit and the launch gave up
  uint32_t progress;   // phases completed so far (what waiting workgroups watch)
  int32_t pad;
};

// Mixed precision: a solve's FP64 refinement stops (done, stalled) when one
// outer step no longer halves the FP64 residual, or after REFINE_MAX steps:
// the tolerance then lies below what the FP32 inner solves can deliver.
constexpr int REFINE_MAX = 60;

struct SlotCtl {
  double dt, ub, rtol, rtol_inner;   // rtol_inner: smallest relative reduction asked of one FP32 inner solve
  int32_t active, mode, with_st, max_it;
  int32_t last_corr, substep, n_sub, pad;   // last_corr: n_corr - 1; substep: index within the relaxation
  double tol;
};

// Geometric multigrid hierarchy of the pressure matrix (preconditioner):
// every dimension halved (rounding up) per level until a level has at most
// MG_COARSEST cells (at most MG_MAXL levels); the coarsest level is solved
// with its dense inverse, so it may have at most MG_DENSE_MAX cells.  The
// levels from the first one with at most MG_TAIL_CELLS cells whose arrays
// fit MG_TAIL_LDS bytes (the tail) run in one workgroup out of LDS; their
// arrays form one contiguous block (mg_tail_bytes).
constexpr int MG_MAXL = 12;
constexpr int MG_COARSEST = 16;
constexpr int MG_TAIL_CELLS = 2048;
constexpr int MG_DENSE_MAX = 64;
constexpr int MG_TAIL_LDS = 160 * 1024;   // LDS of one gfx950 workgroup
// A grid-wide level of at least MG_SPLIT_MIN cells with two sweeps per side
// runs each sweep as a launch of its own (a context's launches; the
// engine's and the persistent solve's keep the fused kernels, with bitwise
// the same results).
constexpr int MG_SPLIT_MIN = 1 << 17;
struct MGLevel {
  int32_t nx, ny, nz, nc, nxy, nblocks;
  void *cf[3];        // coefficient of each cell's low face per direction (T)
  void *cout;         // outlet coefficient of the cell (T)
  void *invD;         // inverse diagonal (T, 0 for cells without fluid)
  void *b, *x, *t;    // right-hand side, pre-smoothed correction, final correction (T)
};
struct MGInfo {
  int32_t L;          // coarsest level (levels 1..L); 0 = no hierarchy
  int32_t tail;       // first level handled by the single-workgroup tail kernel
  int32_t nu2;        // bit l: grid-wide level l takes two smoothing sweeps per side (else one)
  MGLevel lv[MG_MAXL + 1];
  void *Ainv;         // dense inverse of the coarsest operator, row-major (T)
  void *tail_base;    // block of Ainv, per level tail..L cf[dim], cout, invD, the tail level's b, then the
                      // arrays the tail writes before it reads them: the other levels' b, every level's x and t
  int32_t tail_bytes; // its size (a multiple of 16)
  int32_t tail_load;  // bytes of the block that the tail reads before writing (a multiple of 16)
};

// bytes of the tail block when the tail starts at level l (elements of w bytes)
inline int64_t mg_tail_bytes(const MGInfo &mg, int l, int dim, int w) {
  int64_t n = (int64_t)mg.lv[mg.L].nc * mg.lv[mg.L].nc;
  for (int m = l; m <= mg.L; ++m) n += (int64_t)(dim + 5) * mg.lv[m].nc;
  return (n * w + 15) / 16 * 16;
}

struct Slot {
  int32_t dim, nx, ny, nz;
  int32_t nc, nf0, nf1, nf2, nftot, nxy;   // counts (the host keeps them below 2^31)
  int32_t block0, nblocks, n_fluid, precision;
  int32_t mules_iter;           // limiting passes of the alpha transport (>= 1)
  int32_t mg_pc;                // 1: multigrid-preconditioned CG, 0: Jacobi
  int32_t bcf[6];               // face type of each box side
  uint32_t outlet;              // bit f: box side f is an outlet (f < 2*dim)
  double h, V, S, Sh, S2h, hh, delta, cos_t, sin_t;
  double rho1, mu1, rho2, mu2, sigma, u_inlet;
  const uint8_t *flags;         // bit f: face f interior; bit 6: solid
  // fields (element type R = double in FP64 mode, float in mixed mode)
  void *alpha, *alpha_old, *U_vd, *U_cr, *U_sum, *U, *phi_vd, *phi_prev, *phi_cr;
  double *p_vd, *p_cr, *p;
  void *kappa, *nhatf, *grad, *gradU, *Fm, *aP, *rAU, *b, *HbyA, *FL, *Af, *Rp, *Rm;
  void *Af2;                    // unused antidiffusive flux between limiting passes (mules_iter > 1)
  // balanced-force face sums (pressure gradient against surface tension)
  // are formed in FP64 in both modes: predicted flux, right-hand side
  double *phiH, *rhs, *Mp, *r64;
  // conjugate-gradient vectors (element type T = R): residual r, w = A M^-1 r
  // and s = A p in ping-pong pairs, search direction p, FP32 correction e
  void *invD, *cr[2], *cw[2], *cs[2], *cp, *e;
  double *part;                 // NCH * NVAL * nblocks reduction partials
  MGInfo mg;
  SlotState *st;
  SlotCtl *ctl;
};

struct CtlUpdate {
  static constexpr int MAXN = 32;
  int32_t n;
  int32_t slot[MAXN];
  SlotCtl ctl[MAXN];
};

// host launchers (kernels.hip); all enqueue on `stream`
struct Launch {
  const Slot *slots;       // device
  const int2 *btab;        // device block table
  int nblocks;             // total blocks
  int nslots;              // slots in the table (per-slot finalisers use one block each)
  hipStream_t stream;
};

template <typename R> void launch_copy_phi_prev(const Launch &L);
template <typename R> void launch_normals(const Launch &L, bool curvature);
// npass: the largest mules_iter of the slots in the launch
template <typename R> void launch_advect(const Launch &L, int npass);
template <typename R> void launch_assemble(const Launch &L);
template <typename R> void launch_predictor(const Launch &L);
template <typename R> void launch_pressure_setup(const Launch &L, bool normres);
template <typename R> void launch_cg_init(const Launch &L);
// Measurement only: a launch given a non-null `ts` (TS_WORDS zeroed 64-bit
// words) leaves in ts[2b], ts[2b+1] the start and end of its workgroup b on
// the device's constant-rate wall clock; k_ts_span reduces such regions and
// zeroes those of the groups of `per` regions flagged in the bit mask
// `clear` (at most 64 groups).
constexpr int TS_WORDS = 2 * 1040;   // two words per workgroup, at most 1040 workgroups per launch
void launch_ts_span(unsigned long long *ts, int nregions, unsigned long long *out, int per, unsigned long long clear,
                    hipStream_t stream);
// n iterations from it0 (with ts: n = 1)
template <typename R> void launch_cg_iters(const Launch &L, int it0, int n, unsigned long long *ts = nullptr);
template <typename R> void launch_refine(const Launch &L);
// corr: the corrector's index; each slot's last corrector (ctl.last_corr)
// adds its velocity to the relaxation sum
template <typename R> void launch_correct(const Launch &L, int corr);
template <typename R> void launch_finalize(const Launch &L);
template <typename R> void launch_zero_usum(const Launch &L);
void launch_ctl_update(const Launch &L, const CtlUpdate &u);
void launch_state_reset(const Launch &L, int nslots);

// multigrid-preconditioned CG (single slot; mg.hip)
// (the multigrid kernels take the context's slot record by value: `hs`, the
// host copy, whose pointers are device addresses)
template <typename R> void launch_mg_setup(const Slot &hs, hipStream_t st);
// part 0: fine pre-smoothing with restriction (and the CG update of
// iteration it >= 0); part 1: the coarse levels; part 2: fine prolongation,
// post-smoothing and the next reduction; mode: that of the slot's control
// block (which pressure the FP64 update of part 0 acts on)
// (with ts: one TS_WORDS region per launch, launches of part 1 in
// consecutive regions; mg_part_launches gives their number)
template <typename R> void launch_mg_cycle_part(const Slot &hs, const Launch &L, int it, int part, int mode,
                                                unsigned long long *ts = nullptr);

// Batched multigrid launches over slots of the serving engine (host view):
// the device slot table, the fine-level block table of the batch's slots, and
// per dimension the device list of its slots with the largest workgroup count
// each level's launch needs over them.
struct MGBatch {
  const Slot *slots = nullptr;   // device slot table
  const int2 *btab = nullptr;    // fine-level block table of the batch's slots (device)
  int nblocks = 0;               // its entries
  hipStream_t stream = nullptr;
  struct Dim {
    const int *act = nullptr;    // device list of the slot indices of this dimension
    int n = 0;
    int maxL = 0;                // deepest coarsest level
    int maxtail = 0;             // latest tail start
    int tail_bytes = 0;          // largest tail block (LDS of the tail launch)
    int setup_b[MG_MAXL + 1];    // per level: workgroups per slot of the setup launch
    int smooth_b[MG_MAXL + 1];   // of the pre-smoothing launch (0: no slot runs it)
    int up_b[MG_MAXL + 1];       // of the prolongation launch
  } dim[2];                      // 2D, 3D
};
// fill one dimension's level figures from host copies of its slots
void mg_batch_levels(MGBatch::Dim &d, const Slot *const *hs, int n, int dim);
template <typename R> void launch_mg_setup_b(const MGBatch &B);
template <typename R> void launch_mg_dir_b(const MGBatch &B, int it);
// part as in launch_mg_cycle_part; the FP64 update reads each slot's mode
template <typename R> void launch_mg_cycle_part_b(const MGBatch &B, int it, int part);
inline bool mg_split(const Slot &hs, int l) { return ((hs.mg.nu2 >> l) & 1) && hs.mg.lv[l].nc >= MG_SPLIT_MIN; }
inline int mg_part_launches(const Slot &hs, int part) {
  if (part != 1) return 1;
  int n = 2 * (hs.mg.tail - 1) + 1;
  for (int l = 1; l < hs.mg.tail; ++l) n += mg_split(hs, l) ? 2 : 0;
  return n;
}
template <typename R> void launch_mg_dir(const Slot &hs, const Launch &L, int it, unsigned long long *ts = nullptr);
void launch_gather_states(const Launch &L, int nslots, SlotState *out);

// Persistent pressure solve (mg.hip): one launch runs the whole solve --
// every CG iteration, multigrid cycle and FP64 refinement step -- of the
// slots slots[list[k]] (slots[k] when list is null), k < n, whose set-up
// (and multigrid coarse operators) are enqueued before it.  pq_init readies
// each slot's first phase (none when the set-up found it solved) and the
// batch words g; pq_solve then runs with `wgs` workgroups and `lds` bytes of
// LDS for the multigrid tail (a larger tail block runs from global memory).
// idle_ticks: wall-clock ticks without a completed phase after which the
// launch gives up (g->err = 1) rather than wait further.
void launch_pq_init(const Slot *slots, const int *list, int n, PQGlobal *g, hipStream_t stream);
// copy a host list of n slot indices to dst (device) in stream order, by value
void launch_pq_list(int *dst, const int *host, int n, hipStream_t stream);
template <typename R>
void launch_pq_solve(const Slot *slots, const int *list, int n, PQGlobal *g, int wgs, int lds, long long idle_ticks,
                     hipStream_t stream);
// workgroups of one pq_solve launch that fit the device at once with `lds`
// bytes of dynamic LDS each
template <typename R> int pq_resident_wgs(int lds);

// blocks per slot: ceil(cells/BLOCK), capped at `cap` (0: MAX_BLOCKS;
// grid-stride beyond the cap)
constexpr int MAX_BLOCKS = 1024;
int blocks_for(int64_t nc, int cap);

}  // namespace oscar
