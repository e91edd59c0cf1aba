// Device-side declarations shared by the PCDN kernels and the host driver.
//
// Layout in HBM (per context):
//   X       : col_ptr int64[p+1], row_idx int32[nnz], val fp32[nnz], y int8[n]
//   state   : w fp64[p], cache fp64[n] (e^{w^T x_i} or b_i), dtx 8 bytes[n]
//             (the single-workgroup kernel's fixed-point d^T x when a bundle
//             has too many rows for LDS; all zero between inner iterations)
//   bundle  : perm int32[p] (slot -> feature), per-slot g, h, d, dterm fp64
//   order   : per outer iteration, X copied into partition order (pri, pv,
//             pslot: the nonzeros of slot r at [poff[r], poff[r+1])), built
//             by kPermW-position ranges of the output: rfirst int32[] = the
//             slot holding each range's first position, psrc int64[p] = the
//             first nonzero of each slot's column; and the same nonzeros in
//             bundle-row order (grouped by bundle, rows ascending).
//
// Synchronisation model: on gfx950 a device-scope fence or grid barrier costs
// far more than a kernel boundary, so every global dependency of the bundle
// sweep is a kernel boundary and no kernel waits on another block.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

namespace pcdn {

constexpr int kWave = 64;
constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kChunk = 256;    // nonzeros per wavefront range of the bundle sweep (default)
constexpr int kChunkMin = 64;  // smallest selectable (the partials are sized for it)
constexpr int kQMax = 32;      // line-search candidates evaluated per pass
constexpr int kQGroup = 4;     // candidates per line-search thread (grid y covers the rest)
constexpr int kSumGrid = 256;  // blocks of the first reduction level
constexpr int kLogistic = 0;
constexpr int kL2Svm = 1;

// Cumulative device-side counters (read back by the host at sync points).
// Data-dependent counters, updated by one thread per block (never per
// wavefront: same-address atomics from thousands of waves serialise).
struct Stats {
  unsigned long long bundles;        // inner iterations
  unsigned long long ls_steps;       // candidates tested (q + 1, or max_ls on failure)
  unsigned long long ls_fail;        // inner iterations without an accepted step
  unsigned long long nnz_scat_rows;  // nonzeros with d_j != 0 in the multi-kernel d^T x pass
  unsigned long long nnz_unused;
  unsigned long long rows_touched;   // rows with d^T x_i != 0, summed over bundles
  // counted by the single-workgroup kernel for its own bundles (the others
  // above count every bundle of any schedule)
  unsigned long long nnz_scat_narrow;      // nonzeros it scattered, columns of <= chunk
  unsigned long long rows_touched_narrow;  // part of rows_touched from it
  unsigned long long nnz_gh_narrow;        // bundle nonzeros it swept
  unsigned long long slots_narrow;         // bundle slots it processed
  unsigned long long nnz_scat_narrow_split;  // nonzeros it scattered, longer columns
  // smallest Armijo margin |dF - sigma Delta_q| / |sigma Delta_q| since the
  // last reset, as the bits of a non-negative double (their integer order
  // is the numeric order)
  unsigned long long min_margin_bits;
  // retained quantities set outside their range (see in_range)
  unsigned long long range_leaves;
  unsigned long long pad[3];
};

// Result of the line search of the current inner iteration.
struct StepState {
  double alpha;   // accepted beta^q (0 if none)
  double delta;   // Delta, eq. (7)
  double dF;      // objective change at the accepted q
  int32_t q;      // accepted q, -1 if none
  int32_t pad;
};

// Outer-iteration counter used by graph replays: the partition of iteration
// k is keyed by SplitMix64 output k of `seed`; the final reduction of every
// stopping sweep advances k.
struct IterState {
  uint64_t seed;
  int64_t k;
};

struct SweepArgs {
  const int32_t* ri;
  const float* v;
  const int8_t* y;
  const double* cache;
  const double2* rw;          // per-row term weights (row_weights of cache and y)
  const double* w;
  // X in partition order (bundle sweep): the nonzeros of slot r are
  // pri/pv/pslot[poff[r] .. poff[r+1]), pslot holding r; pw[r] = w[perm[r]]
  const int64_t* poff;
  const int32_t* pri;
  const float* pv;
  const int32_t* pslot;
  const double* pw;
  int64_t slot_lo, slot_hi;   // this launch covers slots [slot_lo, slot_hi)
  double* g;                  // per-slot outputs, indexed by the absolute slot
  double* h;
  double* d;
  double* dterm;              // g d + gamma h d^2 + R_j(w + d) - R_j(w)
  double* sg;                 // stopping mode: |grad^S_j F|
  double2* part;              // bundle sweep: the ranges' open-slot partials (2 per range)
  int32_t W;                  // bundle sweep: nonzeros per wavefront range (64 .. 512)
  double* dtx;                // d^T x accumulator
  Stats* stats;
  const double* Cp;           // C (device scalar: one captured graph serves every C)
  double gamma, nu;
  // regulariser R_j(u) = ra |u| + (rb/2) u^2 (eq. (1): ra = 1, rb = 0)
  double ra, rb;
  // shrinking (all nullable): bundle mode clips the slots to the first
  // *p_active; stopping mode writes act[j] = 1 if feature j stays active
  // (w_j != 0 or |g_j| >= *thr), else 0
  const double* p_active;
  double* act;
  const double* thr;
};

// Stopping sweep (full gradient, every feature) over X in column order, in
// ranges of kStopW nonzeros, one wavefront per range: a segmented wavefront
// scan keyed by column sums g_j of the columns that lie inside the range and
// finishes them; a column that crosses a range boundary leaves a partial
// (part[m].x: its part in range m when it began before m, part[m].y: when it
// begins in m and continues), and k_stop_finish completes those and the empty
// columns, adding the partials in range order.
constexpr int kStopW = 256;
constexpr int kStopTile = 16384;  // nonzeros per workgroup of the tiled stopping sweep
struct StopArgs {
  const int32_t* ri;
  const float* v;
  const int32_t* ccol;       // column of each nonzero
  const int64_t* cp;
  const int8_t* y;
  const double* cache;
  const double2* rw;         // per-row term weights (row_weights of cache and y)
  const double* w;           // nullable: treated as zero
  int64_t p, nnz;
  double* sg;                // |grad^S_j F|
  double* act;               // nullable (shrinking): next active mask, threshold *thr
  const double* thr;
  double2* part;             // per range
  const double* Cp;          // C (device scalar)
  double ra, rb;
  // nullable: per kStopTile tile of consecutive nonzeros, the tile's
  // nonzeros in row order (row, position in the tile)
  const int32_t* srow;
  const uint16_t* spos;
  double* gwc;               // with the tiles: n doubles of working storage (the rows'
  int64_t n;                 //   gradient weights, packed for the tiles' gathers)
};

// Multi-kernel bundle after the sweep: the bundle's nonzeros in row order
// (bundle-row order: bundles ascending, rows ascending inside a bundle,
// columns ascending inside a row) give d^T x_i of each touched row as one
// fixed-order sum, fused with the first line-search candidates; the apply
// then updates the touched rows.  The nonzeros of bundle t are split into
// ranges of kRangeW; range r owns the rows whose first nonzero lies in it
// and lists them (row, d^T x_i) at u_row/u_dtx[r kRangeW ...], u_cnt[r] of
// them, rows with d^T x_i = 0 left out.
constexpr int kRangeW = 256;
constexpr int kRowsGridMax = 2048;  // blocks of the d^T x / line-search launch (at most)
struct RowsArgs {
  const int32_t* br_row;     // bundle-row order: row, slot and value of each nonzero
  const int32_t* br_slot;
  const float* br_val;
  const int64_t* poff;       // slot -> first nonzero of the slot's bundle-row block
  int64_t slot_lo, slot_hi;  // this bundle
  const double* d;           // per-slot outputs of the sweep
  const double* dterm;
  double* w;
  const double* pw;          // w in partition order: w[perm[slot]] for this bundle's slots
                             // until its apply (only that apply changes them)
  const int32_t* perm;       // slot -> feature
  double* cache;
  double2* rw;               // per-row term weights, kept with cache
  const int8_t* y;
  int32_t* u_cnt;            // rows listed per range (u_cap entries; the d^T x launch
                             // zeroes those of its wavefronts that have no range)
  int64_t u_cap;
  int32_t* u_row;
  double* u_dtx;
  double* part;              // [v * G + block]: Q loss sums, Q regulariser sums, Delta, touched
                             // rows, nonzeros with d_j != 0, Q sums of |loss change|,
                             // Q sums of |regulariser change| (4Q + 3 rows)
  int32_t G;                 // blocks of the d^T x / line-search launch
  StepState* st;
  Stats* stats;
  const double* Cp;          // C (device scalar)
  double beta, ra, rb, sigma;
  int Q, max_ls;
  const double* p_active;    // nullable: slots clipped to the first *p_active
};

// One pass of the stable counting sort that puts X's nonzeros into
// bundle-row order: the key of a nonzero is its bundle (slot / P; a nonzero
// of a feature outside the order, slot -1, takes bundle nb), 8 bits per pass,
// least significant first.  Pass 0 reads the CSR copy (rows ascending,
// columns ascending in a row) with columns mapped through islot; later
// passes read the previous pass's output.
constexpr int kBrRounds = 8;
struct BrArgs {
  const int32_t* islot;      // pass 0: feature -> slot (-1: not in the order); else null
  const int32_t* srow;
  const int32_t* scol;       // pass 0: columns; later passes: slots
  const float* sval;
  int32_t* drow;
  int32_t* dslot;
  float* dval;
  int32_t* hist;             // [256][ntiles] digit counts, scanned between the passes
  int32_t* slot_out;         // pass 0 histogram: the slots, in source order
  int64_t m, ntiles, P;
  int32_t shift, nb;
};
struct SlotLenArgs {         // column length (and w) in slot order
  const int32_t* perm;
  const int64_t* cp;
  int64_t p;
  int32_t* len;
  const double* w;           // nullable: no copy of w
  double* pw;
  int64_t* src;              // nullable: first nonzero of the slot's column (cp[perm[r]])
  int32_t* islot;            // nullable: islot[perm[r]] = r
};
constexpr int kPermW = 256;  // output positions per wavefront of the copy into partition order
struct WidenArgs {
  const int32_t* in;
  int64_t m;
  int64_t* out;
  int32_t* rfirst;           // nullable: slot of each kPermW-range's first position
};
// X copied into partition order: pri/pv[poff[slot] + e] = nonzero e of the
// slot's column and, if pslot is not null, pslot = the slot.
struct PermuteArgs {
  const int32_t* ri;
  const float* v;
  const int64_t* src;        // slot -> first nonzero of its column
  const int64_t* poff;       // slot -> first output position (p + 1 entries)
  const int32_t* rfirst;     // range -> slot holding its first position
  int64_t p;                 // slots
  int32_t* pri;
  float* pv;
  int32_t* pslot;
};



// Stopping reduction with shrinking: sums ||grad^S F||_1 = sum sg, the
// largest violation M = max sg, and the next iteration's active count and
// nonzeros (sum act, sum act_j nnz_j); the final level writes scal[0] = the
// norm, scal[3] = M, scal[4] = 1 - M/n (the next threshold), scal[5] = the
// active count, scal[6] = their nonzeros, and advances it->k.
struct StopSumArgs {
  const double* sg;
  const double* act;
  const int64_t* cp;
  int64_t p, n;
  double* part;              // 4 partials per block of the first level
  double* scal;
  IterState* it;
  int32_t nb;
  double ra;                 // L1 weight of the regulariser (threshold ra - M/n)
};

struct SumArgs {
  const double* x;
  int64_t m;
  double* part;              // one partial per block of the first level
  double* out;
  IterState* it;             // nullable: advanced by the final level
  int32_t nb;                // blocks of the first level
};

// Partition kernels as executor tasks (the launches of launch_perm_keys and
// launch_radix_sort, one task per launch).
struct PermKeysArgs {
  const IterState* it;
  uint64_t seed;
  int64_t k, p;
  const double* act;
  uint32_t* keys;
  int32_t* idx;
};
struct RadixArgs {          // one histogram or scatter pass
  const uint32_t* kin;
  const int32_t* iin;
  uint32_t* kout;
  int32_t* iout;
  int32_t* hist;            // digit offsets (scanned histogram)
  int64_t p, ntiles;
  int32_t shift;
};
struct ScanArgs {           // exclusive scan of in[0..m) into out (out[m] = total)
  const int32_t* in;
  int32_t* out;
  int32_t* tmp;             // block totals
  int64_t m, nb;
};

// One kernel invocation of one problem, as run by the multi-problem
// executor: the kernel, its arguments, and the grid a launch of its own
// would have (nblk blocks; the line search's grid is gx x nblk/gx).
enum TaskKind : int32_t {
  kTaskSweepRanges = 0,
  kTaskStopRanges,
  kTaskSweepFinish,
  kTaskStopFinish,
  kTaskRowsDtx,
  kTaskRowsApply,
  kTaskSumPartial,
  kTaskSumFinal,
  kTaskStopPartial,
  kTaskStopFinal,
  kTaskPermKeys,
  kTaskRadixHist,
  kTaskRadixScatter,
  kTaskScanSmall,
  kTaskScanBlocks,
  kTaskScanAdd,
  kTaskSlotLen,
  kTaskWiden,
  kTaskBrHist,
  kTaskBrScatter,
  kTaskPermute,
};
struct Task {
  int32_t kind;
  int32_t loss;
  int32_t nblk;
  int32_t gx;
  union {
    SweepArgs sw;
    StopArgs so;
    RowsArgs rw;
    BrArgs br;
    SlotLenArgs sl;
    WidenArgs wd;
    PermuteArgs pm;
    SumArgs sum;
    StopSumArgs stop;
    PermKeysArgs pk;
    RadixArgs rx;
    ScanArgs scan;
  } u;
};

// Single-workgroup schedule: bundles t_begin .. t_end-1 of one outer iteration
// (bundle t = slots [tP, min((t+1)P, p))), with X in partition order: the
// nonzeros of slot r are pri/pv[poff[r] .. poff[r+1]).  P <= kNarrowMaxP.
constexpr int kNarrowMaxP = 1024;
struct NarrowArgs {
  SweepArgs sw;        // ri/v unused; cache, y, g, h, d, dtx, C, gamma, nu used
  double* cache;       // the same arrays as sw.cache / sw.w, writable
  double2* rw;         // per-row term weights, kept with cache
  double* w;
  const int32_t* perm;
  const int64_t* poff; // p+1 partition-order offsets
  const int32_t* pri;
  const float* pv;
  const double* pw;    // w in partition order, taken with the partition (a bundle's
                       // features are updated only by that bundle)
  double2* part;       // global chunk partials when a bundle has > 32768 nonzeros
  int64_t n, p, P;
  int64_t t_begin, t_end;
  StepState* st;       // record of the last bundle
  Stats* stats;
  double* dtx_copy;    // nullable: receives d^T x of the (last) bundle
  double sigma, beta;
  int max_ls;
  int loss;            // kLogistic / kL2Svm (read by the multi-problem kernel)
  const double* p_active;  // nullable: bundles stop at ceil(*p_active / P)
  // bundle-local row ids (launch_bundle_rows; nullable: none): plid[k] is the
  // rank of nonzero k's row among the distinct rows of its bundle, pR[t] the
  // number of distinct rows of bundle t or -1 (more than kNarrowLidCap)
  const uint16_t* plid;
  const int32_t* pR;
  int32_t chunk;       // the multi-kernel chunk length (for the scatter counters)
  // max_i sum_j |x_ij| over X: with D = max_j |d_j| of a bundle, D * xrow
  // bounds every partial sum of d^T x_i, which sets the bundle's fixed-point
  // scale
  double xrow;
};

// Largest number of distinct rows of a bundle whose d^T x the
// single-workgroup kernel keeps in LDS.
constexpr int kNarrowLidCap = 4096;
// Bundle-local row ids are computed from a bitmap of the n rows in LDS:
// n <= 32 * kRowsMaxWords.
constexpr int64_t kRowsMaxWords = 7936;

// Bundles with at least kHeavyNnz nonzeros run on the multi-kernel path
// between single-workgroup segments (batch engine, automatic schedule); at
// most kHeavyCap of them per outer iteration are listed.  At kNarrowLidCap,
// every bundle left to the single workgroup keeps its d^T x in LDS.
constexpr int64_t kHeavyNnz = 4096;
constexpr int kHeavyCap = 256;

// ---- host-callable launchers (pcdn_kernels.hip) -------------------------
hipError_t launch_fill(double* a, double v, int64_t n, hipStream_t s);
// Bundle-local row ids of the bundles [tP, min((t+1)P, p_slots)) of X in
// partition order (poff, pri): see NarrowArgs.  Needs n <= 32 * kRowsMaxWords.
hipError_t launch_bundle_rows(const int64_t* poff, const int32_t* pri, int64_t p_slots, int64_t P,
                              int64_t n, uint16_t* plid, int32_t* pR, hipStream_t s);
// out[0] = number of bundles t (of P slots over p_slots) with at least
// `thresh` nonzeros in partition order (poff), capped at `cap`; out[1..] their
// indices in ascending order.  out holds cap + 1 entries.
hipError_t launch_heavy_bundles(const int64_t* poff, int64_t p_slots, int64_t P, int64_t thresh,
                                int32_t cap, int32_t* out, hipStream_t s);
// Keys of the partition of outer iteration it->k (or of the given k if it is
// null): upper 32 bits of SplitMix64 output j of the stream seeded with output
// k of the stream seeded with `seed`.
// act (nullable, shrinking): inactive features (act[j] == 0) take key
// 0xFFFFFFFF and active ones keep theirs capped at 0xFFFFFFFE, so the active
// features lead the order.
hipError_t launch_perm_keys(const IterState* it, uint64_t seed, int64_t k, int64_t p,
                            const double* act, uint32_t* keys, int32_t* idx, hipStream_t s);
// Stable LSD radix sort of (keys, idx) by the 32-bit keys; results end in keys0/idx0.
hipError_t launch_radix_sort(uint32_t* keys0, int32_t* idx0, uint32_t* keys1, int32_t* idx1,
                             int64_t p, int32_t* hist, int32_t* scan_tmp, hipStream_t s);
int64_t scan_tmp_ints(int64_t m);
int64_t radix_hist_ints(int64_t p);
// Exclusive scan of in[0..m) into out[0..m], out[m] = total (int32).
hipError_t launch_scan(const int32_t* in, int32_t* out, int64_t m, int32_t* tmp, hipStream_t s);
// The bundle sweep (X in partition order, ranges of a.W nonzeros) and
// its finish over the bundle's slots, with the grids they take for a bundle
// of `slots` slots and about `nnz_bundle` nonzeros.
int sweep_ranges_grid(double nnz_bundle, int W);
int sweep_finish_grid(int64_t slots);
hipError_t launch_sweep_ranges(int loss, const SweepArgs& a, int grid, hipStream_t s);
hipError_t launch_sweep_finish(int loss, const SweepArgs& a, hipStream_t s);
// The stopping sweep (both kernels) and the grids they take.
int stop_ranges_grid(int64_t nnz);
int stop_finish_grid(int64_t p);
hipError_t launch_stop_sweep(int loss, const StopArgs& a, hipStream_t s);
int sum_grid(int64_t m);
// Blocks of the d^T x / line-search launch for bundles of about `nnz_bundle`
// nonzeros (RowsArgs::G).
int rows_grid(double nnz_bundle);
// d^T x of the bundle's touched rows and the first kQGroup line-search
// candidates (a.G blocks); then the Armijo decision and the update.
hipError_t launch_rows_dtx(int loss, const RowsArgs& a, hipStream_t s);
hipError_t launch_rows_apply(int loss, const RowsArgs& a, hipStream_t s);
// X's nonzeros in bundle-row order for bundles of P over the order perm
// (p_slots slots; with p_slots < p the other features' nonzeros go last):
// poff (p_slots + 1) and the br arrays; tmp arrays and hist / scan_tmp as
// working storage (br_hist_ints(nnz) and scan_tmp_ints of it).
int br_passes(int64_t p_slots, int64_t P);
int64_t br_hist_ints(int64_t nnz);
// The same pass also copies X into partition order (pri, pv, pslot at poff;
// psrc and rfirst as working storage, p and nnz / kPermW + 1 entries) and w
// into slot order (pw).
struct BrPlan {
  const int32_t* perm;
  int64_t p, p_slots, P;
  const int64_t* cp;
  const int32_t* rr;     // the CSR copy of X
  const int32_t* rc;
  const float* rv;
  int64_t nnz;
  const int32_t* ri;     // X as loaded (CSC)
  const float* v;
  int64_t* psrc;
  int32_t* rfirst;
  const double* w;
  int32_t* islot;
  int32_t* len_tmp;
  int32_t* off32;
  int32_t* scan_tmp;
  int64_t* poff;
  int32_t* br_row;
  int32_t* br_slot;
  float* br_val;
  int32_t* bt_row;
  int32_t* bt_slot;
  float* bt_val;
  int32_t* hist;
  int32_t* pri;
  float* pv;
  int32_t* pslot;
  double* pw;
};
hipError_t launch_bundle_row_order(const BrPlan& b, hipStream_t s);
// The same as executor tasks (appended to out).
void bundle_row_tasks(int loss, const BrPlan& b, std::vector<Task>& out);
// dense[i] = d^T x_i of the touched rows listed by the last d^T x launch of
// the bundle [a.slot_lo, a.slot_hi) (dense must be zero elsewhere).
hipError_t launch_rows_scatter(const RowsArgs& a, double* dense, hipStream_t s);
hipError_t launch_narrow(int loss, const NarrowArgs& a, hipStream_t s);
// The partition of one outer iteration (launch_perm_keys and
// launch_radix_sort on the same buffers) as executor tasks, appended to out;
// the same permutation as those launches.
void partition_tasks(int loss, const IterState* it, uint64_t seed, int64_t p, const double* act,
                     uint32_t* keys0, int32_t* idx0, uint32_t* keys1, int32_t* idx1,
                     int32_t* hist, int32_t* scan_tmp, std::vector<Task>& out);
// Every task of tasks[0..count) in one launch of `blocks` blocks: task i
// takes blocks [first[i], first[i+1]) (first[count] = blocks).
hipError_t launch_exec(const Task* tasks, const int32_t* first, int count, int blocks,
                       hipStream_t s);
// dst[i] = *src[i] for i < count (device pointers).
hipError_t launch_gather(const double* const* src, double* dst, int count, hipStream_t s);
// One workgroup per entry of the device table tab[0..count) (each entry
// with its own loss).
hipError_t launch_narrow_multi(const NarrowArgs* tab, int count, hipStream_t s);
// X in partition order for the single-workgroup schedule (needs nnz < 2^31),
// and w in the same slot order (pw), over the first p slots of perm (their
// columns hold at most nnz nonzeros); psrc (p) and rfirst (nnz / kPermW + 1)
// are working storage.
hipError_t launch_permute(const int32_t* perm, const int64_t* cp, int64_t p, int64_t nnz,
                          const int32_t* ri, const float* v, int64_t* psrc, int32_t* rfirst,
                          int32_t* len_tmp, int32_t* off32, int32_t* scan_tmp, int64_t* poff,
                          int32_t* pri, float* pv, int32_t* pslot, const double* w, double* pw,
                          hipStream_t s);
// Deterministic two-kernel sum of x[0..m) into *out; optional: advance it->k.
hipError_t launch_sum(const double* x, int64_t m, double* part, double* out, IterState* it,
                      hipStream_t s);
// The stopping reduction with shrinking (see StopSumArgs); part holds
// 4 * sum_grid(p) doubles.
hipError_t launch_stop_sum(const StopSumArgs& a, hipStream_t s);
hipError_t launch_loss_terms(int loss, const double* cache, const int8_t* y, int64_t n,
                             double* out, hipStream_t s);
hipError_t launch_reg_terms(const double* w, int64_t p, double ra, double rb, double* out,
                            hipStream_t s);
// Retained quantities from w (e^{x_i^T w}, or 1 - y_i x_i^T w) with X in CSR
// order (rp int64[n+1], col, v); deterministic.
// Per-row weights of the gradient and Hessian-diagonal terms from the
// retained quantities and labels (after they are set in bulk).
hipError_t launch_row_weights(int loss, const double* cache, const int8_t* y, int64_t n,
                              double2* rw, hipStream_t s);
hipError_t launch_margins_rows(int loss, const int64_t* rp, const int32_t* col, const float* v,
                               const double* w, const int8_t* y, int64_t n, double* cache,
                               Stats* stats, hipStream_t s);
hipError_t launch_cache_from_z(int loss, double* z_to_cache, const int8_t* y, int64_t n,
                               hipStream_t s);

}  // namespace pcdn
