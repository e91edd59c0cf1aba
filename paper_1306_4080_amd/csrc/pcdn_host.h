// Host-side state of a PCDN context and the internal driver functions shared
// by the single-problem entry points (pcdn_api.hip) and the multi-problem
// drivers (pcdn_batch.hip).  Not part of the public ABI.
#pragma once

#include <chrono>
#include <string>
#include <vector>

#include "../../include/pcdn.h"
#include "pcdn_device.h"

namespace pcdn {
namespace host {

// sweep, split scatter, line search, apply, stopping sweep, single-workgroup bundles
constexpr int kProfClasses = 6;

struct Profiler {
  int mask = 0;
  std::vector<hipEvent_t> pool;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pending;
  double ms[kProfClasses] = {};
  int64_t launches[kProfClasses] = {};
};

template <class T>
hipError_t dalloc(T** p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  return hipMalloc((void**)p, count * sizeof(T));
}

}  // namespace host
}  // namespace pcdn

using pcdn::IterState;
using pcdn::Stats;
using pcdn::StepState;

struct pcdn_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string err;

  // data
  int64_t n = 0, p = 0, nnz = 0;
  bool loaded = false;
  uint64_t data_hash = 0;  // fingerprint of the loaded X and y (data_fingerprint)
  int64_t* cp = nullptr;
  int32_t* ri = nullptr;
  float* v = nullptr;
  int8_t* y = nullptr;

  // state
  int loss = -1;
  double C = 0.0;
  // regulariser of the state: the one the last solve, iteration or step ran
  // with (pcdn_reset: eq. (1)); pcdn_evaluate reports F with it
  int penalty = 0;
  double l2 = 0.0;
  bool has_state = false;
  double* w = nullptr;
  double* cache = nullptr;
  double2* rw = nullptr;         // per-row term weights, kept with cache
  double* dtx = nullptr;  // single-workgroup kernel's fixed-point d^T x (bundles of many rows)
  double* tmp_n = nullptr;
  double* tmp_p = nullptr;
  double* g = nullptr;
  double* h = nullptr;
  double* d = nullptr;
  double* dterm = nullptr;

  // partition and chunk bookkeeping
  uint32_t* keys0 = nullptr;
  uint32_t* keys1 = nullptr;
  int32_t* idx0 = nullptr;
  int32_t* idx1 = nullptr;
  int32_t* hist = nullptr;
  int32_t* scan_tmp = nullptr;
  int32_t* nch = nullptr;
  int32_t* rfirst = nullptr;     // copy into partition order: slot of each range's first position
  int32_t* srow = nullptr;       // stopping-sweep tiles: each tile's nonzeros in row order
  uint16_t* spos = nullptr;      //   and their positions in the tile (null: no tiles)
  int64_t* psrc = nullptr;       // first nonzero of each slot's column
  int32_t* step_perm = nullptr;
  double2* part = nullptr;
  int64_t part_len = 0;
  // X in partition order (single-workgroup schedule)
  int32_t* pri = nullptr;
  int32_t* pslot = nullptr;      // slot of each nonzero in partition order
  float* pv = nullptr;
  int64_t* poff = nullptr;
  int32_t* off32 = nullptr;
  uint16_t* plid = nullptr;  // bundle-local row ids of X in partition order
  int32_t* pR = nullptr;     // distinct rows per bundle (or -1)
  double* pw = nullptr;      // w in partition order (taken with the partition)
  // shrinking: active mask (1/0 per feature), reduction partials, and the
  // host's copy of the next iteration's active count and nonzeros
  double* act = nullptr;
  double* stop_part = nullptr;
  double p_active_h = 0.0, nnz_active_h = 0.0;
  unsigned long long range_seen = 0;  // Stats::range_leaves at the last range check
  // X in CSR order (warm-start margins, and the source of the bundle-row
  // order): row pointers, and per nonzero its row, column and value
  int64_t* rp = nullptr;
  int32_t* ccol = nullptr;  // column of each nonzero in CSC order (stopping sweep)
  int32_t* rr = nullptr;
  int32_t* rc = nullptr;
  float* rv = nullptr;
  // multi-kernel schedule: X in bundle-row order for the current order
  // (br_*, with bt_* the sort's other buffer and br_hist its digit counts),
  // feature -> slot, and the touched rows of the current bundle per range
  int32_t* islot = nullptr;
  int32_t* br_row = nullptr;
  int32_t* br_slot = nullptr;
  float* br_val = nullptr;
  int32_t* bt_row = nullptr;
  int32_t* bt_slot = nullptr;
  float* bt_val = nullptr;
  int32_t* br_hist = nullptr;
  int32_t* u_cnt = nullptr;
  int32_t* u_row = nullptr;
  double* u_dtx = nullptr;
  // max_i sum_j |x_ij| (the single-workgroup kernel's fixed-point scale)
  double xrow = 0.0;

  // reductions and small device records
  double* ls_part = nullptr;
  IterState* iter = nullptr;
  StepState* st = nullptr;
  Stats* stats = nullptr;
  double* scal = nullptr;        // [0] stopping norm, [1] loss sum, [2] l1 sum, ...,
                                 // [kScalC] C
  double* sum_part = nullptr;

  // pinned host mirrors
  double* hscal = nullptr;
  Stats* hstats = nullptr;
  StepState* hst = nullptr;
  IterState* hiter = nullptr;

  // replayable outer iteration (HIP graph) and the key it was captured for
  hipGraphExec_t graph = nullptr;
  bool use_graphs = true;
  struct GraphKey {
    int64_t P = -1;
    int loss = -1;
    double sigma = 0, beta = 0, gamma = 0, nu = 0;
    int max_ls = 0;
    int schedule = -1;
    int shrink = -1;
    int penalty = -1;
    double l2 = 0;
    int chunk = 0;
    bool operator==(const GraphKey& o) const {
      return P == o.P && loss == o.loss && sigma == o.sigma && beta == o.beta &&
             gamma == o.gamma && nu == o.nu && max_ls == o.max_ls && schedule == o.schedule &&
             shrink == o.shrink && penalty == o.penalty && l2 == o.l2 && chunk == o.chunk;
    }
  } graph_key;
  // the same outer iteration in two parts around the bundles, for drivers
  // that run the bundles of several problems in one launch
  hipGraphExec_t graph_pre = nullptr;   // partition, chunking, partition-order copy of X
  hipGraphExec_t graph_post = nullptr;  // counters, stopping sweep (advances the iteration)
  GraphKey split_key;

  // counters known on the host (launch structure): sweep and stopping work
  // of every schedule (the single-workgroup kernel's share is counted on the
  // device, in Stats)
  struct HostCounts {
    double nnz_gh = 0, slots = 0, nnz_stop = 0, stop_sweeps = 0;
  } hc, prof_hc;
  std::vector<int64_t> h_cp;  // host copy of col_ptr
  // top_len[k]: nonzeros of the k longest columns (k <= kNarrowMaxP), an
  // upper bound on the nonzeros of any bundle of k features
  std::vector<int64_t> top_len;
  // heavy-bundle list of the current partition (device, and pinned host copy)
  int32_t* heavy = nullptr;
  int32_t* hheavy = nullptr;

  pcdn::host::Profiler prof;
  Stats prof_base{};
};

namespace pcdn {
namespace host {

// Record msg as ctx's last error and return code.
int fail(pcdn_ctx* c, int code, const std::string& msg);
// The calling thread's error record of the entry points without a context
// (pcdn_create, pcdn_solve_static), returned by pcdn_last_error(NULL).
std::string& global_error();

#define HIPCHK(ctx, expr)                                                              \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail((ctx), PCDN_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define ALLOC(ctx, ptr, count)                                                         \
  do {                                                                                 \
    if (dalloc(&(ptr), (size_t)(count)) != hipSuccess) {                               \
      (void)hipGetLastError();                                                         \
      return fail((ctx), PCDN_E_OOM, "device allocation failed for " #ptr);            \
    }                                                                                  \
  } while (0)

struct Opts {
  uint64_t seed;
  int max_outer, max_ls;
  double sigma, beta, gamma, nu;
  const double* w0;
  int schedule;
  int shrink;
  int penalty;  // PCDN_PENALTY_*
  double l2;
  int chunk;    // nonzeros per wavefront work item of the multi-kernel schedule
  // the regulariser sum_j ra |w_j| + (rb/2) w_j^2
  double ra() const { return penalty == PCDN_PENALTY_L2 ? 0.0 : 1.0; }
  double rb() const { return penalty == PCDN_PENALTY_L1 ? 0.0 : l2; }
};

// Options with defaults filled in and validated (o may be null).
int resolve_opts(pcdn_ctx* c, const pcdn_opts* o, Opts* r);
int check_loss(pcdn_ctx* c, int loss);
// The slot of the context's device scalars that holds C (the kernels read
// it there, so captured graphs do not depend on C).
constexpr int kScalC = 7;
int set_C(pcdn_ctx* c, double C);
uint64_t data_fingerprint(int64_t n, int64_t p, int64_t nnz, const int64_t* cp,
                          const int32_t* ri, const float* v, const int8_t* y);
// Record the regulariser that the state is being advanced with.
void note_regulariser(pcdn_ctx* c, const Opts& o);
// Whether outer iterations with bundle size P run in one workgroup.
bool use_narrow(const pcdn_ctx* c, const Opts& o, int64_t P);
// Whether the batch engine runs this single-workgroup job's bundles of at
// least kHeavyNnz nonzeros on the multi-kernel path (automatic schedule, and
// such bundles can exist).
bool use_hybrid(const pcdn_ctx* c, const Opts& o, int64_t P);
// Single-workgroup arguments for bundles [t_begin, t_end) of the current
// outer iteration's partition.
pcdn::NarrowArgs segment_narrow_args(pcdn_ctx* c, const Opts& o, int64_t P, int64_t t_begin,
                                     int64_t t_end);
// The multi-kernel bundle on slots [lo, hi) of the order perm (chunk
// descriptors and bundle-row order of that order already built).
int run_bundle(pcdn_ctx* c, const Opts& o, const int32_t* perm, int64_t lo, int64_t hi, bool clip,
               int64_t P);
// X in bundle-row order for bundles of P over the first p_slots slots of perm.
int build_bundle_rows(pcdn_ctx* c, const int32_t* perm, int64_t p_slots, int64_t P);
// Arguments of the single-workgroup kernel for bundles [t_begin, t_end).
pcdn::NarrowArgs make_narrow_args(pcdn_ctx* c, const Opts& o, const int32_t* perm,
                                  int64_t p_slots, int64_t P, int64_t t_begin, int64_t t_end,
                                  double* dtx_copy);
// ... for every bundle of the current outer iteration's partition.
pcdn::NarrowArgs outer_narrow_args(pcdn_ctx* c, const Opts& o, int64_t P);
// The kernels of one outer iteration (partition, every bundle, counters,
// stopping sweep) as tasks for the multi-problem executor, with the
// arguments and grids of the single-problem launches (the partition's scans
// in smaller blocks, with the same integer results); multi-kernel schedule
// only.
int outer_tasks(pcdn_ctx* c, const Opts& o, int64_t P, std::vector<pcdn::Task>& out);
// Capture (once per key) the two halves of an outer iteration around the
// single-workgroup bundles: graph_pre and graph_post (see pcdn_ctx).
int ensure_split_graphs(pcdn_ctx* c, const Opts& o, int64_t P);
// Capture (once per key) a whole outer iteration (graph).
int ensure_graph(pcdn_ctx* c, const Opts& o, int64_t P);
// Device bytes a context holding (n, p, nnz) allocates (admission estimate).
int64_t ctx_footprint_bytes(int64_t n, int64_t p, int64_t nnz);
// Host-known work of `count` outer iterations (sweep and stopping counters).
void count_outer(pcdn_ctx* c, const Opts& o, int64_t P, int64_t count);
// Set the device-side outer-iteration record (seed, k) read by graph replays.
int set_iter(pcdn_ctx* c, uint64_t seed, int64_t k);
int read_stats(pcdn_ctx* c);
// PCDN_E_NUMERIC with `what` if retained quantities left their range since
// the last check (Stats::range_leaves); range_check reads the counters first.
int range_check(pcdn_ctx* c, const char* what);
int range_noted(pcdn_ctx* c, const char* what);
constexpr const char* kRangeStep =
    "a step put e^{w^T x_i} outside the normal doubles (|w^T x_i| > ~708) or b_i outside the "
    "finite ones";
// Outer iterations k_first .. k_first+count-1 (graph replays unless profiling).
int run_outer(pcdn_ctx* c, const Opts& o, int64_t P, int64_t k_first, int64_t count);
// Copy c->scal[idx] to the host (synchronises the stream).
int read_scalar(pcdn_ctx* c, int idx, double* out);
// The scalars after an outer iteration (the stopping norm into *G; the next
// active count and nonzeros into the context's host copy).
int read_outer(pcdn_ctx* c, double* G);
// Shrinking state at the start of a solve: every feature active.
int init_shrink(pcdn_ctx* c);

// One pcdn_solve in progress: solve_begin validates nothing (callers do),
// computes the reference norm at w = 0 and sets up w; the caller runs outer
// iterations until `converged` or max_outer, then solve_end reports.
struct SolveRun {
  pcdn_ctx* c = nullptr;
  Opts o{};
  double C = 0.0, eps = 0.0;
  int64_t P = 0;
  int loss = 0;
  Stats base{};
  pcdn_ctx::HostCounts hbase{};
  double G0 = 0.0, G = 0.0;
  bool converged = false;
  int outer = 0;
  double min_stop_margin = 0.0;  // (set by solve_begin) smallest |G_k - eps G0| / (eps G0) so far
  bool w0_device = false;  // warm start from the w already on the device
  std::chrono::steady_clock::time_point t0;
};
// Validate the arguments of a solve (as pcdn_solve does).
int check_solve_args(pcdn_ctx* c, double C, int64_t P, double eps, int loss,
                     const pcdn_opts* opts, Opts* o);
int solve_begin(SolveRun& r);
// Record a finished outer iteration whose stopping norm is G.
int solve_note_outer(SolveRun& r, double G);
int solve_end(SolveRun& r, double* w_out, pcdn_info* info);

}  // namespace host
}  // namespace pcdn
