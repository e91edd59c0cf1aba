// C ABI of the PCDN library: context, data validation and upload, and the host
// driver of Algorithm 3 (outer loop over random partitions, inner loop over
// bundles).  All arithmetic of the method runs in the kernels of
// pcdn_kernels.hip; this file only sizes launches, orders them on the
// context's stream and reads back scalars.
#include <algorithm>
#include <functional>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "pcdn_host.h"

using namespace pcdn;

namespace {

// Algorithmic bytes per unit of work: what the method must move.
constexpr double kBytesPerNnzSweep = 17.0;    // row idx 4 + value 4 + retained gather 8 + label 1
constexpr double kBytesPerSlotSweep = 60.0;   // col_ptr pair 16 + perm 4 + w 8 + g,h,d,dterm 32
constexpr double kBytesPerNnzScatter = 24.0;  // row idx 4 + value 4 + FP64 read-modify-write 16
constexpr double kBytesPerRowLs = 17.0;       // d^T x 8 + retained 8 + label 1
constexpr double kBytesPerSlotLs = 28.0;      // perm 4 + w 8 + d 8 + dterm 8
constexpr double kBytesPerRowApply = 33.0;    // d^T x 8 + retained RMW 16 + label 1 + clear 8
constexpr double kBytesPerSlotApply = 28.0;   // perm 4 + d 8 + w RMW 16
// the single-workgroup kernel keeps a bundle's w, d and Delta terms in LDS:
// perm 4 + col_ptr pair 16 + w 8 + g, h, d out 24 + w write 8
constexpr double kBytesPerSlotNarrow = 60.0;
constexpr double kBytesPerNnzStop = 17.0;
constexpr double kBytesPerFeatStop = 32.0;    // col_ptr pair 16 + w 8 + |grad^S| 8

}  // namespace

namespace pcdn {
namespace host {

int fail(pcdn_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

void drop_graph(pcdn_ctx* c) {
  if (c->graph) (void)hipGraphExecDestroy(c->graph);
  c->graph = nullptr;
  c->graph_key = pcdn_ctx::GraphKey();
  if (c->graph_pre) (void)hipGraphExecDestroy(c->graph_pre);
  if (c->graph_post) (void)hipGraphExecDestroy(c->graph_post);
  c->graph_pre = c->graph_post = nullptr;
  c->split_key = pcdn_ctx::GraphKey();
}

template <class T>
void dfree(T*& ptr) {
  if (ptr) (void)hipFree((void*)ptr);
  ptr = nullptr;
}

void free_data(pcdn_ctx* c) {
  dfree(c->cp); dfree(c->ri); dfree(c->v); dfree(c->y);
  dfree(c->w); dfree(c->cache); dfree(c->rw); dfree(c->dtx); dfree(c->tmp_n); dfree(c->tmp_p);
  dfree(c->g); dfree(c->h); dfree(c->d); dfree(c->dterm);
  dfree(c->keys0); dfree(c->keys1); dfree(c->idx0); dfree(c->idx1);
  dfree(c->hist); dfree(c->scan_tmp); dfree(c->nch); dfree(c->rfirst); dfree(c->psrc); dfree(c->srow); dfree(c->spos);
  dfree(c->step_perm);
  dfree(c->ccol); dfree(c->rr); dfree(c->islot); dfree(c->br_row); dfree(c->br_slot); dfree(c->br_val);
  dfree(c->bt_row); dfree(c->bt_slot); dfree(c->bt_val); dfree(c->br_hist);
  dfree(c->u_cnt); dfree(c->u_row); dfree(c->u_dtx);
  dfree(c->part); dfree(c->ls_part);
  dfree(c->pri); dfree(c->pv); dfree(c->pslot); dfree(c->poff); dfree(c->off32); dfree(c->plid); dfree(c->pR);
  dfree(c->pw);
  dfree(c->rp); dfree(c->rc); dfree(c->rv);
  dfree(c->act);
  drop_graph(c);
  c->loaded = false;
  c->has_state = false;
  c->n = c->p = c->nnz = 0;
}

// Average nonzeros per bundle up to which one workgroup runs the bundles.
constexpr double kNarrowMaxBundleNnz = 8192.0;
// Nonzero positions are int32 in the partition and bundle-row orders.
constexpr int64_t kMaxNnz = ((int64_t)1 << 31) - ((int64_t)1 << 16);

int resolve_opts(pcdn_ctx* c, const pcdn_opts* o, Opts* r) {
  r->seed = o ? o->seed : 0;
  r->max_outer = (o && o->max_outer) ? o->max_outer : 1000;
  r->max_ls = (o && o->max_ls) ? o->max_ls : 30;
  r->sigma = (o && o->sigma != 0.0) ? o->sigma : 0.01;
  r->beta = (o && o->beta != 0.0) ? o->beta : 0.5;
  r->gamma = o ? o->gamma : 0.0;
  r->nu = (o && o->nu != 0.0) ? o->nu : 1e-12;
  r->w0 = o ? o->w0 : nullptr;
  r->schedule = o ? o->schedule : PCDN_SCHED_AUTO;
  if (r->schedule < PCDN_SCHED_AUTO || r->schedule > PCDN_SCHED_NARROW)
    return fail(c, PCDN_E_ARG, "unknown schedule");
  r->shrink = o ? o->shrink : 0;
  if (r->shrink != 0 && r->shrink != 1) return fail(c, PCDN_E_ARG, "shrink must be 0 or 1");
  r->chunk = (o && o->chunk) ? o->chunk : kChunk;
  if (r->chunk != 64 && r->chunk != 128 && r->chunk != 256 && r->chunk != 512)
    return fail(c, PCDN_E_ARG, "chunk must be 0, 64, 128, 256 or 512");
  r->penalty = o ? o->penalty : PCDN_PENALTY_L1;
  r->l2 = o ? o->l2 : 0.0;
  if (r->penalty < PCDN_PENALTY_L1 || r->penalty > PCDN_PENALTY_L2)
    return fail(c, PCDN_E_ARG, "unknown penalty");
  if (r->penalty == PCDN_PENALTY_L1 && r->l2 != 0.0)
    return fail(c, PCDN_E_ARG, "l2 must be 0 with the L1 penalty");
  if (r->penalty != PCDN_PENALTY_L1 && !(r->l2 > 0.0 && std::isfinite(r->l2)))
    return fail(c, PCDN_E_ARG, "l2 must be finite and > 0 for the elastic-net and ridge penalties");
  if (r->max_outer < 0) return fail(c, PCDN_E_ARG, "max_outer must be >= 0");
  if (r->max_ls < 1 || r->max_ls > kQMax) return fail(c, PCDN_E_ARG, "max_ls must lie in [1, 32]");
  if (!(r->sigma > 0.0 && r->sigma < 1.0)) return fail(c, PCDN_E_ARG, "sigma must lie in (0, 1)");
  if (!(r->beta > 0.0 && r->beta < 1.0)) return fail(c, PCDN_E_ARG, "beta must lie in (0, 1)");
  if (!(r->gamma >= 0.0 && r->gamma < 1.0)) return fail(c, PCDN_E_ARG, "gamma must lie in [0, 1)");
  if (!(r->nu > 0.0) || !std::isfinite(r->nu)) return fail(c, PCDN_E_ARG, "nu must be > 0");
  return PCDN_OK;
}

void note_regulariser(pcdn_ctx* c, const Opts& o) {
  c->penalty = o.penalty;
  c->l2 = o.l2;
}

int check_loss(pcdn_ctx* c, int loss) {
  if (loss != PCDN_LOSS_LOGISTIC && loss != PCDN_LOSS_L2SVM)
    return fail(c, PCDN_E_ARG, "unknown loss");
  return PCDN_OK;
}

// --- profiling -----------------------------------------------------------
hipEvent_t prof_event(pcdn_ctx* c) {
  if (!c->prof.pool.empty()) {
    hipEvent_t e = c->prof.pool.back();
    c->prof.pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Harvest finished event pairs (the stream has been synchronised).
void prof_harvest(pcdn_ctx* c) {
  for (auto& pe : c->prof.pending) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, pe.second.first, pe.second.second) == hipSuccess) {
      c->prof.ms[pe.first] += ms;
      c->prof.launches[pe.first] += 1;
    } else {
      (void)hipGetLastError();  // do not leave the failure for the next launch check
    }
    c->prof.pool.push_back(pe.second.first);
    c->prof.pool.push_back(pe.second.second);
  }
  c->prof.pending.clear();
}

struct ProfScope {
  pcdn_ctx* c;
  int cls;
  hipEvent_t a = nullptr, b = nullptr;
  ProfScope(pcdn_ctx* c_, int cls_) : c(c_), cls(cls_) {
    if (c->prof.mask & (1 << cls)) {
      if (c->prof.pending.size() > 8192) {
        (void)hipStreamSynchronize(c->stream);
        prof_harvest(c);
      }
      a = prof_event(c);
      b = prof_event(c);
      if (a && hipEventRecord(a, c->stream) != hipSuccess) {
        (void)hipGetLastError();
        a = nullptr;
      }
    }
  }
  ~ProfScope() {
    if (a && b) {
      (void)hipEventRecord(b, c->stream);
      c->prof.pending.push_back({cls, {a, b}});
    }
  }
};

// --- kernel sequences -------------------------------------------------------
SweepArgs sweep_args(pcdn_ctx* c, const Opts& o) {
  SweepArgs a{};
  a.ri = c->ri;
  a.v = c->v;
  a.y = c->y;
  a.cache = c->cache;
  a.rw = c->rw;
  a.w = c->w;
  a.g = c->g;
  a.h = c->h;
  a.d = c->d;
  a.dterm = c->dterm;
  a.W = o.chunk;
  a.sg = c->tmp_p;
  a.part = c->part;
  a.dtx = c->dtx;
  a.stats = c->stats;
  a.Cp = c->scal + kScalC;
  a.gamma = o.gamma;
  a.nu = o.nu;
  a.ra = o.ra();
  a.rb = o.rb();
  return a;
}

// Inner iteration of Algorithm 3 on slots [lo, hi) of the order X was copied
// into, first half: the sweep over the bundle's nonzeros (g_j, h_j partials
// per range) and its finish per slot (d_j and the Delta terms).
// clip: the bundle is one of an outer iteration with shrinking (its slots
// are clipped to the active count on the device)
SweepArgs bundle_sweep_args(pcdn_ctx* c, const Opts& o, int64_t lo, int64_t hi, bool clip) {
  SweepArgs a = sweep_args(c, o);
  a.poff = c->poff;
  a.pri = c->pri;
  a.pv = c->pv;
  a.pslot = c->pslot;
  a.pw = c->pw;
  a.slot_lo = lo;
  a.slot_hi = hi;
  a.p_active = clip ? c->scal + 5 : nullptr;
  return a;
}

// Blocks of a bundle sweep over slots [lo, hi) in ranges of W nonzeros:
// sized for the bundle's expected nonzeros.
int bundle_sweep_grid(const pcdn_ctx* c, int64_t lo, int64_t hi, int W) {
  return sweep_ranges_grid((double)c->nnz * (double)(hi - lo) / (double)c->p, W);
}

int bundle_sweep(pcdn_ctx* c, const Opts& o, int64_t lo, int64_t hi, bool clip) {
  const SweepArgs a = bundle_sweep_args(c, o, lo, hi, clip);
  {
    ProfScope ps(c, 0);
    HIPCHK(c, launch_sweep_ranges(c->loss, a, bundle_sweep_grid(c, lo, hi, a.W), c->stream));
  }
  {
    ProfScope ps(c, 1);
    HIPCHK(c, launch_sweep_finish(c->loss, a, c->stream));
  }
  return PCDN_OK;
}

// Second half: d^T x by row with the first line-search candidates, then the
// decision and the update.  With the first half, four kernel boundaries
// are the only synchronisation of a bundle.
RowsArgs rows_args(pcdn_ctx* c, const Opts& o, const int32_t* perm, int64_t lo, int64_t hi,
                   bool clip, int64_t P) {
  RowsArgs r{};
  r.br_row = c->br_row;
  r.br_slot = c->br_slot;
  r.br_val = c->br_val;
  r.poff = c->poff;
  r.slot_lo = lo;
  r.slot_hi = hi;
  r.d = c->d;
  r.dterm = c->dterm;
  r.w = c->w;
  r.pw = c->pw;
  r.perm = perm;
  r.cache = c->cache;
  r.rw = c->rw;
  r.y = c->y;
  r.u_cnt = c->u_cnt;
  r.u_cap = (c->nnz + kRangeW - 1) / kRangeW + 1;  // as allocated
  r.u_row = c->u_row;
  r.u_dtx = c->u_dtx;
  r.part = c->ls_part;
  r.G = rows_grid((double)c->nnz * (double)P / (double)c->p);
  r.st = c->st;
  r.stats = c->stats;
  r.beta = o.beta;
  r.ra = o.ra();
  r.rb = o.rb();
  r.Cp = c->scal + kScalC;
  r.sigma = o.sigma;
  r.Q = o.max_ls;
  r.max_ls = o.max_ls;
  r.p_active = clip ? c->scal + 5 : nullptr;
  return r;
}

int bundle_ls_apply(pcdn_ctx* c, const Opts& o, const int32_t* perm, int64_t lo, int64_t hi,
                    bool clip, int64_t P) {
  const RowsArgs r = rows_args(c, o, perm, lo, hi, clip, P);
  {
    ProfScope ps(c, 2);
    HIPCHK(c, launch_rows_dtx(c->loss, r, c->stream));
  }
  {
    ProfScope ps(c, 3);
    HIPCHK(c, launch_rows_apply(c->loss, r, c->stream));
  }
  return PCDN_OK;
}

int run_bundle(pcdn_ctx* c, const Opts& o, const int32_t* perm, int64_t lo, int64_t hi,
               bool clip, int64_t P) {
  int rc = bundle_sweep(c, o, lo, hi, clip);
  if (rc) return rc;
  return bundle_ls_apply(c, o, perm, lo, hi, clip, P);
}

// The bundle-row order and X in partition order for bundles of P over the
// order perm (p_slots slots).
BrPlan br_plan(pcdn_ctx* c, const int32_t* perm, int64_t p_slots, int64_t P) {
  BrPlan b{};
  b.perm = perm;
  b.p = c->p;
  b.p_slots = p_slots;
  b.P = P;
  b.cp = c->cp;
  b.rr = c->rr;
  b.rc = c->rc;
  b.rv = c->rv;
  b.nnz = c->nnz;
  b.ri = c->ri;
  b.v = c->v;
  b.psrc = c->psrc;
  b.rfirst = c->rfirst;
  b.w = c->w;
  b.islot = c->islot;
  b.len_tmp = c->nch;
  b.off32 = c->off32;
  b.scan_tmp = c->scan_tmp;
  b.poff = c->poff;
  b.br_row = c->br_row;
  b.br_slot = c->br_slot;
  b.br_val = c->br_val;
  b.bt_row = c->bt_row;
  b.bt_slot = c->bt_slot;
  b.bt_val = c->bt_val;
  b.hist = c->br_hist;
  b.pri = c->pri;
  b.pv = c->pv;
  b.pslot = c->pslot;
  b.pw = c->pw;
  return b;
}

int build_bundle_rows(pcdn_ctx* c, const int32_t* perm, int64_t p_slots, int64_t P) {
  HIPCHK(c, launch_bundle_row_order(br_plan(c, perm, p_slots, P), c->stream));
  return PCDN_OK;
}

// ||grad^S F(w)||_1 over all features into c->scal[0] (w == nullptr: w = 0);
// `it` (nullable) is advanced by the final reduction.
StopArgs stop_args(pcdn_ctx* c, const Opts& o, const double* w) {
  StopArgs a{};
  a.ri = c->ri;
  a.v = c->v;
  a.ccol = c->ccol;
  a.srow = c->srow;
  a.spos = c->spos;
  a.gwc = c->tmp_n;
  a.n = c->n;
  a.cp = c->cp;
  a.y = c->y;
  a.cache = c->cache;
  a.rw = c->rw;
  a.w = w;
  a.p = c->p;
  a.nnz = c->nnz;
  a.sg = c->tmp_p;
  a.part = c->part;
  a.Cp = c->scal + kScalC;
  a.ra = o.ra();
  a.rb = o.rb();
  return a;
}

int launch_stopping(pcdn_ctx* c, const Opts& o, const double* w, IterState* it) {
  const StopArgs a = stop_args(c, o, w);
  {
    ProfScope ps(c, 4);
    HIPCHK(c, launch_stop_sweep(c->loss, a, c->stream));
  }
  HIPCHK(c, launch_sum(c->tmp_p, c->p, c->sum_part, c->scal, it, c->stream));
  return PCDN_OK;
}

// Stopping sweep of an outer iteration with shrinking: the norm, the next
// active mask (threshold scal[4] of the previous iteration), the largest
// violation, the next threshold, active count and nonzeros (scal[0..6]).
int launch_stopping_shrink(pcdn_ctx* c, const Opts& o, IterState* it) {
  StopArgs a = stop_args(c, o, c->w);
  a.act = c->act;
  a.thr = c->scal + 4;
  {
    ProfScope ps(c, 4);
    HIPCHK(c, launch_stop_sweep(c->loss, a, c->stream));
  }
  const StopSumArgs s{c->tmp_p, c->act, c->cp, c->p, c->n, c->stop_part, c->scal, it,
                      sum_grid(c->p), o.ra()};
  HIPCHK(c, launch_stop_sum(s, c->stream));
  return PCDN_OK;
}

// Every feature active, threshold below any |g| (the first outer iterations).
int init_shrink(pcdn_ctx* c) {
  HIPCHK(c, launch_fill(c->act, 1.0, c->p, c->stream));
  HIPCHK(c, launch_fill(c->scal + 4, -1e300, 1, c->stream));
  HIPCHK(c, launch_fill(c->scal + 5, (double)c->p, 1, c->stream));
  HIPCHK(c, launch_fill(c->scal + 6, (double)c->nnz, 1, c->stream));
  c->p_active_h = (double)c->p;
  c->nnz_active_h = (double)c->nnz;
  return PCDN_OK;
}

// The scalars after an outer iteration: *G = the stopping norm; the host's
// copy of the next active count and nonzeros (shrinking) is refreshed.
int read_outer(pcdn_ctx* c, double* G) {
  HIPCHK(c, hipMemcpyAsync(c->hscal, c->scal, 8 * sizeof(double), hipMemcpyDeviceToHost,
                           c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (c->prof.mask) prof_harvest(c);
  *G = c->hscal[0];
  c->p_active_h = c->hscal[5];
  c->nnz_active_h = c->hscal[6];
  return PCDN_OK;
}

int read_scalar(pcdn_ctx* c, int idx, double* out) {
  HIPCHK(c, hipMemcpyAsync(c->hscal + idx, c->scal + idx, sizeof(double), hipMemcpyDeviceToHost,
                           c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (c->prof.mask) prof_harvest(c);
  *out = c->hscal[idx];
  return PCDN_OK;
}

int stopping_norm(pcdn_ctx* c, const Opts& o, const double* w, double* G) {
  int rc = launch_stopping(c, o, w, nullptr);
  if (rc) return rc;
  c->hc.nnz_stop += (double)c->nnz;
  c->hc.stop_sweeps += 1;
  return read_scalar(c, 0, G);
}

// F(w) = R(w) + C sum_i phi_i with the regulariser of o.
int objective(pcdn_ctx* c, const Opts& o, double* F) {
  HIPCHK(c, launch_loss_terms(c->loss, c->cache, c->y, c->n, c->tmp_n, c->stream));
  HIPCHK(c, launch_sum(c->tmp_n, c->n, c->sum_part, c->scal + 1, nullptr, c->stream));
  HIPCHK(c, launch_reg_terms(c->w, c->p, o.ra(), o.rb(), c->tmp_p, c->stream));
  HIPCHK(c, launch_sum(c->tmp_p, c->p, c->sum_part, c->scal + 2, nullptr, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->hscal + 1, c->scal + 1, 2 * sizeof(double), hipMemcpyDeviceToHost,
                           c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  *F = c->hscal[2] + c->C * c->hscal[1];
  return PCDN_OK;
}

// Retained quantities from w (device): z = X w, then e^z or 1 - y z.
int cache_from_w(pcdn_ctx* c, bool w_is_zero) {
  if (w_is_zero) {
    HIPCHK(c, launch_fill(c->cache, 1.0, c->n, c->stream));  // e^0 = 1, b = 1
    HIPCHK(c, launch_row_weights(c->loss, c->cache, c->y, c->n, c->rw, c->stream));
    return PCDN_OK;
  }
  HIPCHK(c, launch_margins_rows(c->loss, c->rp, c->rc, c->rv, c->w, c->y, c->n, c->cache,
                                c->stats, c->stream));
  HIPCHK(c, launch_row_weights(c->loss, c->cache, c->y, c->n, c->rw, c->stream));
  return range_check(c, "w puts e^{w^T x_i} outside the normal doubles (|w^T x_i| > ~708)");
}

// A 64-bit fingerprint of (n, p, nnz, X, y): 8-byte words mixed by
// multiply and xor-shift, to tell whether two contexts hold the same data.
uint64_t data_fingerprint(int64_t n, int64_t p, int64_t nnz, const int64_t* cp,
                          const int32_t* ri, const float* v, const int8_t* y) {
  uint64_t h = 0x243f6a8885a308d3ull;
  auto mix = [&h](uint64_t x) {
    h ^= x + 0x9e3779b97f4a7c15ull + (h << 6) + (h >> 2);
    h *= 0xff51afd7ed558ccdull;
    h ^= h >> 33;
  };
  auto bytes = [&mix](const void* a, size_t len) {
    const unsigned char* b = (const unsigned char*)a;
    size_t i = 0;
    for (; i + 8 <= len; i += 8) {
      uint64_t x;
      std::memcpy(&x, b + i, 8);
      mix(x);
    }
    uint64_t t = 0;
    std::memcpy(&t, b + i, len - i);
    mix(t ^ ((uint64_t)(len - i) << 56));
  };
  mix((uint64_t)n);
  mix((uint64_t)p);
  mix((uint64_t)nnz);
  bytes(cp, (size_t)(p + 1) * sizeof(int64_t));
  if (nnz) {
    bytes(ri, (size_t)nnz * sizeof(int32_t));
    bytes(v, (size_t)nnz * sizeof(float));
  }
  bytes(y, (size_t)n);
  return h;
}

// C on the host and in the device scalar the kernels read (scal[kScalC]).
int set_C(pcdn_ctx* c, double C) {
  c->C = C;
  HIPCHK(c, launch_fill(c->scal + kScalC, C, 1, c->stream));
  return PCDN_OK;
}

int set_w(pcdn_ctx* c, const double* w_host) {
  if (w_host) {
    for (int64_t j = 0; j < c->p; ++j)
      if (!std::isfinite(w_host[j])) return fail(c, PCDN_E_ARG, "w contains a non-finite value");
    HIPCHK(c, hipMemcpyAsync(c->w, w_host, c->p * sizeof(double), hipMemcpyHostToDevice,
                             c->stream));
  } else {
    HIPCHK(c, launch_fill(c->w, 0.0, c->p, c->stream));
  }
  return cache_from_w(c, w_host == nullptr);
}

// Partition of outer iteration k (it != null: k and seed read on the device).
int device_permutation(pcdn_ctx* c, uint64_t seed, int64_t k, const IterState* it,
                       const double* act = nullptr) {
  HIPCHK(c, launch_perm_keys(it, seed, k, c->p, act, c->keys0, c->idx0, c->stream));
  HIPCHK(c, launch_radix_sort(c->keys0, c->idx0, c->keys1, c->idx1, c->p, c->hist, c->scan_tmp,
                              c->stream));
  return PCDN_OK;
}


bool use_narrow(const pcdn_ctx* c, const Opts& o, int64_t P) {
  if (P > kNarrowMaxP || c->nnz >= ((int64_t)1 << 31)) return false;
  if (o.schedule == PCDN_SCHED_NARROW) return true;
  if (o.schedule == PCDN_SCHED_WIDE) return false;
  return (double)c->nnz * (double)P / (double)c->p <= kNarrowMaxBundleNnz;
}

bool use_hybrid(const pcdn_ctx* c, const Opts& o, int64_t P) {
  if (o.schedule != PCDN_SCHED_AUTO || !use_narrow(c, o, P) || c->top_len.empty()) return false;
  const int64_t k = std::min<int64_t>(P, (int64_t)c->top_len.size() - 1);
  return c->top_len[k] >= kHeavyNnz;
}

// Whether bundles of P over p_slots slots get local row ids (the
// single-workgroup kernel then keeps their d^T x in LDS): the row bitmap must
// fit LDS, and the per-bundle bitmap passes must stay cheap.
bool use_bundle_rows(const pcdn_ctx* c, int64_t P, int64_t p_slots) {
  const int64_t words = (c->n + 31) / 32;
  const int64_t bundles = (p_slots + P - 1) / P;
  return words <= kRowsMaxWords && (double)words * (double)bundles <= (double)(1 << 27);
}

// Bundles [t_begin, t_end) of size P over the order `perm` (p_slots slots)
// in one workgroup, after copying X into that order.
NarrowArgs make_narrow_args(pcdn_ctx* c, const Opts& o, const int32_t* perm, int64_t p_slots,
                            int64_t P, int64_t t_begin, int64_t t_end, double* dtx_copy) {
  NarrowArgs na{};
  na.sw = sweep_args(c, o);
  na.cache = c->cache;
  na.rw = c->rw;
  na.w = c->w;
  na.perm = perm;
  na.poff = c->poff;
  na.pri = c->pri;
  na.pv = c->pv;
  na.pw = c->pw;
  na.part = c->part;
  na.n = c->n;
  na.p = p_slots;
  na.P = P;
  na.t_begin = t_begin;
  na.t_end = t_end;
  na.st = c->st;
  na.stats = c->stats;
  na.sigma = o.sigma;
  na.beta = o.beta;
  na.max_ls = o.max_ls;
  na.dtx_copy = dtx_copy;
  na.loss = c->loss;
  na.chunk = o.chunk;
  na.xrow = c->xrow;
  if (use_bundle_rows(c, P, p_slots)) {
    na.plid = c->plid;
    na.pR = c->pR;
  }
  return na;
}

// Copy X into the order `perm` for bundles of P, with the bundles'
// local row ids where the single-workgroup kernel can use them.
int permute_x(pcdn_ctx* c, const int32_t* perm, int64_t p_slots, int64_t P) {
  HIPCHK(c, launch_permute(perm, c->cp, p_slots, c->nnz, c->ri, c->v, c->psrc, c->rfirst, c->nch,
                           c->off32, c->scan_tmp, c->poff, c->pri, c->pv, c->pslot, c->w, c->pw,
                           c->stream));
  if (use_bundle_rows(c, P, p_slots))
    HIPCHK(c, launch_bundle_rows(c->poff, c->pri, p_slots, P, c->n, c->plid, c->pR, c->stream));
  return PCDN_OK;
}

int launch_narrow_bundles(pcdn_ctx* c, const Opts& o, const int32_t* perm, int64_t p_slots,
                          int64_t P, int64_t t_begin, int64_t t_end, double* dtx_copy) {
  int rc = permute_x(c, perm, p_slots, P);
  if (rc) return rc;
  const NarrowArgs na = make_narrow_args(c, o, perm, p_slots, P, t_begin, t_end, dtx_copy);
  ProfScope ps(c, 5);
  HIPCHK(c, launch_narrow(c->loss, na, c->stream));
  return PCDN_OK;
}

// One outer iteration k of Algorithm 3: partition, every bundle, then the
// stopping sweep (result in c->scal[0]).  it != null: k is read from and
// advanced on the device (graph replays).
// The outer iteration in three parts.  Before the bundles: partition and X
// in partition order (with the bundle-row order on the multi-kernel path);
// heavy_list: also the list of heavy bundles, for the batch engine.
int enqueue_pre(pcdn_ctx* c, const Opts& o, int64_t P, int64_t k, IterState* it,
                bool heavy_list) {
  int rc = device_permutation(c, o.seed, k, it, o.shrink ? c->act : nullptr);
  if (rc) return rc;
  if (!use_narrow(c, o, P)) return build_bundle_rows(c, c->idx0, c->p, P);
  rc = permute_x(c, c->idx0, c->p, P);
  if (rc) return rc;
  if (heavy_list && use_hybrid(c, o, P)) {
    HIPCHK(c, launch_heavy_bundles(c->poff, c->p, P, kHeavyNnz, kHeavyCap, c->heavy, c->stream));
    // the heavy bundles run on the multi-kernel path
    rc = build_bundle_rows(c, c->idx0, c->p, P);
    if (rc) return rc;
  }
  return PCDN_OK;
}

// Single-workgroup arguments for every bundle of an outer iteration's
// partition (with shrinking, the kernel stops after the active features).
NarrowArgs outer_narrow_args(pcdn_ctx* c, const Opts& o, int64_t P) {
  return segment_narrow_args(c, o, P, 0, (c->p + P - 1) / P);
}

NarrowArgs segment_narrow_args(pcdn_ctx* c, const Opts& o, int64_t P, int64_t t_begin,
                               int64_t t_end) {
  NarrowArgs na = make_narrow_args(c, o, c->idx0, c->p, P, t_begin, t_end, nullptr);
  if (o.shrink) na.p_active = c->scal + 5;
  return na;
}

// Every bundle of the partition.
int enqueue_bundles(pcdn_ctx* c, const Opts& o, int64_t P) {
  const int64_t nb = (c->p + P - 1) / P;
  if (use_narrow(c, o, P)) {
    const NarrowArgs na = outer_narrow_args(c, o, P);
    ProfScope ps(c, 5);
    HIPCHK(c, launch_narrow(c->loss, na, c->stream));
    return PCDN_OK;
  }
  for (int64_t t = 0; t < nb; ++t) {
    const int64_t lo = t * P, hi = std::min(lo + P, c->p);
    int rc = run_bundle(c, o, c->idx0, lo, hi, o.shrink, P);
    if (rc) return rc;
  }
  return PCDN_OK;
}

// After the bundles: scatter counters and the stopping sweep.
int enqueue_post(pcdn_ctx* c, const Opts& o, int64_t P, IterState* it) {
  if (o.shrink) return launch_stopping_shrink(c, o, it);
  return launch_stopping(c, o, c->w, it);
}

// Every bundle with the heavy ones on the multi-kernel path (the list that
// enqueue_pre wrote is read back first: direct launches only).
int enqueue_bundles_hybrid(pcdn_ctx* c, const Opts& o, int64_t P) {
  HIPCHK(c, hipMemcpyAsync(c->hheavy, c->heavy, (kHeavyCap + 1) * sizeof(int32_t),
                           hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const int64_t nb = (c->p + P - 1) / P;
  const int32_t nh = std::min<int32_t>(std::max<int32_t>(c->hheavy[0], 0), kHeavyCap);
  int64_t t = 0;
  for (int32_t k = 0; k <= nh && t < nb; ++k) {
    const int64_t te = k < nh ? std::min<int64_t>(std::max<int64_t>(c->hheavy[1 + k], t), nb) : nb;
    if (te > t) {
      ProfScope ps(c, 5);
      HIPCHK(c, launch_narrow(c->loss, segment_narrow_args(c, o, P, t, te), c->stream));
    }
    t = te;
    if (k < nh && te < nb) {
      const int64_t lo = te * P, hi = std::min(lo + P, c->p);
      const int rc = run_bundle(c, o, c->idx0, lo, hi, o.shrink, P);
      if (rc) return rc;
      t = te + 1;
    }
  }
  return PCDN_OK;
}

int enqueue_outer(pcdn_ctx* c, const Opts& o, int64_t P, int64_t k, IterState* it) {
  // heavy bundles on the multi-kernel path only for direct launches (not
  // while a graph is captured, it != null)
  const bool hybrid = it == nullptr && use_hybrid(c, o, P);
  int rc = enqueue_pre(c, o, P, k, it, hybrid);
  if (rc) return rc;
  rc = hybrid ? enqueue_bundles_hybrid(c, o, P) : enqueue_bundles(c, o, P);
  if (rc) return rc;
  return enqueue_post(c, o, P, it);
}

int outer_tasks(pcdn_ctx* c, const Opts& o, int64_t P, std::vector<Task>& out) {
  if (use_narrow(c, o, P)) return fail(c, PCDN_E_ARG, "outer_tasks: single-workgroup schedule");
  out.clear();
  // the partition (enqueue_pre of the multi-kernel schedule)
  partition_tasks(c->loss, c->iter, o.seed, c->p, o.shrink ? c->act : nullptr, c->keys0, c->idx0,
                  c->keys1, c->idx1, c->hist, c->scan_tmp, out);
  auto task = [&](int kind, int nblk, int gx) {
    Task t;
    std::memset(&t, 0, sizeof(t));
    t.kind = kind;
    t.loss = c->loss;
    t.nblk = nblk;
    t.gx = gx;
    return t;
  };
  bundle_row_tasks(c->loss, br_plan(c, c->idx0, c->p, P), out);
  const int64_t nb = (c->p + P - 1) / P;
  for (int64_t b = 0; b < nb; ++b) {
    const int64_t lo = b * P, hi = std::min(lo + P, c->p);
    Task t = task(kTaskSweepRanges, bundle_sweep_grid(c, lo, hi, o.chunk), 0);
    t.u.sw = bundle_sweep_args(c, o, lo, hi, o.shrink);
    out.push_back(t);
    t.kind = kTaskSweepFinish;
    t.nblk = sweep_finish_grid(hi - lo);
    out.push_back(t);
    const RowsArgs r = rows_args(c, o, c->idx0, lo, hi, o.shrink, P);
    t = task(kTaskRowsDtx, r.G, 0);
    t.u.rw = r;
    out.push_back(t);
    t.kind = kTaskRowsApply;
    out.push_back(t);
  }
  Task t = task(kTaskStopRanges, stop_ranges_grid(c->nnz), 0);
  t.u.so = stop_args(c, o, c->w);
  if (o.shrink) {
    t.u.so.act = c->act;
    t.u.so.thr = c->scal + 4;
  }
  if (c->nnz > 0) out.push_back(t);
  t.kind = kTaskStopFinish;
  t.nblk = stop_finish_grid(c->p);
  out.push_back(t);
  const int sb = sum_grid(c->p);
  if (o.shrink) {
    t = task(kTaskStopPartial, sb, 0);
    t.u.stop = StopSumArgs{c->tmp_p, c->act, c->cp, c->p, c->n, c->stop_part, c->scal, c->iter, sb,
                           o.ra()};
    out.push_back(t);
    t.kind = kTaskStopFinal;
  } else {
    t = task(kTaskSumPartial, sb, 0);
    t.u.sum = SumArgs{c->tmp_p, c->p, c->sum_part, c->scal, c->iter, sb};
    out.push_back(t);
    t.kind = kTaskSumFinal;
  }
  t.nblk = 1;
  out.push_back(t);
  return PCDN_OK;
}

pcdn_ctx::GraphKey graph_key_of(const pcdn_ctx* c, const Opts& o, int64_t P) {
  pcdn_ctx::GraphKey key;
  key.P = P;
  key.loss = c->loss;
  key.sigma = o.sigma;
  key.beta = o.beta;
  key.gamma = o.gamma;
  key.nu = o.nu;
  key.max_ls = o.max_ls;
  key.schedule = o.schedule;
  key.shrink = o.shrink;
  key.penalty = o.penalty;
  key.l2 = o.l2;
  key.chunk = o.chunk;
  return key;
}

// Capture what `enqueue` puts on c's stream as an executable graph.
template <class F>
int capture(pcdn_ctx* c, hipGraphExec_t* out, F enqueue) {
  *out = nullptr;
  hipGraph_t g = nullptr;
  // relaxed: the capture neither restricts nor is restricted by what other
  // host threads do meanwhile (a server uploads requests on a thread of its
  // own while its caller's thread captures a new request's graphs)
  HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed));
  int rc = enqueue();
  hipError_t e = hipStreamEndCapture(c->stream, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return fail(c, PCDN_E_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
  e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    *out = nullptr;
    return fail(c, PCDN_E_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
  }
  return PCDN_OK;
}

int ensure_graph(pcdn_ctx* c, const Opts& o, int64_t P) {
  const pcdn_ctx::GraphKey key = graph_key_of(c, o, P);
  if (c->graph && c->graph_key == key) return PCDN_OK;
  if (c->graph) (void)hipGraphExecDestroy(c->graph);
  c->graph = nullptr;
  c->graph_key = pcdn_ctx::GraphKey();
  int rc = capture(c, &c->graph, [&] { return enqueue_outer(c, o, P, 0, c->iter); });
  if (rc) return rc;
  c->graph_key = key;
  return PCDN_OK;
}

int ensure_split_graphs(pcdn_ctx* c, const Opts& o, int64_t P) {
  const pcdn_ctx::GraphKey key = graph_key_of(c, o, P);
  if (c->graph_pre && c->graph_post && c->split_key == key) return PCDN_OK;
  if (c->graph_pre) (void)hipGraphExecDestroy(c->graph_pre);
  if (c->graph_post) (void)hipGraphExecDestroy(c->graph_post);
  c->graph_pre = c->graph_post = nullptr;
  c->split_key = pcdn_ctx::GraphKey();
  int rc = capture(c, &c->graph_pre, [&] { return enqueue_pre(c, o, P, 0, c->iter, true); });
  if (rc) return rc;
  rc = capture(c, &c->graph_post, [&] { return enqueue_post(c, o, P, c->iter); });
  if (rc) return rc;
  c->split_key = key;
  return PCDN_OK;
}

void count_outer(pcdn_ctx* c, const Opts& o, int64_t P, int64_t count) {
  // every outer iteration sweeps each feature once in a bundle and once more
  // in the stopping test
  // (with shrinking: the active features the previous stopping sweep chose;
  // exact for one iteration at a time, as the drivers run them)
  const double nz = o.shrink ? c->nnz_active_h : (double)c->nnz;
  const double sl = o.shrink ? c->p_active_h : (double)c->p;
  (void)P;
  c->hc.nnz_gh += nz * count;
  c->hc.slots += sl * count;
  c->hc.nnz_stop += (double)c->nnz * count;
  c->hc.stop_sweeps += (double)count;
}

int set_iter(pcdn_ctx* c, uint64_t seed, int64_t k) {
  c->hiter->seed = seed;
  c->hiter->k = k;
  HIPCHK(c, hipMemcpyAsync(c->iter, c->hiter, sizeof(IterState), hipMemcpyHostToDevice,
                           c->stream));
  // the pinned source may be reused only after the copy ran
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return PCDN_OK;
}

// Outer iterations k_first .. k_first+count-1; the last stopping norm stays in
// c->scal[0].  Replays a captured graph unless kernel profiling is on.
int run_outer(pcdn_ctx* c, const Opts& o, int64_t P, int64_t k_first, int64_t count) {
  if (count <= 0) return PCDN_OK;
  count_outer(c, o, P, count);
  // kernel profiling brackets launches with events: launch directly then
  if (c->use_graphs && c->prof.mask == 0) {
    int rc = ensure_graph(c, o, P);
    if (rc) return rc;
    rc = set_iter(c, o.seed, k_first);
    if (rc) return rc;
    for (int64_t k = 0; k < count; ++k) HIPCHK(c, hipGraphLaunch(c->graph, c->stream));
    return PCDN_OK;
  }
  for (int64_t k = k_first; k < k_first + count; ++k) {
    int rc = enqueue_outer(c, o, P, k, nullptr);
    if (rc) return rc;
  }
  return PCDN_OK;
}

int read_stats(pcdn_ctx* c) {
  HIPCHK(c, hipMemcpyAsync(c->hstats, c->stats, sizeof(Stats), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return PCDN_OK;
}

int range_check(pcdn_ctx* c, const char* what) {
  const int rc = read_stats(c);
  if (rc) return rc;
  return range_noted(c, what);
}

int range_noted(pcdn_ctx* c, const char* what) {
  const unsigned long long n = c->hstats->range_leaves;
  if (n == c->range_seen) return PCDN_OK;
  c->range_seen = n;
  return fail(c, PCDN_E_NUMERIC, what);
}

double alg_bytes_of(const Stats& s, const Stats& b, const pcdn_ctx::HostCounts& h,
                    const pcdn_ctx::HostCounts& hb, int cls, int64_t p) {
  // multi-kernel schedule (classes 0-3) and single-workgroup kernel (class 5)
  // (the single-workgroup kernel counts its own bundles on the device, so a
  // heavy bundle run on the multi-kernel path is credited to classes 0-3)
  const double n_nnz_gh = (double)(s.nnz_gh_narrow - b.nnz_gh_narrow);
  const double n_slots = (double)(s.slots_narrow - b.slots_narrow);
  const double n_fused = (double)(s.nnz_scat_narrow - b.nnz_scat_narrow);
  const double n_long = (double)(s.nnz_scat_narrow_split - b.nnz_scat_narrow_split);
  const double n_scat = n_fused + n_long;
  const double n_rows = (double)(s.rows_touched_narrow - b.rows_touched_narrow);
  const double d_nnz_gh = std::max(0.0, h.nnz_gh - hb.nnz_gh - n_nnz_gh);
  const double d_slots = std::max(0.0, h.slots - hb.slots - n_slots);
  const double d_scat = (double)(s.nnz_scat_rows - b.nnz_scat_rows);
  const double d_rows = (double)(s.rows_touched - b.rows_touched) - n_rows;
  const double d_stop = h.nnz_stop - hb.nnz_stop;
  const double d_sweeps = h.stop_sweeps - hb.stop_sweeps;
  switch (cls) {
    case 0: return kBytesPerNnzSweep * d_nnz_gh + kBytesPerSlotSweep * d_slots;
    case 1: return 0.0;  // the sweep's finish: from partials already counted
    case 2: return kBytesPerNnzScatter * d_scat + kBytesPerRowLs * d_rows +
                   kBytesPerSlotLs * d_slots;
    case 3: return kBytesPerRowApply * d_rows + kBytesPerSlotApply * d_slots;
    case 4: return kBytesPerNnzStop * d_stop + kBytesPerFeatStop * (double)p * d_sweeps;
    case 5: return kBytesPerNnzSweep * n_nnz_gh + kBytesPerSlotNarrow * n_slots +
                   kBytesPerNnzScatter * n_scat + (kBytesPerRowLs + kBytesPerRowApply) * n_rows;
    default: return 0.0;
  }
}


int check_solve_args(pcdn_ctx* c, double C, int64_t P, double eps, int loss,
                     const pcdn_opts* opts, Opts* o) {
  if (!c) return PCDN_E_ARG;
  if (!c->loaded) return fail(c, PCDN_E_STATE, "no data loaded");
  int rc = check_loss(c, loss);
  if (rc) return rc;
  if (!(C > 0.0) || !std::isfinite(C)) return fail(c, PCDN_E_ARG, "C must be a finite positive number");
  if (P < 1 || P > c->p) return fail(c, PCDN_E_ARG, "bundle size P must lie in [1, p]");
  if (!(eps >= 0.0) || !std::isfinite(eps)) return fail(c, PCDN_E_ARG, "eps must be finite and >= 0");
  return resolve_opts(c, opts, o);
}

int solve_begin(SolveRun& r) {
  pcdn_ctx* c = r.c;
  HIPCHK(c, hipSetDevice(c->device));
  r.t0 = std::chrono::steady_clock::now();
  int rc = read_stats(c);
  if (rc) return rc;
  r.base = *c->hstats;
  r.hbase = c->hc;
  c->loss = r.loss;
  rc = set_C(c, r.C);
  if (rc) return rc;
  note_regulariser(c, r.o);
  r.outer = 0;
  r.min_stop_margin = INFINITY;
  // the smallest Armijo margin of this solve (Stats::min_margin_bits)
  HIPCHK(c, launch_fill((double*)&c->stats->min_margin_bits, INFINITY, 1, c->stream));
  rc = init_shrink(c);
  if (rc) return rc;
  // reference norm at w = 0 (retained quantities all one)
  HIPCHK(c, launch_fill(c->cache, 1.0, c->n, c->stream));
  HIPCHK(c, launch_row_weights(c->loss, c->cache, c->y, c->n, c->rw, c->stream));
  r.G0 = r.G = 0.0;
  rc = stopping_norm(c, r.o, nullptr, &r.G0);
  if (rc) return rc;
  if (!std::isfinite(r.G0)) return fail(c, PCDN_E_NUMERIC, "non-finite gradient at w = 0");
  if (r.G0 == 0.0) {
    rc = set_w(c, nullptr);
    if (rc) return rc;
    r.converged = true;
  } else {
    if (r.w0_device) {
      rc = cache_from_w(c, false);
    } else {
      rc = set_w(c, r.o.w0);
    }
    if (rc) return rc;
    if (r.o.w0 || r.w0_device) {
      rc = stopping_norm(c, r.o, c->w, &r.G);
      if (rc) return rc;
    } else {
      r.G = r.G0;
    }
    r.converged = r.G <= r.eps * r.G0;
  }
  c->has_state = true;
  return PCDN_OK;
}

int solve_note_outer(SolveRun& r, double G) {
  ++r.outer;
  r.G = G;
  if (!std::isfinite(G)) return fail(r.c, PCDN_E_NUMERIC, "non-finite subgradient norm");
  r.converged = G <= r.eps * r.G0;
  if (r.eps * r.G0 > 0.0)
    r.min_stop_margin = std::min(r.min_stop_margin, std::fabs(G - r.eps * r.G0) / (r.eps * r.G0));
  return PCDN_OK;
}

int solve_end(SolveRun& r, double* w_out, pcdn_info* info) {
  pcdn_ctx* c = r.c;
  double F = 0.0;
  int rc = objective(c, r.o, &F);
  if (rc) return rc;
  if (w_out)
    HIPCHK(c, hipMemcpyAsync(w_out, c->w, c->p * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  rc = range_check(c, kRangeStep);
  if (rc) return rc;
  if (std::isnan(F)) return fail(c, PCDN_E_NUMERIC, "objective is NaN");
  const auto t1 = std::chrono::steady_clock::now();
  if (info) {
    const Stats& s = *c->hstats;
    info->outer_iters = r.outer;
    info->converged = r.converged ? 1 : 0;
    info->bundles = (int64_t)(s.bundles - r.base.bundles);
    info->ls_steps = (int64_t)(s.ls_steps - r.base.ls_steps);
    info->ls_fail = (int64_t)(s.ls_fail - r.base.ls_fail);
    info->nnz_swept = (int64_t)(c->hc.nnz_gh - r.hbase.nnz_gh);
    info->objective = F;
    info->subgrad = r.G0 == 0.0 ? 0.0 : r.G;
    info->subgrad0 = r.G0;
    double bytes = 0.0;
    for (int k = 0; k < kProfClasses; ++k) bytes += alg_bytes_of(s, r.base, c->hc, r.hbase, k, c->p);
    info->alg_bytes = bytes;
    info->seconds = std::chrono::duration<double>(t1 - r.t0).count();
    double m;
    std::memcpy(&m, &s.min_margin_bits, sizeof m);
    info->min_armijo_margin = m;
    info->min_stop_margin = r.min_stop_margin;
    info->schedule = r.o.schedule;
    info->chunk = r.o.chunk;
  }
  return r.converged ? PCDN_OK : PCDN_NOT_CONVERGED;
}

}  // namespace host
}  // namespace pcdn

using namespace pcdn::host;

// ===========================================================================
// C ABI
// ===========================================================================
static thread_local std::string g_create_error;

namespace pcdn {
namespace host {
std::string& global_error() { return g_create_error; }
}  // namespace host
}  // namespace pcdn

extern "C" int pcdn_create(pcdn_ctx** out, int device, void* hip_stream) {
  if (!out) return PCDN_E_ARG;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
    g_create_error = "no HIP device available";
    return PCDN_E_DEVICE;
  }
  if (device < 0 || device >= ndev) {
    g_create_error = "device index out of range";
    return PCDN_E_ARG;
  }
  pcdn_ctx* c = new (std::nothrow) pcdn_ctx();
  if (!c) return PCDN_E_OOM;
  c->device = device;
  auto bail = [&](int code, const char* msg) {
    g_create_error = msg;
    pcdn_destroy(c);
    return code;
  };
  if (hipSetDevice(device) != hipSuccess) return bail(PCDN_E_DEVICE, "hipSetDevice failed");
  if (hip_stream) {
    c->stream = (hipStream_t)hip_stream;
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess)
      return bail(PCDN_E_DEVICE, "hipStreamCreate failed");
    c->own_stream = true;
  }
  if (dalloc(&c->iter, 1) != hipSuccess || dalloc(&c->st, 1) != hipSuccess ||
      dalloc(&c->stats, 1) != hipSuccess || dalloc(&c->scal, 8) != hipSuccess ||
      dalloc(&c->sum_part, kSumGrid) != hipSuccess ||
      dalloc(&c->stop_part, 4 * kSumGrid) != hipSuccess ||
      dalloc(&c->heavy, kHeavyCap + 1) != hipSuccess)
    return bail(PCDN_E_OOM, "device allocation failed");
  if (hipHostMalloc((void**)&c->hscal, 8 * sizeof(double)) != hipSuccess ||
      hipHostMalloc((void**)&c->hstats, sizeof(Stats)) != hipSuccess ||
      hipHostMalloc((void**)&c->hst, sizeof(StepState)) != hipSuccess ||
      hipHostMalloc((void**)&c->hiter, sizeof(IterState)) != hipSuccess ||
      hipHostMalloc((void**)&c->hheavy, (kHeavyCap + 1) * sizeof(int32_t)) != hipSuccess)
    return bail(PCDN_E_OOM, "pinned host allocation failed");
  if (hipMemsetAsync(c->iter, 0, sizeof(IterState), c->stream) != hipSuccess ||
      hipMemsetAsync(c->stats, 0, sizeof(Stats), c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess)
    return bail(PCDN_E_DEVICE, "initialisation failed");
  *out = c;
  return PCDN_OK;
}

extern "C" int pcdn_destroy(pcdn_ctx* c) {
  if (!c) return PCDN_OK;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  free_data(c);
  dfree(c->iter); dfree(c->st); dfree(c->stats); dfree(c->scal); dfree(c->sum_part);
  dfree(c->stop_part);
  dfree(c->heavy);
  if (c->hheavy) (void)hipHostFree(c->hheavy);
  if (c->hscal) (void)hipHostFree(c->hscal);
  if (c->hstats) (void)hipHostFree(c->hstats);
  if (c->hst) (void)hipHostFree(c->hst);
  if (c->hiter) (void)hipHostFree(c->hiter);
  for (auto& pe : c->prof.pending) {
    (void)hipEventDestroy(pe.second.first);
    (void)hipEventDestroy(pe.second.second);
  }
  for (auto e : c->prof.pool) (void)hipEventDestroy(e);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
  // the errors of these releases are ignored: do not leave one for the next
  // launch check of this thread
  (void)hipGetLastError();
  return PCDN_OK;
}

extern "C" const char* pcdn_last_error(const pcdn_ctx* c) {
  return c ? c->err.c_str() : g_create_error.c_str();
}

namespace pcdn {
namespace host {

// Device bytes pcdn_load_csc allocates for (n, p, nnz), each buffer rounded
// up to 4 KiB, plus the context's own small records.
int64_t ctx_footprint_bytes(int64_t n, int64_t p, int64_t nnz) {
  const int64_t hist_m = radix_hist_ints(p);
  const int64_t part_len = 2 * ((nnz + kWave - 1) / kWave) + 2;
  const int64_t br_m = br_hist_ints(nnz);
  const int64_t sizes[] = {
      8 * (p + 1), 4 * nnz, 4 * nnz, n,                    // X, y
      8 * p, 8 * n, 16 * n, 8 * n, 8 * n, 8 * p,           // w, cache, row weights, d^T x, scratch
      8 * p, 8 * p, 8 * p, 8 * p,                          // g, h, d, Delta terms
      4 * p, 4 * p, 4 * p, 4 * p, 4 * hist_m,              // sort keys and payloads, histogram
      4 * (std::max(std::max(scan_tmp_ints(hist_m), scan_tmp_ints(p)), scan_tmp_ints(br_m)) + 1),
      4 * p, 4 * (nnz / kPermW + 2), 8 * p,                // copy into partition order
      4 * p,                                               // step bundle
      16 * part_len, 4 * nnz, 4 * nnz, 4 * nnz, 8 * (p + 1), 4 * (p + 1),  // partials, X in partition order
      8 * p,                                               // w in partition order
      2 * nnz, 4 * (p + 1),                                // bundle-local row ids
      8 * (int64_t)kRowsGridMax * (4 * kQMax + 3),         // line-search partials
      8 * p,                                               // active mask (shrinking)
      8 * (n + 1), 4 * nnz, 4 * nnz, 4 * nnz, 4 * nnz,     // CSR copy, column of each nonzero
      4 * nnz, 2 * nnz,                                    // stopping-sweep tiles in row order
      4 * p, 12 * nnz, 12 * nnz, 4 * br_m,                 // bundle-row order, sort buffers
      4 * ((nnz + kRangeW - 1) / kRangeW + 1), 12 * (nnz + kRangeW)};  // touched rows
  int64_t total = 64 * 1024;
  for (const int64_t b : sizes) total += (std::max<int64_t>(b, 1) + 4095) / 4096 * 4096;
  return total;
}

}  // namespace host
}  // namespace pcdn

extern "C" int pcdn_load_csc(pcdn_ctx* c, int64_t n, int64_t p, int64_t nnz,
                             const int64_t* col_ptr, const int32_t* row_idx, const float* val,
                             const int8_t* y, int ptr_kind) {
  if (!c) return PCDN_E_ARG;
  if (n < 1 || p < 1 || n >= (int64_t)1 << 31 || p >= (int64_t)1 << 31 || nnz < 0)
    return fail(c, PCDN_E_ARG, "sizes out of range (need 1 <= n, p < 2^31, nnz >= 0)");
  if (!col_ptr || !y || (nnz > 0 && (!row_idx || !val)))
    return fail(c, PCDN_E_ARG, "null array");
  if (ptr_kind != 0 && ptr_kind != 1) return fail(c, PCDN_E_ARG, "ptr_kind must be 0 or 1");
  if (nnz > kMaxNnz)
    return fail(c, PCDN_E_ARG, "matrix too large (at most 2^31 - 2^16 nonzeros)");
  HIPCHK(c, hipSetDevice(c->device));

  // host view for validation (device input is copied down once)
  std::vector<int64_t> hcp;
  std::vector<int32_t> hri;
  std::vector<float> hv;
  std::vector<int8_t> hy;
  const int64_t* Hcp = col_ptr;
  const int32_t* Hri = row_idx;
  const float* Hv = val;
  const int8_t* Hy = y;
  if (ptr_kind == 1) {
    hcp.resize(p + 1);
    hri.resize(nnz);
    hv.resize(nnz);
    hy.resize(n);
    HIPCHK(c, hipMemcpy(hcp.data(), col_ptr, (p + 1) * sizeof(int64_t), hipMemcpyDeviceToHost));
    if (nnz) {
      HIPCHK(c, hipMemcpy(hri.data(), row_idx, nnz * sizeof(int32_t), hipMemcpyDeviceToHost));
      HIPCHK(c, hipMemcpy(hv.data(), val, nnz * sizeof(float), hipMemcpyDeviceToHost));
    }
    HIPCHK(c, hipMemcpy(hy.data(), y, n, hipMemcpyDeviceToHost));
    Hcp = hcp.data();
    Hri = hri.data();
    Hv = hv.data();
    Hy = hy.data();
  }
  if (Hcp[0] != 0 || Hcp[p] != nnz) return fail(c, PCDN_E_CSC, "col_ptr must start at 0 and end at nnz");
  for (int64_t j = 0; j < p; ++j) {
    const int64_t lo = Hcp[j], hi = Hcp[j + 1];
    if (hi < lo) return fail(c, PCDN_E_CSC, "col_ptr is decreasing at column " + std::to_string(j));
    for (int64_t k = lo; k < hi; ++k) {
      const int32_t r = Hri[k];
      if (r < 0 || r >= n) return fail(c, PCDN_E_CSC, "row index out of range in column " + std::to_string(j));
      if (k > lo && r <= Hri[k - 1])
        return fail(c, PCDN_E_CSC, "rows not strictly increasing in column " + std::to_string(j));
      if (!std::isfinite(Hv[k])) return fail(c, PCDN_E_CSC, "non-finite value in column " + std::to_string(j));
    }
  }
  for (int64_t i = 0; i < n; ++i)
    if (Hy[i] != 1 && Hy[i] != -1) return fail(c, PCDN_E_CSC, "label not +1/-1 at row " + std::to_string(i));

  HIPCHK(c, hipStreamSynchronize(c->stream));
  free_data(c);
  c->data_hash = data_fingerprint(n, p, nnz, Hcp, Hri, Hv, Hy);
  c->h_cp.assign(Hcp, Hcp + p + 1);
  {
    std::vector<int64_t> lens(p);
    for (int64_t j = 0; j < p; ++j) lens[j] = Hcp[j + 1] - Hcp[j];
    const int64_t k = std::min<int64_t>(p, kNarrowMaxP);
    std::partial_sort(lens.begin(), lens.begin() + k, lens.end(), std::greater<int64_t>());
    c->top_len.assign(k + 1, 0);
    for (int64_t i = 0; i < k; ++i) c->top_len[i + 1] = c->top_len[i] + lens[i];
  }
  c->n = n;
  c->p = p;
  c->nnz = nnz;
  const int64_t hist_m = radix_hist_ints(p);
  ALLOC(c, c->cp, p + 1);
  ALLOC(c, c->ri, nnz);
  ALLOC(c, c->v, nnz);
  ALLOC(c, c->y, n);
  ALLOC(c, c->w, p);
  ALLOC(c, c->cache, n);
  ALLOC(c, c->rw, n);
  ALLOC(c, c->dtx, n);
  ALLOC(c, c->tmp_n, n);
  ALLOC(c, c->tmp_p, p);
  ALLOC(c, c->g, p);
  ALLOC(c, c->h, p);
  ALLOC(c, c->d, p);
  ALLOC(c, c->dterm, p);
  ALLOC(c, c->keys0, p);
  ALLOC(c, c->keys1, p);
  ALLOC(c, c->idx0, p);
  ALLOC(c, c->idx1, p);
  ALLOC(c, c->hist, hist_m);
  const int64_t br_m = br_hist_ints(nnz);
  ALLOC(c, c->scan_tmp,
        std::max(std::max(scan_tmp_ints(hist_m), scan_tmp_ints(p)), scan_tmp_ints(br_m)) + 1);
  ALLOC(c, c->nch, p);
  ALLOC(c, c->rfirst, nnz / kPermW + 2);
  ALLOC(c, c->psrc, p);
  ALLOC(c, c->step_perm, p);
  c->part_len = 2 * ((nnz + kWave - 1) / kWave) + 2;  // two per range of the smallest width
  ALLOC(c, c->part, c->part_len);
  ALLOC(c, c->pri, nnz);
  ALLOC(c, c->pv, nnz);
  ALLOC(c, c->pslot, nnz);
  ALLOC(c, c->poff, p + 1);
  ALLOC(c, c->pw, p);
  ALLOC(c, c->off32, p + 1);
  ALLOC(c, c->plid, nnz);
  ALLOC(c, c->pR, p + 1);
  ALLOC(c, c->ls_part, (size_t)kRowsGridMax * (4 * kQMax + 3));
  ALLOC(c, c->act, p);
  ALLOC(c, c->rp, n + 1);
  ALLOC(c, c->ccol, nnz);
  ALLOC(c, c->rr, nnz);
  ALLOC(c, c->rc, nnz);
  ALLOC(c, c->rv, nnz);
  ALLOC(c, c->srow, nnz);
  ALLOC(c, c->spos, nnz);
  ALLOC(c, c->islot, p);
  ALLOC(c, c->br_row, nnz);
  ALLOC(c, c->br_slot, nnz);
  ALLOC(c, c->br_val, nnz);
  ALLOC(c, c->bt_row, nnz);
  ALLOC(c, c->bt_slot, nnz);
  ALLOC(c, c->bt_val, nnz);
  ALLOC(c, c->br_hist, br_m);
  ALLOC(c, c->u_cnt, (nnz + kRangeW - 1) / kRangeW + 1);
  ALLOC(c, c->u_row, nnz + kRangeW);
  ALLOC(c, c->u_dtx, nnz + kRangeW);
  // CSR copy (rows in order, columns ascending within a row) for the
  // deterministic margin computation of warm starts and the bundle-row
  // order; the largest row 1-norm for the fixed-point d^T x
  {
    std::vector<int64_t> hrp(n + 1, 0);
    for (int64_t k = 0; k < nnz; ++k) ++hrp[Hri[k] + 1];
    for (int64_t i = 0; i < n; ++i) hrp[i + 1] += hrp[i];
    std::vector<int64_t> next(hrp.begin(), hrp.end() - 1);
    std::vector<int32_t> hrr(nnz), hrc(nnz), hk(nnz);
    std::vector<float> hrv(nnz);
    std::vector<double> l1(n, 0.0);
    for (int64_t j = 0; j < p; ++j)
      for (int64_t k = Hcp[j]; k < Hcp[j + 1]; ++k) {
        const int64_t at = next[Hri[k]]++;
        hrr[at] = Hri[k];
        hrc[at] = (int32_t)j;
        hrv[at] = Hv[k];
        hk[at] = (int32_t)k;
        l1[Hri[k]] += std::fabs((double)Hv[k]);
      }
    // the stopping sweep's tiles (kStopTile consecutive nonzeros of the CSC
    // order): each tile's nonzeros in row order, from the CSR order
    if (nnz) {
      std::vector<int32_t> hsr(nnz);
      std::vector<uint16_t> hsp(nnz);
      std::vector<int64_t> fill((nnz + kStopTile - 1) / kStopTile, 0);
      for (int64_t at = 0; at < nnz; ++at) {
        const int64_t t = hk[at] / kStopTile;
        const int64_t e = t * kStopTile + fill[t]++;
        hsr[e] = hrr[at];
        hsp[e] = (uint16_t)(hk[at] - t * kStopTile);
      }
      HIPCHK(c, hipMemcpy(c->srow, hsr.data(), nnz * sizeof(int32_t), hipMemcpyHostToDevice));
      HIPCHK(c, hipMemcpy(c->spos, hsp.data(), nnz * sizeof(uint16_t), hipMemcpyHostToDevice));
    }
    c->xrow = 0.0;
    for (int64_t i = 0; i < n; ++i) c->xrow = std::max(c->xrow, l1[i]);
    HIPCHK(c, hipMemcpy(c->rp, hrp.data(), (n + 1) * sizeof(int64_t), hipMemcpyHostToDevice));
    if (nnz) {
      std::vector<int32_t> hcc(nnz);
      for (int64_t j = 0; j < p; ++j)
        for (int64_t k = Hcp[j]; k < Hcp[j + 1]; ++k) hcc[k] = (int32_t)j;
      HIPCHK(c, hipMemcpy(c->ccol, hcc.data(), nnz * sizeof(int32_t), hipMemcpyHostToDevice));
      HIPCHK(c, hipMemcpy(c->rr, hrr.data(), nnz * sizeof(int32_t), hipMemcpyHostToDevice));
      HIPCHK(c, hipMemcpy(c->rc, hrc.data(), nnz * sizeof(int32_t), hipMemcpyHostToDevice));
      HIPCHK(c, hipMemcpy(c->rv, hrv.data(), nnz * sizeof(float), hipMemcpyHostToDevice));
    }
  }
  const hipMemcpyKind kind = ptr_kind == 1 ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  HIPCHK(c, hipMemcpyAsync(c->cp, col_ptr, (p + 1) * sizeof(int64_t), kind, c->stream));
  if (nnz) {
    HIPCHK(c, hipMemcpyAsync(c->ri, row_idx, nnz * sizeof(int32_t), kind, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->v, val, nnz * sizeof(float), kind, c->stream));
  }
  HIPCHK(c, hipMemcpyAsync(c->y, y, n, kind, c->stream));
  HIPCHK(c, hipMemsetAsync(c->dtx, 0, n * sizeof(double), c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->loaded = true;
  return PCDN_OK;
}

extern "C" int pcdn_load_csc_bias(pcdn_ctx* c, int64_t n, int64_t p, int64_t nnz,
                                  const int64_t* col_ptr, const int32_t* row_idx,
                                  const float* val, const int8_t* y, int ptr_kind, float bias) {
  if (!c) return PCDN_E_ARG;
  if (!std::isfinite(bias) || bias == 0.0f) return fail(c, PCDN_E_ARG, "bias must be finite and non-zero");
  if (n < 1 || p < 1 || n >= (int64_t)1 << 31 || p + 1 >= (int64_t)1 << 31 || nnz < 0)
    return fail(c, PCDN_E_ARG, "sizes out of range (need 1 <= n, p + 1 < 2^31, nnz >= 0)");
  if (!col_ptr || !y || (nnz > 0 && (!row_idx || !val))) return fail(c, PCDN_E_ARG, "null array");
  if (ptr_kind != 0 && ptr_kind != 1) return fail(c, PCDN_E_ARG, "ptr_kind must be 0 or 1");
  HIPCHK(c, hipSetDevice(c->device));
  // X with the constant column appended, on the host (checked by pcdn_load_csc)
  std::vector<int64_t> cp(p + 2);
  std::vector<int32_t> ri(nnz + n);
  std::vector<float> v(nnz + n);
  std::vector<int8_t> hy(n);
  const hipMemcpyKind kind = ptr_kind == 1 ? hipMemcpyDeviceToHost : hipMemcpyHostToHost;
  HIPCHK(c, hipMemcpy(cp.data(), col_ptr, (p + 1) * sizeof(int64_t), kind));
  if (nnz) {
    HIPCHK(c, hipMemcpy(ri.data(), row_idx, nnz * sizeof(int32_t), kind));
    HIPCHK(c, hipMemcpy(v.data(), val, nnz * sizeof(float), kind));
  }
  HIPCHK(c, hipMemcpy(hy.data(), y, n, kind));
  if (cp[p] != nnz) return fail(c, PCDN_E_CSC, "col_ptr must start at 0 and end at nnz");
  cp[p + 1] = nnz + n;
  for (int64_t i = 0; i < n; ++i) {
    ri[nnz + i] = (int32_t)i;
    v[nnz + i] = bias;
  }
  return pcdn_load_csc(c, n, p + 1, nnz + n, cp.data(), ri.data(), v.data(), hy.data(), 0);
}

extern "C" int pcdn_reset(pcdn_ctx* c, int loss, double C, const double* w) {
  if (!c) return PCDN_E_ARG;
  if (!c->loaded) return fail(c, PCDN_E_STATE, "no data loaded");
  int rc = check_loss(c, loss);
  if (rc) return rc;
  if (!(C > 0.0) || !std::isfinite(C)) return fail(c, PCDN_E_ARG, "C must be a finite positive number");
  HIPCHK(c, hipSetDevice(c->device));
  c->loss = loss;
  rc = set_C(c, C);
  if (rc) return rc;
  c->penalty = PCDN_PENALTY_L1;
  c->l2 = 0.0;
  rc = set_w(c, w);
  if (rc) return rc;
  rc = init_shrink(c);
  if (rc) return rc;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->has_state = true;
  return PCDN_OK;
}

extern "C" int pcdn_step(pcdn_ctx* c, const int32_t* bundle, int64_t P, const pcdn_opts* opts,
                         pcdn_step_info* out, double* g, double* h, double* d, double* dtx) {
  if (!c) return PCDN_E_ARG;
  if (!c->loaded || !c->has_state) return fail(c, PCDN_E_STATE, "call pcdn_reset or pcdn_solve first");
  if (!bundle || P < 1 || P > c->p) return fail(c, PCDN_E_ARG, "bundle size must lie in [1, p]");
  Opts o;
  int rc = resolve_opts(c, opts, &o);
  if (rc) return rc;
  note_regulariser(c, o);
  std::vector<unsigned char> seen(c->p, 0);
  for (int64_t t = 0; t < P; ++t) {
    const int32_t j = bundle[t];
    if (j < 0 || j >= c->p) return fail(c, PCDN_E_ARG, "bundle index out of range");
    if (seen[j]) return fail(c, PCDN_E_ARG, "bundle indices must be distinct");
    seen[j] = 1;
  }
  HIPCHK(c, hipSetDevice(c->device));
  HIPCHK(c, hipMemcpyAsync(c->step_perm, bundle, P * sizeof(int32_t), hipMemcpyHostToDevice,
                           c->stream));
  // run the bundle; keep d^T x before it is cleared
  const bool narrow = use_narrow(c, o, P);
  if (narrow) {
    rc = launch_narrow_bundles(c, o, c->step_perm, P, P, 0, 1, dtx ? c->tmp_n : nullptr);
    if (rc) return rc;
  } else {
    rc = build_bundle_rows(c, c->step_perm, P, P);
    if (rc) return rc;
    rc = run_bundle(c, o, c->step_perm, 0, P, false, P);
    if (rc) return rc;
    if (dtx) {
      HIPCHK(c, launch_fill(c->tmp_n, 0.0, c->n, c->stream));
      HIPCHK(c, launch_rows_scatter(rows_args(c, o, c->step_perm, 0, P, false, P), c->tmp_n,
                                    c->stream));
    }
  }
  double swept = 0.0;
  for (int64_t t = 0; t < P; ++t) swept += (double)(c->h_cp[bundle[t] + 1] - c->h_cp[bundle[t]]);
  c->hc.nnz_gh += swept;
  c->hc.slots += (double)P;
  if (g) HIPCHK(c, hipMemcpyAsync(g, c->g, P * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  if (h) HIPCHK(c, hipMemcpyAsync(h, c->h, P * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  if (d) HIPCHK(c, hipMemcpyAsync(d, c->d, P * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->hst, c->st, sizeof(StepState), hipMemcpyDeviceToHost, c->stream));
  if (dtx)
    HIPCHK(c, hipMemcpyAsync(dtx, c->tmp_n, c->n * sizeof(double), hipMemcpyDeviceToHost,
                             c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  rc = range_check(c, kRangeStep);
  if (rc) return rc;
  if (out) {
    out->alpha = c->hst->alpha;
    out->delta = c->hst->delta;
    out->dF = c->hst->dF;
    out->q = c->hst->q;
    out->pad = 0;
  }
  return PCDN_OK;
}

extern "C" int pcdn_permutation(pcdn_ctx* c, uint64_t seed, int64_t k, int32_t* perm_out) {
  if (!c) return PCDN_E_ARG;
  if (!c->loaded) return fail(c, PCDN_E_STATE, "no data loaded");
  if (!perm_out || k < 0) return fail(c, PCDN_E_ARG, "bad argument");
  HIPCHK(c, hipSetDevice(c->device));
  int rc = device_permutation(c, seed, k, nullptr);
  if (rc) return rc;
  HIPCHK(c, hipMemcpyAsync(perm_out, c->idx0, c->p * sizeof(int32_t), hipMemcpyDeviceToHost,
                           c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return PCDN_OK;
}

extern "C" int pcdn_solve(pcdn_ctx* c, double C, int64_t P, double eps, int loss,
                          const pcdn_opts* opts, double* w_out, pcdn_info* info) {
  SolveRun r;
  int rc = check_solve_args(c, C, P, eps, loss, opts, &r.o);
  if (rc) return rc;
  if (use_hybrid(c, r.o, P) && !c->prof.mask) {
    // heavy bundles on the multi-kernel path: the batch engine's rounds
    pcdn_job job{c, C, P, eps, loss, PCDN_OK, opts, w_out, info};
    rc = pcdn_solve_batch(&job, 1);
    return rc < 0 ? rc : job.status;
  }
  r.c = c;
  r.C = C;
  r.P = P;
  r.eps = eps;
  r.loss = loss;
  rc = solve_begin(r);
  if (rc) return rc;
  while (!r.converged && r.outer < r.o.max_outer) {
    rc = run_outer(c, r.o, P, r.outer, 1);
    if (rc) return rc;
    double G = 0.0;
    rc = read_outer(c, &G);
    if (rc) return rc;
    rc = solve_note_outer(r, G);
    if (rc) return rc;
  }
  return solve_end(r, w_out, info);
}

extern "C" int pcdn_iterate(pcdn_ctx* c, int64_t P, int64_t k_first, int64_t count,
                            const pcdn_opts* opts, double* subgrad) {
  if (!c) return PCDN_E_ARG;
  if (!c->loaded || !c->has_state) return fail(c, PCDN_E_STATE, "call pcdn_reset or pcdn_solve first");
  if (P < 1 || P > c->p) return fail(c, PCDN_E_ARG, "bundle size P must lie in [1, p]");
  if (k_first < 0 || count < 0) return fail(c, PCDN_E_ARG, "k_first and count must be >= 0");
  Opts o;
  int rc = resolve_opts(c, opts, &o);
  if (rc) return rc;
  if (count > 0 && use_hybrid(c, o, P) && !c->prof.mask)  // as pcdn_solve
    return pcdn_iterate_batch(&c, &P, 1, k_first, count, opts, subgrad);
  note_regulariser(c, o);
  HIPCHK(c, hipSetDevice(c->device));
  rc = run_outer(c, o, P, k_first, count);
  if (rc) return rc;
  if (subgrad) {
    if (count == 0) {
      rc = launch_stopping(c, o, c->w, nullptr);
      if (rc) return rc;
    }
    rc = read_scalar(c, 0, subgrad);
    if (rc) return rc;
  } else {
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (c->prof.mask) prof_harvest(c);
  }
  return PCDN_OK;
}

extern "C" int pcdn_get_w(pcdn_ctx* c, double* w_out) {
  if (!c || !w_out) return c ? fail(c, PCDN_E_ARG, "null output") : PCDN_E_ARG;
  if (!c->loaded || !c->has_state) return fail(c, PCDN_E_STATE, "no state");
  HIPCHK(c, hipSetDevice(c->device));
  HIPCHK(c, hipMemcpyAsync(w_out, c->w, c->p * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return PCDN_OK;
}

extern "C" int pcdn_get_cache(pcdn_ctx* c, double* out) {
  if (!c || !out) return c ? fail(c, PCDN_E_ARG, "null output") : PCDN_E_ARG;
  if (!c->loaded || !c->has_state) return fail(c, PCDN_E_STATE, "no state");
  HIPCHK(c, hipSetDevice(c->device));
  HIPCHK(c, hipMemcpyAsync(out, c->cache, c->n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return PCDN_OK;
}

extern "C" int pcdn_evaluate(pcdn_ctx* c, double* F, double* G) {
  if (!c) return PCDN_E_ARG;
  if (!c->loaded || !c->has_state) return fail(c, PCDN_E_STATE, "no state");
  HIPCHK(c, hipSetDevice(c->device));
  Opts o;
  int rc = resolve_opts(c, nullptr, &o);
  if (rc) return rc;
  o.penalty = c->penalty;
  o.l2 = c->l2;
  if (G) {
    rc = stopping_norm(c, o, c->w, G);
    if (rc) return rc;
  }
  if (F) {
    rc = objective(c, o, F);
    if (rc) return rc;
  }
  return PCDN_OK;
}

extern "C" int pcdn_profile(pcdn_ctx* c, int mask) {
  if (!c) return PCDN_E_ARG;
  HIPCHK(c, hipSetDevice(c->device));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  prof_harvest(c);
  for (int k = 0; k < kProfClasses; ++k) {
    c->prof.ms[k] = 0.0;
    c->prof.launches[k] = 0;
  }
  c->prof.mask = mask & ((1 << kProfClasses) - 1);
  int rc = read_stats(c);
  if (rc) return rc;
  c->prof_base = *c->hstats;
  c->prof_hc = c->hc;
  return PCDN_OK;
}

extern "C" int pcdn_profile_read(pcdn_ctx* c, int which, double* ms, int64_t* launches,
                                 double* alg_bytes) {
  if (!c) return PCDN_E_ARG;
  if (which < 0 || which >= kProfClasses) return fail(c, PCDN_E_ARG, "unknown kernel class");
  HIPCHK(c, hipSetDevice(c->device));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  prof_harvest(c);
  int rc = read_stats(c);
  if (rc) return rc;
  if (ms) *ms = c->prof.ms[which];
  if (launches) *launches = c->prof.launches[which];
  if (alg_bytes)
    *alg_bytes = alg_bytes_of(*c->hstats, c->prof_base, c->hc, c->prof_hc, which, c->p);
  return PCDN_OK;
}
