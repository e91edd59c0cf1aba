// Drivers over several solves on one device: independent problems advanced
// together (pcdn_solve_batch), a request server with continuous batching
// (pcdn_server_*), the warm-started regularisation path (pcdn_solve_path)
// and the bundle-size autotuner (pcdn_autotune).  Each problem follows
// exactly the sequence of kernels pcdn_solve would run for it; only the
// interleaving across problems differs.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "pcdn_host.h"

using namespace pcdn;
using namespace pcdn::host;

namespace {

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

// Point a context's stream at another stream for the launches in a scope.
struct StreamSwap {
  pcdn_ctx* c;
  hipStream_t own;
  StreamSwap(pcdn_ctx* c_, hipStream_t s) : c(c_), own(c_->stream) { c->stream = s; }
  ~StreamSwap() { c->stream = own; }
  StreamSwap(const StreamSwap&) = delete;
  StreamSwap& operator=(const StreamSwap&) = delete;
};

// One solve inside the engine.
struct EngineJob {
  SolveRun run;
  bool narrow = false;
  bool hybrid = false;           // single-workgroup segments between heavy bundles, own stream
  std::vector<Task> tasks;       // multi-kernel jobs: the outer iteration, partition included
  hipEvent_t pre_done = nullptr;  // partition done (or, heavy-bundle jobs: chain done)
  bool fresh = true;             // no round yet: the executor waits for its set-up once
  bool active = false;
  int64_t id = 0;                // owner's handle
  bool resume = false;           // continue the context's state (no set-up, no stopping rule)
  int64_t k_first = 0;           // first outer-iteration index when resuming
};

// Grow-only device + pinned buffer pair.
struct Staging {
  void* dev = nullptr;
  void* host = nullptr;
  size_t bytes = 0;
  hipError_t reserve(size_t want) {
    if (want <= bytes) return hipSuccess;
    release();
    want = std::max(want, (size_t)4096);
    hipError_t e = hipMalloc(&dev, want);
    if (e == hipSuccess) e = hipHostMalloc(&host, want);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      release();
      return e;
    }
    bytes = want;
    return hipSuccess;
  }
  void release() {
    if (dev) (void)hipFree(dev);
    if (host) (void)hipHostFree(host);
    dev = host = nullptr;
    bytes = 0;
  }
};

// Rounds of one outer iteration over a changing set of solves.  Jobs on the
// single-workgroup schedule share one launch per round (one workgroup each),
// their partitions and stopping sweeps replayed graphs on their own
// contexts' streams; jobs on the multi-kernel schedule run their recorded
// outer iteration, partition included, in lock-step executor launches
// (launch s runs task s of every such job).
class Engine {
 public:
  std::string err;

  ~Engine() {
    (void)hipSetDevice(device_);
    for (hipStream_t st : chain_stream_)
      if (st) (void)hipStreamSynchronize(st);
    if (narrow_stream_) (void)hipStreamSynchronize(narrow_stream_);
    if (wide_stream_) (void)hipStreamSynchronize(wide_stream_);
    for (EngineJob* j : jobs_) drop_event(j);
    if (fused_done_) (void)hipEventDestroy(fused_done_);
    narrow_tab_.release();
    exec_.release();
    gather_.release();
    if (narrow_stream_) (void)hipStreamDestroy(narrow_stream_);
    if (wide_stream_) (void)hipStreamDestroy(wide_stream_);
    for (hipStream_t st : chain_stream_)
      if (st) (void)hipStreamDestroy(st);
  }

  int init(int device) {
    device_ = device;
    // The chain streams and the executor's stream first: the runtime gives a
    // new stream the hardware queue with the fewest streams, so streams
    // created one after another tend to land on different queues, and
    // launches on one queue run one after another whatever their streams
    // (two heavy-bundle chains on one queue would take the sum of their
    // times, and executor launches queued behind a chain would wait for it).
    if (hipSetDevice(device) != hipSuccess ||
        hipStreamCreateWithFlags(&chain_stream_[0], hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&chain_stream_[1], hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&wide_stream_, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&narrow_stream_, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&fused_done_, hipEventDisableTiming) != hipSuccess)
      return dev_fail("engine set-up", hipGetLastError());
    return PCDN_OK;
  }

  size_t size() const { return jobs_.size(); }

  // Start a job whose run fields (c, o, C, P, eps, loss, w0_device) are set:
  // reference norm and w (solve_begin), graphs or tasks, iteration record.
  // Returns an error code on the job's context; afterwards j->active tells
  // whether it needs rounds (it joins the engine then).
  int add(EngineJob* j) {
    SolveRun& r = j->run;
    int rc = PCDN_OK;
    if (j->resume) {  // iterations only: run.o.max_outer of them, no stopping test
      r.converged = false;
      r.outer = 0;
      r.G0 = 1.0;
      r.eps = -1.0;
    } else {
      rc = solve_begin(r);
      if (rc) return rc;
    }
    j->narrow = use_narrow(r.c, r.o, r.P);
    j->hybrid = j->narrow && use_hybrid(r.c, r.o, r.P);
    // single-workgroup jobs replay the two halves of an outer iteration
    // around their bundles; multi-kernel jobs run theirs as executor tasks
    rc = j->narrow ? ensure_split_graphs(r.c, r.o, r.P) : outer_tasks(r.c, r.o, r.P, j->tasks);
    if (rc) return rc;
    rc = set_iter(r.c, r.o.seed, j->resume ? j->k_first : 0);
    if (rc) return rc;
    j->active = !r.converged && r.outer < r.o.max_outer;
    if (!j->active) return PCDN_OK;
    if (hipEventCreateWithFlags(&j->pre_done, hipEventDisableTiming) != hipSuccess)
      return fail(r.c, PCDN_E_DEVICE, "event creation failed");
    jobs_.push_back(j);
    if (!j->narrow) plan_stale_ = true;
    return PCDN_OK;
  }

  // One outer iteration of every job; the jobs that stop (stopping rule or
  // max_outer) leave the engine and are appended to `done`.  Errors of a
  // job's context come back as its code with the message on that context
  // (*err_ctx set to it); engine-level errors as PCDN_E_DEVICE in `err`.
  int round(std::vector<EngineJob*>& done, pcdn_ctx** err_ctx) {
    *err_ctx = nullptr;
    if (jobs_.empty()) return PCDN_OK;
    if (hipSetDevice(device_) != hipSuccess) return dev_fail("hipSetDevice", hipGetLastError());
    int rc = plan_stale_ ? build_plan() : PCDN_OK;
    if (rc) return rc;
    // partitions, each on its job's stream (the multi-kernel jobs': executor
    // tasks); the single-workgroup jobs' table, one launch for all of them
    size_t m = 0;
    bool any_hybrid = false;
    for (EngineJob* j : jobs_) {
      any_hybrid = any_hybrid || j->hybrid;
      if (j->narrow && !j->hybrid) ++m;
    }
    if (narrow_tab_.reserve(sizeof(NarrowArgs) * m) != hipSuccess)
      return dev_fail("table allocation", hipErrorOutOfMemory);
    NarrowArgs* htab = (NarrowArgs*)narrow_tab_.host;
    size_t at = 0;
    for (EngineJob* j : jobs_) {
      pcdn_ctx* c = j->run.c;
      *err_ctx = c;
      count_outer(c, j->run.o, j->run.P, 1);
      if (!j->narrow) {  // partition and bundles in the executor launches
        if (j->fresh) {
          HIPCHK(c, hipEventRecord(j->pre_done, c->stream));
          HIPCHK(c, hipStreamWaitEvent(wide_stream_, j->pre_done, 0));
        }
        j->fresh = false;
        continue;
      }
      HIPCHK(c, hipGraphLaunch(c->graph_pre, c->stream));
      if (j->hybrid) {  // its bundles follow on its own stream once the list is read
        HIPCHK(c, hipMemcpyAsync(c->hheavy, c->heavy, (kHeavyCap + 1) * sizeof(int32_t),
                                 hipMemcpyDeviceToHost, c->stream));
        continue;
      }
      HIPCHK(c, hipEventRecord(j->pre_done, c->stream));
      HIPCHK(c, hipStreamWaitEvent(narrow_stream_, j->pre_done, 0));
      htab[at++] = outer_narrow_args(c, j->run.o, j->run.P);
    }
    *err_ctx = nullptr;
    // single-workgroup jobs: one launch (both losses), then each job's
    // stopping sweep
    if (m > 0) {
      const char* step = "table upload";
      hipError_t e = hipMemcpyAsync(narrow_tab_.dev, htab, sizeof(NarrowArgs) * m,
                                    hipMemcpyHostToDevice, narrow_stream_);
      if (e == hipSuccess) {
        step = "single-workgroup launch";
        e = launch_narrow_multi((const NarrowArgs*)narrow_tab_.dev, (int)m, narrow_stream_);
      }
      if (e == hipSuccess) {
        step = "event record";
        e = hipEventRecord(fused_done_, narrow_stream_);
      }
      if (e != hipSuccess) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        (void)hipStreamIsCapturing(narrow_stream_, &cs);
        return dev_fail((std::string("multi-problem launch (") + step + ", stream capture status " +
                         std::to_string((int)cs) + ")").c_str(), e);
      }
      for (EngineJob* j : jobs_) {
        if (!j->narrow || j->hybrid) continue;
        pcdn_ctx* c = j->run.c;
        *err_ctx = c;
        HIPCHK(c, hipStreamWaitEvent(c->stream, fused_done_, 0));
        HIPCHK(c, hipGraphLaunch(c->graph_post, c->stream));
        HIPCHK(c, hipMemcpyAsync(c->hscal, c->scal, 8 * sizeof(double), hipMemcpyDeviceToHost,
                                 c->stream));
      }
      *err_ctx = nullptr;
    }
    // single-workgroup jobs with heavy bundles, each on a chain stream: the
    // segments between heavy bundles in one workgroup, each heavy bundle on
    // the multi-kernel path, in partition order.  They are enqueued before
    // the multi-kernel jobs' executor launches: their chains of dependent
    // launches are the round's longest, so they must not start behind the
    // host time of the executor's enqueue.  A job's partition ran on its own
    // stream (the host waited for it to read the heavy-bundle list); its
    // stopping sweep follows there once its chain is done.
    if (any_hybrid) {
      std::vector<EngineJob*> hj;
      std::vector<int64_t> next;  // first bundle not yet enqueued, per job
      for (EngineJob* j : jobs_) {
        if (!j->hybrid) continue;
        pcdn_ctx* c = j->run.c;
        *err_ctx = c;
        HIPCHK(c, hipStreamSynchronize(c->stream));
        hj.push_back(j);
        next.push_back(0);
      }
      // enqueue the jobs' segments round-robin, so that every job starts at once
      for (int32_t k = 0;; ++k) {
        bool more = false;
        for (size_t i = 0; i < hj.size(); ++i) {
          pcdn_ctx* c = hj[i]->run.c;
          const Opts& o = hj[i]->run.o;
          const int64_t P = hj[i]->run.P, nb = (c->p + P - 1) / P;
          const int32_t nh = std::min<int32_t>(std::max<int32_t>(c->hheavy[0], 0), kHeavyCap);
          int64_t& t = next[i];
          if (k > nh || t >= nb) continue;
          *err_ctx = c;
          StreamSwap on_chain(c, chain_stream_[i % 2]);  // run_bundle launches on c->stream
          const int64_t te =
              k < nh ? std::min<int64_t>(std::max<int64_t>(c->hheavy[1 + k], t), nb) : nb;
          if (te > t) HIPCHK(c, launch_narrow(c->loss, segment_narrow_args(c, o, P, t, te), c->stream));
          t = te;
          if (k < nh && te < nb) {
            const int64_t lo = te * P, hi = std::min(lo + P, c->p);
            rc = run_bundle(c, o, c->idx0, lo, hi, o.shrink, P);
            if (rc) return rc;
            t = te + 1;
          }
          more = true;
        }
        if (!more) break;
      }
      for (size_t i = 0; i < hj.size(); ++i) {
        EngineJob* j = hj[i];
        pcdn_ctx* c = j->run.c;
        *err_ctx = c;
        HIPCHK(c, hipEventRecord(j->pre_done, chain_stream_[i % 2]));
        HIPCHK(c, hipStreamWaitEvent(c->stream, j->pre_done, 0));
        HIPCHK(c, hipGraphLaunch(c->graph_post, c->stream));
        HIPCHK(c, hipMemcpyAsync(c->hscal, c->scal, 8 * sizeof(double), hipMemcpyDeviceToHost,
                                 c->stream));
      }
      *err_ctx = nullptr;
    }
    // multi-kernel jobs: partition, every bundle and the stopping sweep in
    // lock-step launches
    if (!plan_jobs_.empty()) {
      const char* base = (const char*)exec_.dev;
      for (size_t st = 0; st < plan_count_.size(); ++st) {
        const hipError_t e = launch_exec((const Task*)(base + plan_task_byte_[st]),
                                         (const int32_t*)(base + plan_first_byte_[st]),
                                         plan_count_[st], plan_blocks_[st], wide_stream_);
        if (e != hipSuccess) return dev_fail("executor launch", e);
      }
      hipError_t e = launch_gather((const double* const*)(base + plan_src_byte_),
                                   (double*)gather_.dev, 3 * (int)plan_jobs_.size(), wide_stream_);
      if (e == hipSuccess)
        e = hipMemcpyAsync(gather_.host, gather_.dev, 3 * sizeof(double) * plan_jobs_.size(),
                           hipMemcpyDeviceToHost, wide_stream_);
      if (e != hipSuccess) return dev_fail("gather", e);
    }
    // the staging tables and every pinned result are reused next round
    hipError_t e = hipStreamSynchronize(narrow_stream_);
    if (e == hipSuccess) e = hipStreamSynchronize(wide_stream_);
    if (e != hipSuccess) return dev_fail("round", e);
    for (size_t k = 0; k < plan_jobs_.size(); ++k) {
      const double* gv = (const double*)gather_.host + 3 * k;
      pcdn_ctx* c = plan_jobs_[k]->run.c;
      c->hscal[0] = gv[0];
      c->hscal[5] = gv[1];
      c->hscal[6] = gv[2];
    }
    std::vector<EngineJob*> keep;
    keep.reserve(jobs_.size());
    for (EngineJob* j : jobs_) {
      pcdn_ctx* c = j->run.c;
      *err_ctx = c;
      HIPCHK(c, hipStreamSynchronize(c->stream));
      c->p_active_h = c->hscal[5];  // next active count and nonzeros (shrinking)
      c->nnz_active_h = c->hscal[6];
      rc = solve_note_outer(j->run, c->hscal[0]);
      if (rc) return rc;
      j->active = !j->run.converged && j->run.outer < j->run.o.max_outer;
      if (j->active) {
        keep.push_back(j);
      } else {
        drop_event(j);
        done.push_back(j);
        if (!j->narrow) plan_stale_ = true;
      }
    }
    *err_ctx = nullptr;
    jobs_.swap(keep);
    return PCDN_OK;
  }

 private:
  int device_ = 0;
  // the heavy-bundle jobs' chains (job i of a round on chain i mod 2)
  hipStream_t chain_stream_[2] = {nullptr, nullptr};
  hipStream_t narrow_stream_ = nullptr;                // the single-workgroup jobs' launch
  hipStream_t wide_stream_ = nullptr;                  // the executor launches
  hipEvent_t fused_done_ = nullptr;
  std::vector<EngineJob*> jobs_;
  Staging narrow_tab_, exec_, gather_;
  bool plan_stale_ = true;
  // lock-step plan of the multi-kernel jobs (byte offsets into exec_)
  std::vector<EngineJob*> plan_jobs_;
  std::vector<size_t> plan_task_byte_, plan_first_byte_;
  std::vector<int> plan_count_, plan_blocks_;
  size_t plan_src_byte_ = 0;

  int dev_fail(const char* what, hipError_t e) {
    (void)hipGetLastError();
    err = std::string(what) + ": " + hipGetErrorString(e);
    return PCDN_E_DEVICE;
  }

  static void drop_event(EngineJob* j) {
    if (j->pre_done) (void)hipEventDestroy(j->pre_done);
    j->pre_done = nullptr;
  }

  // Launch s runs task s of every multi-kernel job that has one.
  int build_plan() {
    plan_jobs_.clear();
    plan_task_byte_.clear();
    plan_first_byte_.clear();
    plan_count_.clear();
    plan_blocks_.clear();
    size_t L = 0, n_tasks = 0;
    for (EngineJob* j : jobs_) {
      if (j->narrow) continue;
      plan_jobs_.push_back(j);
      L = std::max(L, j->tasks.size());
      n_tasks += j->tasks.size();
    }
    plan_stale_ = false;
    if (plan_jobs_.empty()) return PCDN_OK;
    const size_t task_bytes = align_up(sizeof(Task) * n_tasks);
    const size_t first_bytes = align_up(sizeof(int32_t) * (n_tasks + L));
    const size_t src_bytes = align_up(3 * sizeof(double*) * plan_jobs_.size());
    // the previous plan's tables may still be read by nothing: rounds end synchronised
    if (exec_.reserve(task_bytes + first_bytes + src_bytes) != hipSuccess ||
        gather_.reserve(3 * sizeof(double) * plan_jobs_.size()) != hipSuccess)
      return dev_fail("executor table allocation", hipErrorOutOfMemory);
    char* h = (char*)exec_.host;
    Task* htasks = (Task*)h;
    int32_t* hfirst = (int32_t*)(h + task_bytes);
    const double** hsrc = (const double**)(h + task_bytes + first_bytes);
    size_t nt = 0, nf = 0;
    for (size_t st = 0; st < L; ++st) {
      plan_task_byte_.push_back(sizeof(Task) * nt);
      plan_first_byte_.push_back(task_bytes + sizeof(int32_t) * nf);
      int cnt = 0, blk = 0;
      hfirst[nf++] = 0;
      for (EngineJob* j : plan_jobs_) {
        if (st >= j->tasks.size()) continue;
        const Task& t = j->tasks[st];
        htasks[nt++] = t;
        blk += t.nblk;
        hfirst[nf++] = blk;
        ++cnt;
      }
      plan_count_.push_back(cnt);
      plan_blocks_.push_back(blk);
    }
    // per job: the stopping norm, the next active count and nonzeros
    for (size_t k = 0; k < plan_jobs_.size(); ++k) {
      double* sc = plan_jobs_[k]->run.c->scal;
      hsrc[3 * k] = sc;
      hsrc[3 * k + 1] = sc + 5;
      hsrc[3 * k + 2] = sc + 6;
    }
    plan_src_byte_ = task_bytes + first_bytes;
    const hipError_t e = hipMemcpyAsync(exec_.dev, exec_.host, task_bytes + first_bytes + src_bytes,
                                        hipMemcpyHostToDevice, wide_stream_);
    if (e != hipSuccess) return dev_fail("executor table upload", e);
    return PCDN_OK;
  }
};

}  // namespace

extern "C" int pcdn_solve_batch(pcdn_job* jobs, int32_t count) {
  if (count == 0) return PCDN_OK;
  if (!jobs || count < 0) return PCDN_E_ARG;
  // argument checks for every job before any work
  std::vector<EngineJob> ej(count);
  for (int32_t i = 0; i < count; ++i) {
    pcdn_job& j = jobs[i];
    j.status = PCDN_E_ARG;
    if (!j.ctx) return PCDN_E_ARG;
    for (int32_t k = 0; k < i; ++k)
      if (jobs[k].ctx == j.ctx) return fail(j.ctx, PCDN_E_ARG, "two jobs share a context");
    if (j.ctx->device != jobs[0].ctx->device)
      return fail(j.ctx, PCDN_E_ARG, "the contexts of a batch must share one device");
    SolveRun& r = ej[i].run;
    const int rc = check_solve_args(j.ctx, j.C, j.P == 0 ? 1 : j.P, j.eps, j.loss, j.opts, &r.o);
    if (rc) {
      j.status = rc;
      return rc;
    }
    r.c = j.ctx;
    r.C = j.C;
    r.P = j.P;
    r.eps = j.eps;
    r.loss = j.loss;
  }
  // bundle sizes left to the autotuner
  for (int32_t i = 0; i < count; ++i) {
    if (jobs[i].P != 0) continue;
    SolveRun& r = ej[i].run;
    pcdn_tune t;
    const int rc = pcdn_autotune(r.c, r.loss, r.C, r.eps, jobs[i].opts, &t);
    if (rc) {
      jobs[i].status = rc;
      return rc;
    }
    r.P = t.P;
    r.o.schedule = t.schedule;
    r.o.chunk = t.chunk;
    jobs[i].P = t.P;
  }
  Engine eng;
  int rc = eng.init(jobs[0].ctx->device);
  if (rc) return fail(jobs[0].ctx, rc, eng.err);
  for (int32_t i = 0; i < count; ++i) {
    rc = eng.add(&ej[i]);
    if (rc) return rc;
  }
  std::vector<EngineJob*> done;
  while (eng.size() > 0) {
    pcdn_ctx* ec = nullptr;
    rc = eng.round(done, &ec);
    if (rc) return ec ? rc : fail(jobs[0].ctx, rc, eng.err);
  }
  int first_err = PCDN_OK;
  for (int32_t i = 0; i < count; ++i) {
    rc = solve_end(ej[i].run, jobs[i].w_out, jobs[i].info);
    jobs[i].status = rc;
    if (rc < 0 && first_err == PCDN_OK) first_err = rc;
  }
  return first_err;
}

extern "C" int pcdn_iterate_batch(pcdn_ctx* const* ctxs, const int64_t* P, int32_t count,
                                  int64_t k_first, int64_t iters, const pcdn_opts* opts,
                                  double* subgrads) {
  if (count == 0) return PCDN_OK;
  if (!ctxs || !P || count < 0) return PCDN_E_ARG;
  std::vector<EngineJob> ej(count);
  for (int32_t i = 0; i < count; ++i) {
    pcdn_ctx* c = ctxs[i];
    if (!c) return PCDN_E_ARG;
    for (int32_t k = 0; k < i; ++k)
      if (ctxs[k] == c) return fail(c, PCDN_E_ARG, "a context appears twice");
    if (c->device != ctxs[0]->device)
      return fail(c, PCDN_E_ARG, "the contexts must share one device");
    if (!c->loaded || !c->has_state) return fail(c, PCDN_E_STATE, "call pcdn_reset or pcdn_solve first");
    if (P[i] < 1 || P[i] > c->p) return fail(c, PCDN_E_ARG, "bundle size P must lie in [1, p]");
    if (k_first < 0 || iters < 1 || iters > (1 << 30))
      return fail(c, PCDN_E_ARG, "k_first must be >= 0 and iters in [1, 2^30]");
    SolveRun& r = ej[i].run;
    const int rc = resolve_opts(c, opts, &r.o);
    if (rc) return rc;
    note_regulariser(c, r.o);
    r.o.max_outer = (int)iters;
    r.c = c;
    r.C = c->C;
    r.P = P[i];
    r.loss = c->loss;
    ej[i].resume = true;
    ej[i].k_first = k_first;
  }
  Engine eng;
  int rc = eng.init(ctxs[0]->device);
  if (rc) return fail(ctxs[0], rc, eng.err);
  for (int32_t i = 0; i < count; ++i) {
    rc = eng.add(&ej[i]);
    if (rc) return rc;
  }
  std::vector<EngineJob*> done;
  while (eng.size() > 0) {
    pcdn_ctx* ec = nullptr;
    rc = eng.round(done, &ec);
    if (rc) return ec ? rc : fail(ctxs[0], rc, eng.err);
  }
  if (subgrads)
    for (int32_t i = 0; i < count; ++i) subgrads[i] = ej[i].run.G;
  return PCDN_OK;
}

// ===========================================================================
// Solve server: continuous batching.  Requests wait in arrival order; a step
// admits them while their device state fits the budget, runs one engine
// round over everything admitted, and finishes (and frees) what stopped.
// ===========================================================================
namespace {

struct ServerReq {
  int64_t id = 0;
  pcdn_request r{};
  pcdn_opts opts{};
  bool has_opts = false;
  int64_t footprint = 0;
  pcdn_ctx* ctx = nullptr;
  int load_rc = PCDN_OK;  // the loader's outcome (pcdn_create + pcdn_load_csc)
  std::string msg;        // its error message
  EngineJob job;
  ~ServerReq() {
    if (ctx) pcdn_destroy(ctx);
  }
};

struct ServerResult {
  std::vector<double> w;
  pcdn_info info{};
  int32_t status = PCDN_OK;
  std::string msg;  // error message of a failed request
};

}  // namespace

// Requests pass through three queues: waiting (submitted), then loading and
// loaded on the loader thread, which uploads one request at a time in
// submission order once its state fits the budget (the budget is reserved
// when the upload starts), and running once step() has set the solve up in
// the engine.  Uploads (host checks, copies, the CSR copy's sort) thus overlap
// with the engine's rounds, which run on the caller's thread.
struct pcdn_server {
  int device = 0;
  int64_t budget = 0, used = 0;  // used: reserved by uploads and admitted solves
  int64_t next_id = 1;
  std::string err;
  mutable std::mutex mu;         // guards waiting, loaded, loading, used and stop
  // held by the loader while it uploads and by the caller's thread while it
  // sets a solve up (which captures graphs): the HIP runtime has refused
  // other threads' calls while a stream was being captured, whatever the
  // capture mode, so the two never overlap
  std::mutex capture_mu;
  std::condition_variable cv;
  bool stop = false;
  std::thread loader;
  // declared before the engine so that the engine (which refers to the
  // admitted jobs) is destroyed first
  std::deque<std::unique_ptr<ServerReq>> waiting;
  std::deque<std::unique_ptr<ServerReq>> loaded;
  int32_t loading = 0;           // uploads in progress (0 or 1)
  int64_t loading_id = 0;        // the request being uploaded
  std::map<int64_t, std::unique_ptr<ServerReq>> running;
  std::map<int64_t, ServerResult> finished;
  Engine eng;
  ~pcdn_server() {
    {
      std::lock_guard<std::mutex> lk(mu);
      stop = true;
    }
    cv.notify_all();
    if (loader.joinable()) loader.join();
  }
};

namespace {

int server_fail(pcdn_server* s, int code, const std::string& msg) {
  s->err = msg;
  return code;
}

// Record the outcome of an admitted or rejected request and free its state.
void server_finish(pcdn_server* s, std::unique_ptr<ServerReq> q, int status, bool ran) {
  ServerResult res;
  res.status = status;
  if (ran) {
    res.w.assign((size_t)q->r.p, 0.0);
    res.status = solve_end(q->job.run, res.w.data(), &res.info);
  }
  if (res.status < 0) res.msg = !q->msg.empty() ? q->msg : q->ctx ? pcdn_last_error(q->ctx) : "";
  const int64_t fp = q->footprint, id = q->id;
  q.reset();  // the request's context (device memory) is released here
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->used -= fp;
  }
  s->cv.notify_all();  // the loader may now fit the next request
  s->finished[id] = std::move(res);
}

// The loader thread: uploads the next waiting request once it fits.
void server_loader(pcdn_server* s) {
  // this thread's runtime calls must not be refused because the caller's
  // thread is capturing a graph meanwhile
  hipStreamCaptureMode mode = hipStreamCaptureModeRelaxed;
  (void)hipThreadExchangeStreamCaptureMode(&mode);
  for (;;) {
    std::unique_ptr<ServerReq> q;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv.wait(lk, [s] {
        return s->stop ||
               (!s->waiting.empty() && s->used + s->waiting.front()->footprint <= s->budget);
      });
      if (s->stop) return;
      q = std::move(s->waiting.front());
      s->waiting.pop_front();
      s->used += q->footprint;
      ++s->loading;
      s->loading_id = q->id;
    }
    int rc;
    {
      std::lock_guard<std::mutex> cap(s->capture_mu);
      rc = pcdn_create(&q->ctx, s->device, nullptr);
      if (rc) {
        q->msg = pcdn_last_error(nullptr);
      } else {
        const pcdn_request& r = q->r;
        rc = pcdn_load_csc(q->ctx, r.n, r.p, r.nnz, r.col_ptr, r.row_idx, r.val, r.y, 0);
        if (rc) q->msg = pcdn_last_error(q->ctx);
      }
    }
    q->load_rc = rc;
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->loaded.push_back(std::move(q));
      --s->loading;
      s->loading_id = 0;
    }
    s->cv.notify_all();
  }
}

// Set up an uploaded request's solve; on success it joins the engine (or has
// already stopped, e.g. w = 0 optimal).
int server_admit(pcdn_server* s, ServerReq* q) {
  if (q->load_rc) return q->load_rc;
  const pcdn_request& r = q->r;
  SolveRun& run = q->job.run;
  const int64_t P = r.P == 0 ? std::max<int64_t>(1, std::llround(0.05 * (double)r.p)) : r.P;
  int rc = check_solve_args(q->ctx, r.C, P, r.eps, r.loss, q->has_opts ? &q->opts : nullptr,
                            &run.o);
  if (rc) return rc;
  run.c = q->ctx;
  run.C = r.C;
  run.P = P;
  run.eps = r.eps;
  run.loss = r.loss;
  q->job.id = q->id;
  std::lock_guard<std::mutex> cap(s->capture_mu);
  return s->eng.add(&q->job);
}

}  // namespace

extern "C" int pcdn_server_create(pcdn_server** out, int device, int64_t hbm_budget_bytes) {
  if (!out) return PCDN_E_ARG;
  *out = nullptr;
  if (hbm_budget_bytes <= 0) return PCDN_E_ARG;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return PCDN_E_DEVICE;
  if (device < 0 || device >= ndev) return PCDN_E_ARG;
  pcdn_server* s = new (std::nothrow) pcdn_server();
  if (!s) return PCDN_E_OOM;
  s->device = device;
  s->budget = hbm_budget_bytes;
  if (s->eng.init(device) != PCDN_OK) {
    delete s;
    return PCDN_E_DEVICE;
  }
  try {
    s->loader = std::thread(server_loader, s);
  } catch (...) {
    delete s;
    return PCDN_E_OOM;
  }
  *out = s;
  return PCDN_OK;
}

extern "C" int pcdn_server_submit(pcdn_server* s, const pcdn_request* r, int64_t* id) {
  if (!s) return PCDN_E_ARG;
  if (!r || !id) return server_fail(s, PCDN_E_ARG, "null argument");
  if (r->n < 1 || r->p < 1 || r->nnz < 0 || r->n >= ((int64_t)1 << 31) || r->p >= ((int64_t)1 << 31))
    return server_fail(s, PCDN_E_ARG, "sizes out of range");
  if (!r->col_ptr || !r->y || (r->nnz > 0 && (!r->row_idx || !r->val)))
    return server_fail(s, PCDN_E_ARG, "null array");
  if (r->loss != PCDN_LOSS_LOGISTIC && r->loss != PCDN_LOSS_L2SVM)
    return server_fail(s, PCDN_E_ARG, "unknown loss");
  if (!(r->C > 0.0) || !std::isfinite(r->C)) return server_fail(s, PCDN_E_ARG, "C must be > 0");
  if (!(r->eps >= 0.0) || !std::isfinite(r->eps)) return server_fail(s, PCDN_E_ARG, "eps must be >= 0");
  if (r->P < 0 || r->P > r->p) return server_fail(s, PCDN_E_ARG, "P must lie in [0, p]");
  if (r->reserved != 0) return server_fail(s, PCDN_E_ARG, "reserved field must be 0");
  auto q = std::make_unique<ServerReq>();
  q->r = *r;
  if (r->opts) {
    q->opts = *r->opts;
    q->has_opts = true;
  }
  q->footprint = ctx_footprint_bytes(r->n, r->p, r->nnz);
  if (q->footprint > s->budget)
    return server_fail(s, PCDN_E_OOM, "the request's device state exceeds the server's budget");
  q->id = s->next_id++;
  *id = q->id;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->waiting.push_back(std::move(q));
  }
  s->cv.notify_all();
  return PCDN_OK;
}

extern "C" int pcdn_server_step(pcdn_server* s, int32_t* finished) {
  if (!s) return PCDN_E_ARG;
  int32_t nfin = 0;
  if (finished) *finished = 0;
  // admission of the uploaded requests, in submission order; with nothing
  // running, wait for the next upload instead of returning idle
  std::deque<std::unique_ptr<ServerReq>> ready;
  {
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->eng.size() == 0 && s->loaded.empty() && (s->loading > 0 || !s->waiting.empty()))
      s->cv.wait(lk, [s] { return !s->loaded.empty() || (s->loading == 0 && s->waiting.empty()); });
    ready.swap(s->loaded);
  }
  std::sort(ready.begin(), ready.end(),
            [](const std::unique_ptr<ServerReq>& x, const std::unique_ptr<ServerReq>& y) {
              return x->id < y->id;
            });
  for (auto& qr : ready) {
    std::unique_ptr<ServerReq> q = std::move(qr);
    const int rc = server_admit(s, q.get());
    if (rc != PCDN_OK) {
      server_finish(s, std::move(q), rc, false);
      ++nfin;
    } else if (!q->job.active) {
      server_finish(s, std::move(q), PCDN_OK, true);
      ++nfin;
    } else {
      const int64_t id = q->id;
      s->running[id] = std::move(q);
    }
  }
  // one outer iteration of every admitted solve
  if (s->eng.size() > 0) {
    std::vector<EngineJob*> done;
    pcdn_ctx* ec = nullptr;
    const int rc = s->eng.round(done, &ec);
    if (rc) return server_fail(s, rc, ec ? pcdn_last_error(ec) : s->eng.err);
    for (EngineJob* j : done) {
      auto it = s->running.find(j->id);
      if (it == s->running.end()) continue;
      std::unique_ptr<ServerReq> q = std::move(it->second);
      s->running.erase(it);
      server_finish(s, std::move(q), PCDN_OK, true);
      ++nfin;
    }
  }
  if (finished) *finished = nfin;
  return PCDN_OK;
}

extern "C" int pcdn_server_status(const pcdn_server* s, int32_t* waiting, int32_t* running,
                                  int64_t* bytes_in_use) {
  if (!s) return PCDN_E_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  if (waiting) *waiting = (int32_t)(s->waiting.size() + s->loaded.size()) + s->loading;
  if (running) *running = (int32_t)s->running.size();
  if (bytes_in_use) *bytes_in_use = s->used;
  return PCDN_OK;
}

extern "C" int pcdn_server_take(pcdn_server* s, int64_t id, double* w_out, pcdn_info* info,
                                int32_t* status) {
  if (!s) return PCDN_E_ARG;
  auto it = s->finished.find(id);
  if (it == s->finished.end()) {
    if (s->running.count(id)) return server_fail(s, PCDN_E_STATE, "request still running");
    std::lock_guard<std::mutex> lk(s->mu);
    for (const auto& q : s->waiting)
      if (q->id == id) return server_fail(s, PCDN_E_STATE, "request still waiting");
    for (const auto& q : s->loaded)
      if (q->id == id) return server_fail(s, PCDN_E_STATE, "request still waiting");
    if (id == s->loading_id) return server_fail(s, PCDN_E_STATE, "request still waiting");
    return server_fail(s, PCDN_E_ARG, "unknown request id");
  }
  const ServerResult& res = it->second;
  if (w_out && !res.w.empty()) std::memcpy(w_out, res.w.data(), res.w.size() * sizeof(double));
  if (info) *info = res.info;
  if (status) *status = res.status;
  if (res.status < 0) s->err = res.msg;
  s->finished.erase(it);
  return PCDN_OK;
}

extern "C" const char* pcdn_server_last_error(const pcdn_server* s) {
  return s ? s->err.c_str() : "";
}

extern "C" int pcdn_server_destroy(pcdn_server* s) {
  delete s;
  return PCDN_OK;
}

extern "C" int pcdn_solve_path(pcdn_ctx* c, const double* Cs, int32_t count, int64_t P,
                               double eps, int loss, const pcdn_opts* opts, double* W_out,
                               pcdn_info* infos) {
  if (!c) return PCDN_E_ARG;
  if (count < 0 || (count > 0 && !Cs)) return fail(c, PCDN_E_ARG, "bad C list");
  // every C is checked before any work
  for (int32_t k = 0; k < count; ++k) {
    Opts o;
    const int rc = check_solve_args(c, Cs[k], P, eps, loss, opts, &o);
    if (rc) return rc;
  }
  int status = PCDN_OK;
  for (int32_t k = 0; k < count; ++k) {
    SolveRun r;
    int rc = check_solve_args(c, Cs[k], P, eps, loss, opts, &r.o);
    if (rc) return rc;
    r.c = c;
    r.C = Cs[k];
    r.P = P;
    r.eps = eps;
    r.loss = loss;
    r.w0_device = k > 0;  // the previous solution is still on the device
    if (k > 0) r.o.w0 = nullptr;
    if (use_hybrid(c, r.o, P) && !c->prof.mask) {
      // heavy bundles on the multi-kernel path: the engine's rounds, one job
      EngineJob j;
      j.run = r;
      Engine eng;
      rc = eng.init(c->device);
      if (rc) return fail(c, rc, eng.err);
      rc = eng.add(&j);
      if (rc) return rc;
      std::vector<EngineJob*> fin;
      while (eng.size() > 0) {
        pcdn_ctx* ec = nullptr;
        rc = eng.round(fin, &ec);
        if (rc) return ec ? rc : fail(c, rc, eng.err);
      }
      r = j.run;
    } else {
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
    }
    rc = solve_end(r, W_out ? W_out + (size_t)k * (size_t)c->p : nullptr,
                   infos ? infos + k : nullptr);
    if (rc < 0) return rc;
    if (rc == PCDN_NOT_CONVERGED) status = rc;
  }
  return status;
}

extern "C" int pcdn_solve_path_lanes(pcdn_ctx* const* ctxs, int32_t lanes, const double* Cs,
                                     int32_t count, int64_t P, double eps, int loss,
                                     const pcdn_opts* opts, double* W_out, pcdn_info* infos) {
  if (!ctxs || lanes < 1) return PCDN_E_ARG;
  if (count < 0 || (count > 0 && !Cs)) return ctxs[0] ? fail(ctxs[0], PCDN_E_ARG, "bad C list") : PCDN_E_ARG;
  const int32_t L = std::min(lanes, std::max(count, (int32_t)1));
  for (int32_t i = 0; i < L; ++i) {
    pcdn_ctx* c = ctxs[i];
    if (!c) return PCDN_E_ARG;
    for (int32_t k = 0; k < i; ++k)
      if (ctxs[k] == c) return fail(c, PCDN_E_ARG, "a context appears twice");
    if (!c->loaded) return fail(c, PCDN_E_STATE, "no data loaded");
    if (c->device != ctxs[0]->device) return fail(c, PCDN_E_ARG, "the contexts must share one device");
    if (c->n != ctxs[0]->n || c->p != ctxs[0]->p || c->nnz != ctxs[0]->nnz ||
        c->data_hash != ctxs[0]->data_hash)
      return fail(c, PCDN_E_ARG, "the contexts must hold the same X and y");
  }
  pcdn_ctx* c0 = ctxs[0];
  for (int32_t k = 0; k < count; ++k) {
    Opts o;
    const int rc = check_solve_args(c0, Cs[k], P, eps, loss, opts, &o);
    if (rc) return rc;
  }
  if (count == 0) return PCDN_OK;
  // lane i solves Cs[first[i]] .. Cs[first[i + 1] - 1] as a warm-started chain
  std::vector<int32_t> first(L + 1), next(L);
  for (int32_t i = 0; i <= L; ++i) first[i] = (int32_t)(((int64_t)i * count) / L);
  for (int32_t i = 0; i < L; ++i) next[i] = first[i];
  std::vector<std::unique_ptr<EngineJob>> jobs(L);
  std::vector<int32_t> at(L, -1);  // index into Cs of the lane's current solve
  int status = PCDN_OK;
  Engine eng;
  int rc = eng.init(c0->device);
  if (rc) return fail(c0, rc, eng.err);
  // Starts lane i's next solve; solves that stop at once (w already meets
  // the rule) finish here and the lane moves on.
  auto start = [&](int32_t i) -> int {
    while (next[i] < first[i + 1]) {
      const int32_t k = next[i]++;
      auto j = std::make_unique<EngineJob>();
      SolveRun& r = j->run;
      int src = check_solve_args(ctxs[i], Cs[k], P, eps, loss, opts, &r.o);
      if (src) return src;
      r.c = ctxs[i];
      r.C = Cs[k];
      r.P = P;
      r.eps = eps;
      r.loss = loss;
      r.w0_device = k > first[i];  // the lane's previous solution is on the device
      if (k > first[i]) r.o.w0 = nullptr;
      j->id = i;
      src = eng.add(j.get());
      if (src) return src;
      at[i] = k;
      jobs[i] = std::move(j);
      if (jobs[i]->active) return PCDN_OK;
      src = solve_end(jobs[i]->run, W_out ? W_out + (size_t)k * (size_t)c0->p : nullptr,
                      infos ? infos + k : nullptr);
      if (src < 0) return src;
      if (src == PCDN_NOT_CONVERGED) status = src;
      jobs[i].reset();
    }
    return PCDN_OK;
  };
  for (int32_t i = 0; i < L; ++i) {
    rc = start(i);
    if (rc) return rc;
  }
  std::vector<EngineJob*> done;
  while (eng.size() > 0) {
    pcdn_ctx* ec = nullptr;
    done.clear();
    rc = eng.round(done, &ec);
    if (rc) return ec ? rc : fail(c0, rc, eng.err);
    for (EngineJob* j : done) {
      const int32_t i = (int32_t)j->id, k = at[i];
      rc = solve_end(j->run, W_out ? W_out + (size_t)k * (size_t)c0->p : nullptr,
                     infos ? infos + k : nullptr);
      if (rc < 0) return rc;
      if (rc == PCDN_NOT_CONVERGED) status = rc;
      jobs[i].reset();
      rc = start(i);
      if (rc) return rc;
    }
  }
  return status;
}

extern "C" int pcdn_autotune(pcdn_ctx* c, int loss, double C, double eps, const pcdn_opts* opts,
                             pcdn_tune* out) {
  if (!c) return PCDN_E_ARG;
  if (!out) return fail(c, PCDN_E_ARG, "null output");
  Opts o;
  int rc = check_solve_args(c, C, 1, eps, loss, opts, &o);
  if (rc) return rc;
  std::memset(out, 0, sizeof(*out));
  const int64_t p = c->p;
  const int max_tried = (int)(sizeof(out->tried) / sizeof(out->tried[0]));
  const bool tune_schedule = o.schedule == PCDN_SCHED_AUTO;
  const bool tune_chunk = !(opts && opts->chunk);
  // the paper's pilot start, about 5% of the features, then its neighbours
  // on a factor-4 ladder, nearest first
  const int64_t P0 = std::max<int64_t>(1, std::llround(0.05 * (double)p));
  using clock = std::chrono::steady_clock;
  double best = INFINITY;          // fastest finished pilot
  double best_progress = -1.0;     // fallback when none finishes: log-decrease per second
  int best_narrow = use_narrow(c, o, P0) ? 1 : 0;
  out->P = P0;
  out->schedule = o.schedule;
  out->chunk = o.chunk;
  out->predicted_seconds = INFINITY;
  bool done = false;               // a pilot met the rule at its start
  // One pilot: the solve through the batch engine (one job), timed after its
  // set-up, abandoned once slower than the fastest finished pilot.
  auto pilot = [&](int64_t P, int schedule, int chunk) -> int {
    if (done || out->n_tried >= max_tried) return PCDN_OK;
    EngineJob j;
    SolveRun& r = j.run;
    r.o = o;
    r.o.schedule = schedule;
    r.o.chunk = chunk;
    r.c = c;
    r.C = C;
    r.P = P;
    r.eps = eps;
    r.loss = loss;
    Engine eng;
    int prc = eng.init(c->device);
    if (prc) return fail(c, prc, eng.err);
    prc = eng.add(&j);
    if (prc) return prc;
    pcdn_tune_point& tp = out->tried[out->n_tried++];
    tp.P = P;
    tp.schedule = schedule;
    tp.chunk = chunk;
    tp.narrow = j.narrow ? 1 : 0;
    if (!j.active && r.converged) {  // w = 0 (or the warm start) already meets the rule
      tp.predicted_seconds = 0.0;
      out->P = P;
      out->schedule = schedule;
      out->chunk = chunk;
      out->predicted_seconds = 0.0;
      done = true;
      return PCDN_OK;
    }
    bool pruned = false;
    const auto t0 = clock::now();
    double elapsed = 0.0;
    std::vector<EngineJob*> fin;
    while (eng.size() > 0) {
      pcdn_ctx* ec = nullptr;
      prc = eng.round(fin, &ec);
      if (prc) return ec ? prc : fail(c, prc, eng.err);
      elapsed = std::chrono::duration<double>(clock::now() - t0).count();
      if (eng.size() > 0 && elapsed > best) {  // already slower than the best finished pilot
        pruned = true;
        break;
      }
    }
    tp.outer = (int32_t)r.outer;
    tp.sec_per_outer = r.outer > 0 ? elapsed / r.outer : 0.0;
    tp.rate = (r.outer > 0 && r.G > 0.0) ? std::log(r.G0 / r.G) / r.outer : 0.0;
    tp.predicted_seconds = r.converged ? elapsed : INFINITY;
    if (r.converged && elapsed < best) {
      best = elapsed;
      best_narrow = tp.narrow;
      out->P = P;
      out->schedule = schedule;
      out->chunk = chunk;
      out->predicted_seconds = elapsed;
    } else if (!std::isfinite(best) && !pruned) {
      // nothing has finished yet: keep the pilot that went furthest per second
      const double progress = elapsed > 0.0 ? std::log(r.G0 / std::max(r.G, 1e-300)) / elapsed : 0.0;
      if (progress > best_progress) {
        best_progress = progress;
        best_narrow = tp.narrow;
        out->P = P;
        out->schedule = schedule;
        out->chunk = chunk;
      }
    }
    return PCDN_OK;
  };
  // 1. bundle size
  std::vector<int64_t> cands;
  for (const int k : {0, -1, 1, -2, 2, -3}) {
    const double v = (double)P0 * std::pow(4.0, k);
    const int64_t P = std::min<int64_t>(p, std::max<int64_t>(1, std::llround(v)));
    if (std::find(cands.begin(), cands.end(), P) == cands.end()) cands.push_back(P);
  }
  for (const int64_t P : cands) {
    rc = pilot(P, o.schedule, o.chunk);
    if (rc) return rc;
  }
  // 2. the schedule the automatic choice did not take, at the best P
  const int64_t Pb = out->P;
  if (tune_schedule && !done) {
    Opts on = o;
    on.schedule = PCDN_SCHED_NARROW;
    if (best_narrow)
      rc = pilot(Pb, PCDN_SCHED_WIDE, o.chunk);
    else if (use_narrow(c, on, Pb))
      rc = pilot(Pb, PCDN_SCHED_NARROW, o.chunk);
    if (rc) return rc;
  }
  // 3. the other range widths of the bundle sweep (nonzeros per wavefront),
  //    when multi-kernel bundles ran (WIDE, or the heavy bundles of the
  //    automatic single-workgroup schedule)
  Opts ob = o;
  ob.schedule = out->schedule;
  if (tune_chunk && !done && (!best_narrow || use_hybrid(c, ob, Pb))) {
    const int sched = out->schedule;
    for (const int ch : {64, 128, 512}) {
      rc = pilot(Pb, sched, ch);
      if (rc) return rc;
    }
  }
  return PCDN_OK;
}
