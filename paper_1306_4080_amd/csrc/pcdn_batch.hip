// Drivers over several solves on one device: independent problems advanced
// together (pcdn_solve_batch) and the warm-started regularisation path
// (pcdn_solve_path).  Each problem follows exactly the sequence of kernels
// pcdn_solve would run for it; only the interleaving across problems differs.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "pcdn_host.h"

using namespace pcdn;
using namespace pcdn::host;

namespace {

// Device resources of one pcdn_solve_batch call, released on every exit.
struct BatchRes {
  int device = 0;
  hipStream_t narrow_stream = nullptr;  // the multi-problem single-workgroup launch
  hipStream_t wide_stream = nullptr;    // the executor launches
  hipEvent_t fused_done = nullptr;
  std::vector<hipEvent_t> pre_done;
  NarrowArgs* dtab = nullptr;           // device table of the fused launch
  NarrowArgs* htab = nullptr;           // pinned staging for it
  void* dexec = nullptr;                // executor tables (tasks, block offsets, scalar sources)
  void* hexec = nullptr;                // pinned staging for them
  size_t exec_bytes = 0;
  double* dG = nullptr;                 // gathered stopping norms of the multi-kernel jobs
  double* hG = nullptr;
  ~BatchRes() {
    (void)hipSetDevice(device);
    if (narrow_stream) (void)hipStreamSynchronize(narrow_stream);
    if (wide_stream) (void)hipStreamSynchronize(wide_stream);
    for (hipEvent_t e : pre_done)
      if (e) (void)hipEventDestroy(e);
    if (fused_done) (void)hipEventDestroy(fused_done);
    if (dtab) (void)hipFree(dtab);
    if (htab) (void)hipHostFree(htab);
    if (dexec) (void)hipFree(dexec);
    if (hexec) (void)hipHostFree(hexec);
    if (dG) (void)hipFree(dG);
    if (hG) (void)hipHostFree(hG);
    if (narrow_stream) (void)hipStreamDestroy(narrow_stream);
    if (wide_stream) (void)hipStreamDestroy(wide_stream);
  }
};

// Device error of the batch itself, reported on the first job's context.
int batch_fail(pcdn_ctx* c, hipError_t e, const char* what) {
  (void)hipGetLastError();
  return fail(c, PCDN_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

// Lock-step schedule of the multi-kernel jobs of one round: launch s runs
// task s of every job that has one (a job's tasks are the kernels of its
// outer iteration after the partition, in order).
struct ExecPlan {
  std::vector<int> jobs;          // job indices, in gather order
  std::vector<size_t> task_off;   // per launch: first task (index into the task table)
  std::vector<size_t> first_off;  // per launch: first block offset (index into the offsets)
  std::vector<int> count, blocks; // per launch
  size_t n_tasks = 0, n_first = 0;
};

}  // namespace

extern "C" int pcdn_solve_batch(pcdn_job* jobs, int32_t count) {
  if (count == 0) return PCDN_OK;
  if (!jobs || count < 0) return PCDN_E_ARG;
  // argument checks for every job before any work
  std::vector<SolveRun> runs(count);
  for (int32_t i = 0; i < count; ++i) {
    pcdn_job& j = jobs[i];
    j.status = PCDN_E_ARG;
    if (!j.ctx) return PCDN_E_ARG;
    for (int32_t k = 0; k < i; ++k)
      if (jobs[k].ctx == j.ctx) return fail(j.ctx, PCDN_E_ARG, "two jobs share a context");
    if (j.ctx->device != jobs[0].ctx->device)
      return fail(j.ctx, PCDN_E_ARG, "the contexts of a batch must share one device");
    const int rc = check_solve_args(j.ctx, j.C, j.P == 0 ? 1 : j.P, j.eps, j.loss, j.opts,
                                    &runs[i].o);
    if (rc) {
      j.status = rc;
      return rc;
    }
    runs[i].c = j.ctx;
    runs[i].C = j.C;
    runs[i].P = j.P;
    runs[i].eps = j.eps;
    runs[i].loss = j.loss;
  }
  // bundle sizes left to the autotuner
  for (int32_t i = 0; i < count; ++i) {
    if (jobs[i].P != 0) continue;
    pcdn_tune t;
    const int rc = pcdn_autotune(runs[i].c, runs[i].loss, runs[i].C, runs[i].eps, jobs[i].opts, &t);
    if (rc) {
      jobs[i].status = rc;
      return rc;
    }
    runs[i].P = t.P;
    jobs[i].P = t.P;
  }
  pcdn_ctx* c0 = jobs[0].ctx;
  BatchRes res;
  res.device = c0->device;
  HIPCHK(c0, hipSetDevice(res.device));
  HIPCHK(c0, hipStreamCreateWithFlags(&res.narrow_stream, hipStreamNonBlocking));
  HIPCHK(c0, hipStreamCreateWithFlags(&res.wide_stream, hipStreamNonBlocking));
  HIPCHK(c0, hipEventCreateWithFlags(&res.fused_done, hipEventDisableTiming));
  res.pre_done.assign(count, nullptr);
  for (int32_t i = 0; i < count; ++i)
    HIPCHK(c0, hipEventCreateWithFlags(&res.pre_done[i], hipEventDisableTiming));

  // set-up: reference norm and w per job, graphs or task lists, iteration record
  std::vector<char> narrow(count, 0), active(count, 0);
  std::vector<std::vector<Task>> tasks(count);
  int32_t n_narrow = 0;
  size_t all_tasks = 0, all_first = 0, max_len = 0;
  for (int32_t i = 0; i < count; ++i) {
    SolveRun& r = runs[i];
    int rc = solve_begin(r);
    if (rc) return rc;
    narrow[i] = use_narrow(r.c, r.o, r.P) ? 1 : 0;
    n_narrow += narrow[i];
    rc = ensure_split_graphs(r.c, r.o, r.P);
    if (rc) return rc;
    if (!narrow[i]) {
      rc = outer_tasks(r.c, r.o, r.P, tasks[i]);
      if (rc) return rc;
      all_tasks += tasks[i].size();
      max_len = std::max(max_len, tasks[i].size());
    }
    rc = set_iter(r.c, r.o.seed, 0);
    if (rc) return rc;
    active[i] = !r.converged && r.outer < r.o.max_outer;
  }
  const int32_t n_wide = count - n_narrow;
  // at most one block-offset entry per task plus one per launch
  all_first = all_tasks + max_len;
  if (n_narrow > 0) {
    if (dalloc(&res.dtab, n_narrow) != hipSuccess ||
        hipHostMalloc((void**)&res.htab, sizeof(NarrowArgs) * n_narrow) != hipSuccess) {
      (void)hipGetLastError();
      return fail(c0, PCDN_E_OOM, "allocation failed for the batch table");
    }
  }
  if (n_wide > 0) {
    res.exec_bytes = align_up(sizeof(Task) * all_tasks) + align_up(sizeof(int32_t) * all_first) +
                     align_up(sizeof(double*) * n_wide);
    if (hipMalloc(&res.dexec, res.exec_bytes) != hipSuccess ||
        hipHostMalloc(&res.hexec, res.exec_bytes) != hipSuccess ||
        dalloc(&res.dG, n_wide) != hipSuccess ||
        hipHostMalloc((void**)&res.hG, sizeof(double) * n_wide) != hipSuccess) {
      (void)hipGetLastError();
      return fail(c0, PCDN_E_OOM, "allocation failed for the executor tables");
    }
  }
  Task* const htasks = (Task*)res.hexec;
  int32_t* const hfirst = (int32_t*)((char*)res.hexec + align_up(sizeof(Task) * all_tasks));
  const double** const hsrc =
      (const double**)((char*)hfirst + align_up(sizeof(int32_t) * all_first));
  const Task* const dtasks = (const Task*)res.dexec;
  const int32_t* const dfirst = (const int32_t*)((char*)res.dexec + ((char*)hfirst - (char*)res.hexec));
  const double* const* const dsrc =
      (const double* const*)((char*)res.dexec + ((char*)hsrc - (char*)res.hexec));

  ExecPlan plan;
  bool plan_stale = true;
  // rounds: one outer iteration of every active job
  for (;;) {
    int32_t live = 0;
    for (int32_t i = 0; i < count; ++i) live += active[i];
    if (live == 0) break;
    // multi-kernel jobs: (re)build the lock-step tables when the set changed
    if (plan_stale) {
      plan = ExecPlan();
      for (int32_t i = 0; i < count; ++i)
        if (active[i] && !narrow[i]) plan.jobs.push_back(i);
      size_t L = 0;
      for (int i : plan.jobs) L = std::max(L, tasks[i].size());
      for (size_t st = 0; st < L; ++st) {
        plan.task_off.push_back(plan.n_tasks);
        plan.first_off.push_back(plan.n_first);
        int cnt = 0, blk = 0;
        hfirst[plan.n_first++] = 0;
        for (int i : plan.jobs) {
          if (st >= tasks[i].size()) continue;
          htasks[plan.n_tasks++] = tasks[i][st];
          blk += tasks[i][st].nblk;
          hfirst[plan.n_first++] = blk;
          ++cnt;
        }
        plan.count.push_back(cnt);
        plan.blocks.push_back(blk);
      }
      for (size_t k = 0; k < plan.jobs.size(); ++k) hsrc[k] = runs[plan.jobs[k]].c->scal;
      if (!plan.jobs.empty()) {
        const hipError_t e = hipMemcpyAsync(res.dexec, res.hexec, res.exec_bytes,
                                            hipMemcpyHostToDevice, res.wide_stream);
        if (e != hipSuccess) return batch_fail(c0, e, "executor table upload");
      }
      plan_stale = false;
    }
    // partitions of every active job, each on its own stream
    int32_t m = 0;
    for (int32_t i = 0; i < count; ++i) {
      if (!active[i]) continue;
      pcdn_ctx* c = runs[i].c;
      HIPCHK(c, hipGraphLaunch(c->graph_pre, c->stream));
      HIPCHK(c, hipEventRecord(res.pre_done[i], c->stream));
      hipStream_t group = narrow[i] ? res.narrow_stream : res.wide_stream;
      HIPCHK(c, hipStreamWaitEvent(group, res.pre_done[i], 0));
      if (narrow[i]) {
        const int64_t nb = (c->p + runs[i].P - 1) / runs[i].P;
        res.htab[m++] = make_narrow_args(c, runs[i].o, c->idx0, c->p, runs[i].P, 0, nb, nullptr);
      }
      count_outer(c, runs[i].o, runs[i].P, 1);
    }
    // single-workgroup jobs: one launch, then each job's stopping sweep
    if (m > 0) {
      hipError_t e = hipMemcpyAsync(res.dtab, res.htab, sizeof(NarrowArgs) * m,
                                    hipMemcpyHostToDevice, res.narrow_stream);
      if (e != hipSuccess) return batch_fail(c0, e, "batch table upload");
      e = launch_narrow_multi(res.dtab, m, res.narrow_stream);
      if (e != hipSuccess) return batch_fail(c0, e, "multi-problem launch");
      e = hipEventRecord(res.fused_done, res.narrow_stream);
      if (e != hipSuccess) return batch_fail(c0, e, "event record");
      for (int32_t i = 0; i < count; ++i) {
        if (!active[i] || !narrow[i]) continue;
        pcdn_ctx* c = runs[i].c;
        HIPCHK(c, hipStreamWaitEvent(c->stream, res.fused_done, 0));
        HIPCHK(c, hipGraphLaunch(c->graph_post, c->stream));
        HIPCHK(c, hipMemcpyAsync(c->hscal, c->scal, sizeof(double), hipMemcpyDeviceToHost,
                                 c->stream));
      }
    }
    // multi-kernel jobs: every bundle and stopping sweep in lock-step launches
    if (!plan.jobs.empty()) {
      for (size_t st = 0; st < plan.count.size(); ++st) {
        const hipError_t e = launch_exec(dtasks + plan.task_off[st], dfirst + plan.first_off[st],
                                         plan.count[st], plan.blocks[st], res.wide_stream);
        if (e != hipSuccess) return batch_fail(c0, e, "executor launch");
      }
      hipError_t e = launch_gather(dsrc, res.dG, (int)plan.jobs.size(), res.wide_stream);
      if (e != hipSuccess) return batch_fail(c0, e, "gather");
      e = hipMemcpyAsync(res.hG, res.dG, sizeof(double) * plan.jobs.size(),
                         hipMemcpyDeviceToHost, res.wide_stream);
      if (e != hipSuccess) return batch_fail(c0, e, "gather copy");
    }
    // the staging tables and every pinned result are reused next round
    hipError_t e = hipStreamSynchronize(res.narrow_stream);
    if (e == hipSuccess) e = hipStreamSynchronize(res.wide_stream);
    if (e != hipSuccess) return batch_fail(c0, e, "round");
    for (size_t k = 0; k < plan.jobs.size(); ++k) runs[plan.jobs[k]].c->hscal[0] = res.hG[k];
    for (int32_t i = 0; i < count; ++i) {
      if (!active[i]) continue;
      pcdn_ctx* c = runs[i].c;
      HIPCHK(c, hipStreamSynchronize(c->stream));
      const int rc = solve_note_outer(runs[i], c->hscal[0]);
      if (rc) return rc;
      active[i] = !runs[i].converged && runs[i].outer < runs[i].o.max_outer;
      if (!active[i] && !narrow[i]) plan_stale = true;
    }
  }
  int first_err = PCDN_OK;
  for (int32_t i = 0; i < count; ++i) {
    const int rc = solve_end(runs[i], jobs[i].w_out, jobs[i].info);
    jobs[i].status = rc;
    if (rc < 0 && first_err == PCDN_OK) first_err = rc;
  }
  return first_err;
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
    rc = solve_begin(r);
    if (rc) return rc;
    while (!r.converged && r.outer < r.o.max_outer) {
      rc = run_outer(c, r.o, P, r.outer, 1);
      if (rc) return rc;
      double G = 0.0;
      rc = read_scalar(c, 0, &G);
      if (rc) return rc;
      rc = solve_note_outer(r, G);
      if (rc) return rc;
    }
    rc = solve_end(r, W_out ? W_out + (size_t)k * (size_t)c->p : nullptr,
                   infos ? infos + k : nullptr);
    if (rc < 0) return rc;
    if (rc == PCDN_NOT_CONVERGED) status = rc;
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
  // the paper's pilot start: about 5% of the features
  const int64_t P0 = std::max<int64_t>(1, std::llround(0.05 * (double)p));
  std::vector<int64_t> cands;
  for (int k = -3; k <= 2; ++k) {
    const double v = (double)P0 * std::pow(4.0, k);
    const int64_t P = std::min<int64_t>(p, std::max<int64_t>(1, std::llround(v)));
    if (std::find(cands.begin(), cands.end(), P) == cands.end()) cands.push_back(P);
  }
  // a target below the rounding floor cannot be predicted; eps = 0 tunes for 1e-12
  const double eps_eff = std::max(eps, 1e-12);
  constexpr int kPilot = 3;
  using clock = std::chrono::steady_clock;
  double best = INFINITY, best_speed = -1.0;
  for (const int64_t P : cands) {
    SolveRun r;
    r.o = o;
    r.c = c;
    r.C = C;
    r.P = P;
    r.eps = eps;
    r.loss = loss;
    rc = solve_begin(r);
    if (rc) return rc;
    pcdn_tune_point& tp = out->tried[out->n_tried++];
    tp.P = P;
    tp.schedule = use_narrow(c, o, P) ? PCDN_SCHED_NARROW : PCDN_SCHED_WIDE;
    if (r.converged) {  // w = 0 (or the warm start) already meets the rule
      tp.predicted_seconds = 0.0;
      out->P = P;
      out->schedule = tp.schedule;
      out->predicted_seconds = 0.0;
      return PCDN_OK;
    }
    // iteration 1 pays for graph capture; iterations 2.. are timed
    double G1 = 0.0, timed = 0.0, total = 0.0;
    for (int k = 0; k < kPilot && !r.converged && r.outer < o.max_outer; ++k) {
      const auto t0 = clock::now();
      rc = run_outer(c, o, P, r.outer, 1);
      if (rc) return rc;
      double G = 0.0;
      rc = read_scalar(c, 0, &G);
      if (rc) return rc;
      rc = solve_note_outer(r, G);
      if (rc) return rc;
      const double dt = std::chrono::duration<double>(clock::now() - t0).count();
      total += dt;
      if (k == 0)
        G1 = G;
      else
        timed += dt;
    }
    tp.outer = r.outer;
    tp.sec_per_outer = r.outer > 1 ? timed / (r.outer - 1) : total;
    tp.rate = (r.outer > 1 && G1 > 0.0 && r.G > 0.0) ? (std::log(G1) - std::log(r.G)) / (r.outer - 1)
                                                    : 0.0;
    if (r.G <= eps_eff * r.G0) {
      tp.predicted_seconds = total;
    } else if (tp.rate > 0.0) {
      const double more = std::log(r.G / (eps_eff * r.G0)) / tp.rate;
      tp.predicted_seconds = total + more * tp.sec_per_outer;
    } else {
      tp.predicted_seconds = INFINITY;
    }
    // ties (all unpredictable) go to the fastest decay per second
    const double speed = tp.sec_per_outer > 0.0 ? tp.rate / tp.sec_per_outer : 0.0;
    if (tp.predicted_seconds < best ||
        (!std::isfinite(best) && !std::isfinite(tp.predicted_seconds) && speed > best_speed)) {
      best = tp.predicted_seconds;
      best_speed = speed;
      out->P = P;
      out->schedule = tp.schedule;
      out->predicted_seconds = tp.predicted_seconds;
    }
  }
  return PCDN_OK;
}
