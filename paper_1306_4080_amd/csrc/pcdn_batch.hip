// Drivers over several solves on one device: independent problems advanced
// together (pcdn_solve_batch) and the warm-started regularisation path
// (pcdn_solve_path).  Each problem follows exactly the sequence of kernels
// pcdn_solve would run for it; only the interleaving across problems differs.
#include <cmath>
#include <string>
#include <vector>

#include "pcdn_host.h"

using namespace pcdn;
using namespace pcdn::host;

namespace {

// Device resources of one pcdn_solve_batch call, released on every exit.
struct BatchRes {
  int device = 0;
  hipStream_t stream = nullptr;
  hipEvent_t fused_done = nullptr;
  std::vector<hipEvent_t> pre_done;
  NarrowArgs* dtab = nullptr;   // device table of the fused launch
  NarrowArgs* htab = nullptr;   // pinned staging for it
  ~BatchRes() {
    (void)hipSetDevice(device);
    if (stream) (void)hipStreamSynchronize(stream);
    for (hipEvent_t e : pre_done)
      if (e) (void)hipEventDestroy(e);
    if (fused_done) (void)hipEventDestroy(fused_done);
    if (dtab) (void)hipFree(dtab);
    if (htab) (void)hipHostFree(htab);
    if (stream) (void)hipStreamDestroy(stream);
  }
};

// Device error of the batch itself, reported on the first job's context.
int batch_fail(pcdn_ctx* c, hipError_t e, const char* what) {
  return fail(c, PCDN_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

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
    const int rc = check_solve_args(j.ctx, j.C, j.P, j.eps, j.loss, j.opts, &runs[i].o);
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
  pcdn_ctx* c0 = jobs[0].ctx;
  BatchRes res;
  res.device = c0->device;
  HIPCHK(c0, hipSetDevice(res.device));
  HIPCHK(c0, hipStreamCreateWithFlags(&res.stream, hipStreamNonBlocking));
  HIPCHK(c0, hipEventCreateWithFlags(&res.fused_done, hipEventDisableTiming));
  res.pre_done.assign(count, nullptr);
  for (int32_t i = 0; i < count; ++i)
    HIPCHK(c0, hipEventCreateWithFlags(&res.pre_done[i], hipEventDisableTiming));

  // set-up: reference norm and w per job, graphs, iteration record
  std::vector<char> narrow(count, 0), active(count, 0);
  int32_t n_narrow = 0;
  for (int32_t i = 0; i < count; ++i) {
    SolveRun& r = runs[i];
    int rc = solve_begin(r);
    if (rc) return rc;
    narrow[i] = use_narrow(r.c, r.o, r.P) ? 1 : 0;
    n_narrow += narrow[i];
    rc = narrow[i] ? ensure_split_graphs(r.c, r.o, r.P) : ensure_graph(r.c, r.o, r.P);
    if (rc) return rc;
    rc = set_iter(r.c, r.o.seed, 0);
    if (rc) return rc;
    active[i] = !r.converged && r.outer < r.o.max_outer;
  }
  if (n_narrow > 0) {
    hipError_t e = hipMalloc((void**)&res.dtab, sizeof(NarrowArgs) * n_narrow);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(c0, PCDN_E_OOM, "device allocation failed for the batch table");
    }
    e = hipHostMalloc((void**)&res.htab, sizeof(NarrowArgs) * n_narrow);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(c0, PCDN_E_OOM, "pinned allocation failed for the batch table");
    }
  }

  // rounds: one outer iteration of every active job
  for (;;) {
    int32_t m = 0, live = 0;
    for (int32_t i = 0; i < count; ++i) {
      if (!active[i]) continue;
      ++live;
      pcdn_ctx* c = runs[i].c;
      if (narrow[i]) {
        HIPCHK(c, hipGraphLaunch(c->graph_pre, c->stream));
        HIPCHK(c, hipEventRecord(res.pre_done[i], c->stream));
        HIPCHK(c, hipStreamWaitEvent(res.stream, res.pre_done[i], 0));
        const int64_t nb = (c->p + runs[i].P - 1) / runs[i].P;
        res.htab[m++] = make_narrow_args(c, runs[i].o, c->idx0, c->p, runs[i].P, 0, nb, nullptr);
      } else {
        HIPCHK(c, hipGraphLaunch(c->graph, c->stream));
        HIPCHK(c, hipMemcpyAsync(c->hscal, c->scal, sizeof(double), hipMemcpyDeviceToHost,
                                 c->stream));
      }
      count_outer(c, runs[i].o, runs[i].P, 1);
    }
    if (live == 0) break;
    if (m > 0) {
      hipError_t e = hipMemcpyAsync(res.dtab, res.htab, sizeof(NarrowArgs) * m,
                                    hipMemcpyHostToDevice, res.stream);
      if (e != hipSuccess) return batch_fail(c0, e, "batch table upload");
      e = launch_narrow_multi(res.dtab, m, res.stream);
      if (e != hipSuccess) return batch_fail(c0, e, "multi-problem launch");
      e = hipEventRecord(res.fused_done, res.stream);
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
    // the staging table and every pinned result are reused next round
    HIPCHK(c0, hipStreamSynchronize(res.stream));
    for (int32_t i = 0; i < count; ++i) {
      if (!active[i]) continue;
      pcdn_ctx* c = runs[i].c;
      HIPCHK(c, hipStreamSynchronize(c->stream));
      const int rc = solve_note_outer(runs[i], c->hscal[0]);
      if (rc) return rc;
      active[i] = !runs[i].converged && runs[i].outer < runs[i].o.max_outer;
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
