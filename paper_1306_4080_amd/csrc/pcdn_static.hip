// pcdn_solve_static: pcdn_solve for callers that cannot allocate device
// memory.  Every buffer a context would allocate (the retained quantities,
// the per-slot outputs, the partition and the copy working arrays, the
// partition-order and bundle-row-order copies of X, the CSR copy, the
// reduction partials, the counters) is carved out of one file-scope device
// array, `scratch`, whose device address is looked up once per device.  The
// caller's device arrays hold X, y and w.  The kernels are those of
// pcdn_solve; only the CSR copy, the input checks and the largest row
// 1-norm, which pcdn_load_csc forms on the host, are formed here on the
// device.  Calls on one device share its array: calls that overlap on one
// device race.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>

#include "pcdn_host.h"

using namespace pcdn;
using namespace pcdn::host;

namespace {

// The workspace: at most this many bytes per device, held by every device
// the library runs on until the process ends.
constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;

// Host side of one device's workspace: the device address of `scratch` (set
// once, with the device current), the context the solve runs on, and the
// host records its reads land in (plain host memory: no pinned allocation).
struct StaticDevice {
  bool ready = false;
  unsigned char* base = nullptr;
  pcdn_ctx ctx;
  Stats hstats{};
  double hscal[8] = {};
  StepState hst{};
  IterState hiter{};
  int32_t hheavy[kHeavyCap + 1] = {};
};
StaticDevice g_dev[kMaxDevices];

// ---------------------------------------------------------------------------
// device-side input checks and the CSR copy
// ---------------------------------------------------------------------------
// Error flags (bits): 1 col_ptr, 2 row index out of range or not increasing,
// 4 non-finite value, 8 label not +-1.
__global__ void k_check_colptr(const int64_t* cp, int64_t p, int64_t nnz, int* err) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j == 0 && (cp[0] != 0 || cp[p] != nnz)) atomicOr(err, 1);
  if (j < p && cp[j + 1] < cp[j]) atomicOr(err, 1);
}

// Column of every nonzero (one wavefront per column; needs a checked col_ptr).
__global__ void k_col_ids(const int64_t* cp, int64_t p, int32_t* ccol) {
  const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t nwaves = (int64_t)gridDim.x * blockDim.x / kWave;
  for (int64_t j = wave; j < p; j += nwaves)
    for (int64_t k = cp[j] + lane; k < cp[j + 1]; k += kWave) ccol[k] = (int32_t)j;
}

__global__ void k_check_entries(const int64_t* cp, const int32_t* ri, const float* v,
                                const int32_t* ccol, int64_t n, int64_t nnz, int* err) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= nnz) return;
  const int32_t r = ri[k];
  if (r < 0 || r >= n) atomicOr(err, 2);
  if (k > cp[ccol[k]] && ri[k - 1] >= r) atomicOr(err, 2);
  if (!isfinite(v[k])) atomicOr(err, 4);
}

__global__ void k_check_labels(const int8_t* y, int64_t n, int* err) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n && y[i] != 1 && y[i] != -1) atomicOr(err, 8);
}

// Sort keys (rows) and payloads (positions) of the nonzeros in CSC order.
__global__ void k_csr_keys(const int32_t* ri, int64_t nnz, uint32_t* keys, int32_t* idx) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k < nnz) {
    keys[k] = (uint32_t)ri[k];
    idx[k] = (int32_t)k;
  }
}

// After the stable sort by row: row, column and value of each nonzero in
// CSR order (rows ascending, columns ascending inside a row).
__global__ void k_csr_gather(const uint32_t* keys, const int32_t* idx, const int32_t* ccol,
                             const float* v, int64_t nnz, int32_t* rr, int32_t* rc, float* rv) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k < nnz) {
    const int32_t s = idx[k];
    rr[k] = (int32_t)keys[k];
    rc[k] = ccol[s];
    rv[k] = v[s];
  }
}

// Row pointers from the sorted rows: position k starts every row in
// (rr[k-1], rr[k]] (rows without nonzeros start where the next row does).
__global__ void k_row_ptr(const int32_t* rr, int64_t nnz, int64_t n, int64_t* rp) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k > nnz) return;
  const int64_t prev = k > 0 ? rr[k - 1] : -1;
  const int64_t cur = k < nnz ? rr[k] : n;
  for (int64_t r = prev + 1; r <= cur; ++r) rp[r] = k;
}

// max_i sum_j |x_ij|: each row summed in column order (as the host does in
// pcdn_load_csc), then the largest in one block.
__global__ void k_row_l1(const int64_t* rp, const float* rv, int64_t n, double* l1) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int64_t k = rp[i]; k < rp[i + 1]; ++k) s += fabs((double)rv[k]);
  l1[i] = s;
}

__global__ __launch_bounds__(256) void k_max(const double* x, int64_t n, double* out) {
  __shared__ double m[256];
  double v = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) v = fmax(v, x[i]);
  m[threadIdx.x] = v;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) m[threadIdx.x] = fmax(m[threadIdx.x], m[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = m[0];
}

__global__ void k_zero_words(unsigned long long* a, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0ull;
}

unsigned grid_of(int64_t items) { return (unsigned)std::max<int64_t>(1, (items + 255) / 256); }

// ---------------------------------------------------------------------------
// workspace layout: the buffers of pcdn_create and pcdn_load_csc, 256-byte
// aligned, in one pass that only adds up the sizes (base == nullptr) or also
// assigns the pointers
// ---------------------------------------------------------------------------
struct Carve {
  unsigned char* base;
  size_t off = 0;
  template <class T>
  T* take(int64_t count) {
    off = (off + 255) & ~(size_t)255;
    T* p = base ? (T*)(base + off) : nullptr;
    off += (size_t)std::max<int64_t>(count, 1) * sizeof(T);
    return p;
  }
};

// Extra device buffers of the static path: error flags, the largest row
// 1-norm, and the column of each nonzero (CSR construction).
struct StaticExtra {
  int* err = nullptr;
  double* xrow = nullptr;
  int32_t* ccol = nullptr;
};

size_t carve(unsigned char* base, pcdn_ctx* c, StaticExtra* x, int64_t n, int64_t p,
             int64_t nnz) {
  Carve k{base};
  pcdn_ctx tmp;
  pcdn_ctx* t = c ? c : &tmp;
  StaticExtra xt;
  StaticExtra* e = x ? x : &xt;
  const int64_t hist_p = radix_hist_ints(p);
  const int64_t hist_nnz = radix_hist_ints(nnz);      // the sort by row
  const int64_t br_m = std::max(br_hist_ints(nnz), hist_nnz);
  const int64_t scan_m = std::max({scan_tmp_ints(hist_p), scan_tmp_ints(p), scan_tmp_ints(br_m)});
  t->iter = k.take<IterState>(1);
  t->st = k.take<StepState>(1);
  t->stats = k.take<Stats>(1);
  t->scal = k.take<double>(8);
  t->sum_part = k.take<double>(kSumGrid);
  t->stop_part = k.take<double>(4 * kSumGrid);
  t->heavy = k.take<int32_t>(kHeavyCap + 1);
  t->cache = k.take<double>(n);
  t->rw = k.take<double2>(n);
  t->dtx = k.take<double>(n);
  t->tmp_n = k.take<double>(n);
  t->tmp_p = k.take<double>(p);
  t->g = k.take<double>(p);
  t->h = k.take<double>(p);
  t->d = k.take<double>(p);
  t->dterm = k.take<double>(p);
  t->keys0 = k.take<uint32_t>(p);
  t->keys1 = k.take<uint32_t>(p);
  t->idx0 = k.take<int32_t>(p);
  t->idx1 = k.take<int32_t>(p);
  t->hist = k.take<int32_t>(hist_p);
  t->scan_tmp = k.take<int32_t>(scan_m + 1);
  t->nch = k.take<int32_t>(p);
  t->rfirst = k.take<int32_t>(nnz / kPermW + 2);
  t->psrc = k.take<int64_t>(p);
  t->part_len = 2 * ((nnz + kWave - 1) / kWave) + 2;
  t->part = k.take<double2>(t->part_len);
  t->pri = k.take<int32_t>(nnz);
  t->pv = k.take<float>(nnz);
  t->pslot = k.take<int32_t>(nnz);
  t->poff = k.take<int64_t>(p + 1);
  t->pw = k.take<double>(p);
  t->off32 = k.take<int32_t>(p + 1);
  t->plid = k.take<uint16_t>(nnz);
  t->pR = k.take<int32_t>(p + 1);
  t->ls_part = k.take<double>((int64_t)kRowsGridMax * (4 * kQMax + 3));
  t->act = k.take<double>(p);
  t->rp = k.take<int64_t>(n + 1);
  t->rr = k.take<int32_t>(nnz);
  t->rc = k.take<int32_t>(nnz);
  t->rv = k.take<float>(nnz);
  t->islot = k.take<int32_t>(p);
  t->br_row = k.take<int32_t>(nnz);
  t->br_slot = k.take<int32_t>(nnz);
  t->br_val = k.take<float>(nnz);
  t->bt_row = k.take<int32_t>(nnz);
  t->bt_slot = k.take<int32_t>(nnz);
  t->bt_val = k.take<float>(nnz);
  t->br_hist = k.take<int32_t>(br_m);
  t->u_cnt = k.take<int32_t>((nnz + kRangeW - 1) / kRangeW + 1);
  t->u_row = k.take<int32_t>(nnz + kRangeW);
  t->u_dtx = k.take<double>(nnz + kRangeW);
  t->ccol = k.take<int32_t>(nnz);
  e->err = k.take<int>(1);
  e->xrow = k.take<double>(1);
  e->ccol = t->ccol;
  return k.off;
}

// Errors are reported through pcdn_last_error(NULL), as pcdn_create's are.
int static_fail(int code, const char* msg) {
  global_error() = msg;
  return code;
}

// Device address of this device's `scratch`, looked up once with the device
// current.
int static_setup(int dev, StaticDevice** out) {
  StaticDevice& sd = g_dev[dev];
  if (!sd.ready) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      (void)hipGetLastError();
      global_error() = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
      return PCDN_E_DEVICE;
    }
    sd.base = (unsigned char*)ptr;
    // error messages then fit without a host allocation
    sd.ctx.err.reserve(512);
    global_error().reserve(512);
    sd.ready = true;
  }
  *out = &sd;
  return PCDN_OK;
}

}  // namespace

namespace {

int solve_static(int device, hipStream_t stream, int64_t n, int64_t p, int64_t nnz,
                 const int64_t* col_ptr, const int32_t* row_idx, const float* val, const int8_t* y,
                 double C, int64_t P, double eps, int loss, const pcdn_opts* opts, double* w_out,
                 pcdn_info* info, pcdn_ctx** used) {
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0)
    return static_fail(PCDN_E_DEVICE, "no HIP device available");
  if (device < 0 || device >= ndev || device >= kMaxDevices)
    return static_fail(PCDN_E_ARG, "device index out of range");
  if (n < 1 || p < 1 || nnz < 0 || n >= (int64_t)1 << 31 || p >= (int64_t)1 << 31 ||
      nnz >= (int64_t)1 << 31)
    return static_fail(PCDN_E_ARG, "sizes out of range (need 1 <= n, p < 2^31, 0 <= nnz)");
  if (!col_ptr || !y || !w_out || (nnz > 0 && (!row_idx || !val)))
    return static_fail(PCDN_E_ARG, "null array");
  const size_t need = carve(nullptr, nullptr, nullptr, n, p, nnz);
  if (need > kScratchBytes) {
    char msg[160];
    std::snprintf(msg, sizeof msg,
                  "problem too large for the static workspace: needs %zu bytes, the limit is %zu",
                  need, kScratchBytes);
    return static_fail(PCDN_E_ARG, msg);
  }
  if (hipSetDevice(device) != hipSuccess) return static_fail(PCDN_E_DEVICE, "hipSetDevice failed");
  StaticDevice* sd = nullptr;
  int rc = static_setup(device, &sd);
  if (rc) return rc;
  pcdn_ctx* c = &sd->ctx;
  *used = c;
  // the context over the workspace and the caller's arrays
  c->device = device;
  c->stream = stream;
  c->own_stream = false;
  c->err.clear();
  c->use_graphs = false;  // instantiating a graph allocates
  c->prof.mask = 0;
  c->hc = pcdn_ctx::HostCounts();
  c->hscal = sd->hscal;
  c->hstats = &sd->hstats;
  c->hst = &sd->hst;
  c->hiter = &sd->hiter;
  c->hheavy = sd->hheavy;
  StaticExtra x;
  (void)carve(sd->base, c, &x, n, p, nnz);
  c->n = n;
  c->p = p;
  c->nnz = nnz;
  c->cp = const_cast<int64_t*>(col_ptr);
  // without nonzeros the caller's arrays may be NULL: kernels read element 0
  // of every array (see ldz), so point them at workspace buffers
  c->ri = nnz ? const_cast<int32_t*>(row_idx) : c->rr;
  c->v = nnz ? const_cast<float*>(val) : c->rv;
  c->y = const_cast<int8_t*>(y);
  c->w = w_out;
  // no top_len: k_split always launches (it does nothing without split
  // columns) and heavy bundles stay in the single workgroup
  c->loaded = false;
  c->has_state = false;
  hipStream_t s = c->stream;
  // zero what must start at zero (fill kernels: no memset nodes)
  hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(256), 0, s, (unsigned long long*)c->iter,
                     (int64_t)(sizeof(IterState) / 8));
  hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(256), 0, s, (unsigned long long*)c->stats,
                     (int64_t)(sizeof(Stats) / 8));
  c->range_seen = 0;
  hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(256), 0, s, (unsigned long long*)x.err, (int64_t)1);
  hipLaunchKernelGGL(k_zero_words, dim3(grid_of(n)), dim3(256), 0, s, (unsigned long long*)c->dtx, n);
  // input checks: col_ptr first (the others index through it)
  hipLaunchKernelGGL(k_check_colptr, dim3(grid_of(p)), dim3(256), 0, s, col_ptr, p, nnz, x.err);
  hipLaunchKernelGGL(k_check_labels, dim3(grid_of(n)), dim3(256), 0, s, y, n, x.err);
  int herr = 0;
  HIPCHK(c, hipMemcpyAsync(&herr, x.err, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  if (herr & 1) return fail(c, PCDN_E_CSC, "col_ptr must start at 0, end at nnz and not decrease");
  if (herr & 8) return fail(c, PCDN_E_CSC, "a label is not +1/-1");
  if (nnz > 0) {
    hipLaunchKernelGGL(k_col_ids, dim3(grid_of(p * (int64_t)kWave)), dim3(256), 0, s, col_ptr, p,
                       x.ccol);
    hipLaunchKernelGGL(k_check_entries, dim3(grid_of(nnz)), dim3(256), 0, s, col_ptr, row_idx, val,
                       x.ccol, n, nnz, x.err);
    HIPCHK(c, hipMemcpyAsync(&herr, x.err, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    if (herr & 2) return fail(c, PCDN_E_CSC, "row indices out of range or not strictly increasing in a column");
    if (herr & 4) return fail(c, PCDN_E_CSC, "non-finite value");
    // CSR copy: stable sort of the nonzeros by row (the bundle-row order's
    // buffers hold the keys and payloads meanwhile)
    uint32_t* k0 = (uint32_t*)c->br_row;
    int32_t* i0 = c->br_slot;
    uint32_t* k1 = (uint32_t*)c->bt_row;
    int32_t* i1 = c->bt_slot;
    hipLaunchKernelGGL(k_csr_keys, dim3(grid_of(nnz)), dim3(256), 0, s, row_idx, nnz, k0, i0);
    HIPCHK(c, launch_radix_sort(k0, i0, k1, i1, nnz, c->br_hist, c->scan_tmp, s));
    hipLaunchKernelGGL(k_csr_gather, dim3(grid_of(nnz)), dim3(256), 0, s, k0, i0, x.ccol, val, nnz,
                       c->rr, c->rc, c->rv);
  }
  hipLaunchKernelGGL(k_row_ptr, dim3(grid_of(nnz + 1)), dim3(256), 0, s, c->rr, nnz, n, c->rp);
  hipLaunchKernelGGL(k_row_l1, dim3(grid_of(n)), dim3(256), 0, s, c->rp, c->rv, n, c->tmp_n);
  hipLaunchKernelGGL(k_max, dim3(1), dim3(256), 0, s, c->tmp_n, n, x.xrow);
  HIPCHK(c, hipGetLastError());
  double xrow = 0.0;
  HIPCHK(c, hipMemcpyAsync(&xrow, x.xrow, sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  c->xrow = xrow;
  c->loaded = true;
  // pcdn_solve's loop (direct launches, one read of the stopping norm per
  // outer iteration)
  SolveRun r;
  rc = check_solve_args(c, C, P, eps, loss, opts, &r.o);
  if (rc) return rc;
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
  return solve_end(r, nullptr, info);
}

}  // namespace

extern "C" int pcdn_solve_static(int device, void* hip_stream, int64_t n, int64_t p, int64_t nnz,
                                 const int64_t* col_ptr, const int32_t* row_idx, const float* val,
                                 const int8_t* y, double C, int64_t P, double eps, int loss,
                                 const pcdn_opts* opts, double* w_out, pcdn_info* info) {
  pcdn_ctx* used = nullptr;
  const int rc = solve_static(device, (hipStream_t)hip_stream, n, p, nnz, col_ptr, row_idx, val, y,
                              C, P, eps, loss, opts, w_out, info, &used);
  if (rc < 0 && used) global_error() = used->err;  // within the reserved capacity
  return rc;
}
