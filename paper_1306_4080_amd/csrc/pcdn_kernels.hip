// HIP kernels of the PCDN bundle sweep for gfx950 (CDNA4, 64-wide wavefronts).
//
// The work is sparse gather/scatter at well under one flop per byte, so it is
// bound by memory bandwidth and latency, not by the matrix cores: no MFMA here.
// Every sum is FP64 and deterministic for a fixed launch shape: g_j, h_j,
// the line-search sums and the stopping norm are fixed-order tree sums, and
// d^T x_i is a fixed-order row sum (multi-kernel schedule) or an integer
// fixed-point sum, exact in any order (single workgroup), so a solve gives
// the same bits on every run, alone or beside other problems.
#include <cstring>
#include <utility>

#include "pcdn_device.h"

namespace pcdn {

namespace {

// ---------------------------------------------------------------------------
// wavefront / block reductions
// ---------------------------------------------------------------------------
// One DPP step on an FP64 value (two 32-bit halves); lanes without a source
// (outside the row, or in a masked row) read +0.0.
template <int CTRL, int ROW_MASK, int BANK_MASK>
__device__ inline double dpp_f64(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  int lo = (int)(unsigned)(b & 0xffffffffull);
  int hi = (int)(unsigned)(b >> 32);
  lo = __builtin_amdgcn_update_dpp(0, lo, CTRL, ROW_MASK, BANK_MASK, true);
  hi = __builtin_amdgcn_update_dpp(0, hi, CTRL, ROW_MASK, BANK_MASK, true);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Sum over the 64 lanes of a wavefront, the same value in every lane, in a
// fixed order: prefix sums inside each 16-lane row (row_shr 1, 2, 4, 8), then
// row 0 into row 1 and row 2 into row 3 (row_bcast15), then rows 0-1 into
// rows 2-3 (row_bcast31); lane 63 holds the total.
__device__ inline double wave_sum(double v) {
  v += dpp_f64<0x111, 0xf, 0xf>(v);
  v += dpp_f64<0x112, 0xf, 0xf>(v);
  v += dpp_f64<0x114, 0xf, 0xf>(v);
  v += dpp_f64<0x118, 0xf, 0xf>(v);
  v += dpp_f64<0x142, 0xa, 0xf>(v);
  v += dpp_f64<0x143, 0xc, 0xf>(v);
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b & 0xffffffffull), 63);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), 63);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// One step of a segmented inclusive scan over a wavefront whose keys do not
// decrease along the lanes: add the source lane's running sums when it holds
// the same key (a lane without a source reads key -1, which no valid lane has).
template <int CTRL, int ROW_MASK>
__device__ inline void seg_scan_step(double& g, double& h, int32_t key) {
  const int32_t k2 = __builtin_amdgcn_update_dpp(-1, key, CTRL, ROW_MASK, 0xf, false);
  const double g2 = dpp_f64<CTRL, ROW_MASK, 0xf>(g);
  const double h2 = dpp_f64<CTRL, ROW_MASK, 0xf>(h);
  if (k2 == key) {
    g += g2;
    h += h2;
  }
}

// Segmented inclusive scan of (g, h) by key: the same step sequence as
// wave_sum, each step gated on equal keys.  Keys must not decrease with the
// lane index, so equal keys are contiguous.
__device__ inline void seg_scan(double& g, double& h, int32_t key) {
  seg_scan_step<0x111, 0xf>(g, h, key);
  seg_scan_step<0x112, 0xf>(g, h, key);
  seg_scan_step<0x114, 0xf>(g, h, key);
  seg_scan_step<0x118, 0xf>(g, h, key);
  seg_scan_step<0x142, 0xa>(g, h, key);
  seg_scan_step<0x143, 0xc>(g, h, key);
}

// Segmented inclusive scan of one value (the step sequence of seg_scan).
template <int CTRL, int ROW_MASK>
__device__ inline void seg_scan1_step(double& g, int32_t key) {
  const int32_t k2 = __builtin_amdgcn_update_dpp(-1, key, CTRL, ROW_MASK, 0xf, false);
  const double g2 = dpp_f64<CTRL, ROW_MASK, 0xf>(g);
  if (k2 == key) g += g2;
}

__device__ inline void seg_scan1(double& g, int32_t key) {
  seg_scan1_step<0x111, 0xf>(g, key);
  seg_scan1_step<0x112, 0xf>(g, key);
  seg_scan1_step<0x114, 0xf>(g, key);
  seg_scan1_step<0x118, 0xf>(g, key);
  seg_scan1_step<0x142, 0xa>(g, key);
  seg_scan1_step<0x143, 0xc>(g, key);
}

// Key of the next lane (wave_shl1); lane 63 reads -2.
__device__ inline int32_t next_lane_key(int32_t key) {
  return __builtin_amdgcn_update_dpp(-2, key, 0x130, 0xf, 0xf, false);
}

__device__ inline int lane_id() { return threadIdx.x & (kWave - 1); }
__device__ inline int wave_in_block() { return threadIdx.x / kWave; }

// Sum over a 256-thread block in a fixed order; every thread gets the result.
__device__ inline double block_sum(double v, double* lds4) {
  v = wave_sum(v);
  if (lane_id() == 0) lds4[wave_in_block()] = v;
  __syncthreads();
  const double r = ((lds4[0] + lds4[1]) + lds4[2]) + lds4[3];
  __syncthreads();
  return r;
}

// p[i] when ok, else def, with the load itself unconditional (index 0
// stands in for i; every array has at least one element): a conditional
// load ends its basic block and the wavefront then waits for it before the
// next load issues, which serialises the loads that should overlap.
template <class T>
__device__ __forceinline__ T ldz(const T* p, bool ok, int64_t i, T def) {
  const T x = p[ok ? i : 0];
  return ok ? x : def;
}

// Wave-uniform value as a scalar (lets descriptor loads become scalar loads).
__device__ inline int64_t uniform(int64_t x) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(uint64_t)x);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)x >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// ---------------------------------------------------------------------------
// counter-based generator: SplitMix64 (Steele, Lea, Flood 2014): the state
// walks by the golden-ratio constant and each output is the state run through
// the published 64-bit finaliser.
// ---------------------------------------------------------------------------
__device__ inline uint64_t splitmix_out(uint64_t state) {
  uint64_t z = state;
  z ^= z >> 30;
  z *= 0xBF58476D1CE4E5B9ull;
  z ^= z >> 27;
  z *= 0x94D049BB133111EBull;
  z ^= z >> 31;
  return z;
}

// ---------------------------------------------------------------------------
// loss pieces (Sec. 2 eqs. (2)-(3); Sec. 3.1)
// ---------------------------------------------------------------------------
// sigma(z) and 1 - sigma(z) from E = e^z with one division, exact at E = 0
// and E = inf: s0 = 1 - sigma(z) = 1/(1+E), s1 = sigma(z) = E s0.
__device__ inline void logistic_weights(double E, double& s0, double& s1) {
  s0 = 1.0 / (1.0 + E);
  s1 = isinf(E) ? 1.0 : E * s0;
}

// Gradient / Hessian-diagonal contribution of one nonzero x of sample i with
// retained quantity c_i.  Logistic: for label y the misclassification weight
// 1 - tau(y z) is s0 (y = +1) or s1 (y = -1), and tau (1 - tau) = s0 s1.
template <int LOSS>
__device__ inline void grad_hess_term(double c, int yi, double x, double& gs, double& hs) {
  if (LOSS == kLogistic) {
    double s0, s1;
    logistic_weights(c, s0, s1);
    const double miss = yi > 0 ? s0 : s1;
    gs += (yi > 0 ? -miss : miss) * x;
    hs += (s0 * s1) * (x * x);
  } else {
    if (c > 0.0) {
      gs += (yi > 0 ? c : -c) * x;  // y_i b_i x_ij
      hs += x * x;
    }
  }
}

// The weights of a row's gradient and Hessian-diagonal terms, a function of
// its retained quantity c and label: x.x multiplies x_ij in g_j, x.y
// multiplies x_ij^2 in h_j (logistic: -(1 - tau) or its mirror and
// tau (1 - tau); SVM: y_i b_i and 1 on the active set, zeros off it).  They
// are kept beside the retained quantities (row_weights is applied wherever
// those change), so the sweeps gather one 16-byte value per nonzero instead
// of the retained quantity and the label; the terms are the same products
// as grad_hess_term's.
template <int LOSS>
__device__ inline double2 row_weights(double c, int yi) {
  if (LOSS == kLogistic) {
    double s0, s1;
    logistic_weights(c, s0, s1);
    return make_double2(yi > 0 ? -s0 : s1, s0 * s1);
  }
  return c > 0.0 ? make_double2(yi > 0 ? c : -c, 1.0) : make_double2(0.0, 0.0);
}

template <int LOSS>
__device__ inline void weighted_terms(double2 rw, double x, double& gs, double& hs) {
  if (LOSS == kLogistic) {
    gs += rw.x * x;
    hs += rw.y * (x * x);
  } else if (rw.y > 0.0) {
    gs += rw.x * x;
    hs += x * x;
  }
}

// Loss change of sample i when its margin w^T x_i grows by a (eq. (10)'s
// summand).  Logistic: log(1+e^{-y(z+a)}) - log(1+e^{-yz}); with m = -y a and
// tau = tau(y z) it is log(tau + (1 - tau) e^m), written for t = -|m| <= 0 as
// max(m, 0) + log(A + B e^t) with (A, B) = (tau, 1 - tau) if m <= 0 and
// (1 - tau, tau) if m > 0, so no exponential overflows.  log(A + B e^t) is
// log1p(u), u = B expm1(t), while u >= -1/2 (log1p through log with
// Goldberg's compensation, "What every computer scientist should know about
// floating-point arithmetic", Theorem 4), else log of the small sum
// A + B e^t.  One straight-line path: no divergent branches.
// SVM: max(0, b - y a)^2 - max(0, b)^2.
template <int LOSS>
__device__ inline double loss_delta(double c, int yi, double a) {
  if (LOSS == kLogistic) {
    double s0, s1;
    logistic_weights(c, s0, s1);
    const double tau = yi > 0 ? s1 : s0;
    const double one_minus_tau = yi > 0 ? s0 : s1;
    const double m = yi > 0 ? -a : a;
    const bool pos = m > 0.0;
    const double A = pos ? one_minus_tau : tau;
    const double B = pos ? tau : one_minus_tau;
    const double t = pos ? -m : m;
    const double u = B * expm1(t);
    const bool near_one = u >= -0.5;
    const double z = near_one ? 1.0 + u : A + B * exp(t);
    const double lz = log(z);
    const double r = near_one ? (z == 1.0 ? u : lz * (u / (z - 1.0))) : lz;
    return pos ? m + r : r;
  } else {
    const double bn = yi > 0 ? c - a : c + a;
    const double pn = bn > 0.0 ? bn : 0.0;
    const double po = c > 0.0 ? c : 0.0;
    return pn * pn - po * po;
  }
}

// Instrumentation of the Armijo decisions (no decision depends on it).
// The rounding scale of one loss change: what its computed value inherits
// from the rounding of its operands.  LR: the change itself plus |a| (the
// change moves by at most |da| for an error da in its argument); SVM: the
// two squares it is the difference of, plus 2 max(0, b - y a) |a|.
template <int LOSS>
__device__ inline double loss_delta_scale(double c, int yi, double a, double ld) {
  if (LOSS == kLogistic) return fabs(ld) + fabs(a);
  const double bn = yi > 0 ? c - a : c + a;
  const double pn = bn > 0.0 ? bn : 0.0;
  const double po = c > 0.0 ? c : 0.0;
  return pn * pn + po * po + 2.0 * pn * fabs(a);
}

// The rounding scale of R_j(w + s) - R_j(w): the magnitudes it is formed
// from, ra (|w + s| + |w|) and |rb s| (|w| + |s|/2).
__device__ inline double reg_change_scale(double w, double s, double ra, double rb) {
  return ra * (fabs(w + s) + fabs(w)) + fabs(rb * s) * (fabs(w) + 0.5 * fabs(s));
}

// |f - thr| / S for an Armijo test f <= thr, S = |thr| + scale (the summed
// rounding scales of the terms f is formed from, C included): the
// decision's distance from its threshold on the scale of the rounding
// errors of its two sides (+inf when S = 0).
__device__ inline double armijo_margin(double f, double thr, double abs_terms) {
  const double S = fabs(thr) + abs_terms;
  return S != 0.0 ? fabs(f - thr) / S : INFINITY;
}

// The range a retained quantity must stay in.  e^{w^T x_i} must be a
// positive normal double (|w^T x_i| below about 708): at 0, a subnormal or
// inf it no longer determines z_i, and 1/E or E/(1 + E) stop being exact.
// b_i = 1 - y_i w^T x_i must be finite.  A value outside is counted in
// Stats::range_leaves (the host reports it as a numeric error).
template <int LOSS>
__device__ inline bool in_range(double c) {
  if (LOSS == kLogistic) return c >= 2.2250738585072014e-308 && c <= 1.7976931348623157e308;
  return fabs(c) <= 1.7976931348623157e308;
}

template <int LOSS>
__device__ inline void count_range(double c, Stats* stats) {
  if (!in_range<LOSS>(c)) atomicAdd(&stats->range_leaves, 1ull);
}

// A retained quantity and its row's weights, with the range check.
template <int LOSS>
__device__ inline void store_retained(double* p, double2* rwp, double c, int yi, Stats* stats) {
  *p = c;
  *rwp = row_weights<LOSS>(c, yi);
  count_range<LOSS>(c, stats);
}

// Minimiser of g d + h d^2/2 + R(w + d) with R(u) = ra |u| + (rb/2) u^2
// (eq. (4) with the separable regulariser in place of |u|; for ra = 1,
// rb = 0 the soft-threshold form of eq. (5)).  u = w + d is > 0 exactly
// when g + ra < h w and < 0 exactly when g - ra > h w.
__device__ inline double newton_dir(double g, double h, double w, double ra, double rb) {
  const double hw = h * w;
  if (g + ra <= hw) return -(g + ra + rb * w) / (h + rb);
  if (g - ra >= hw) return -(g - ra + rb * w) / (h + rb);
  return -w;
}

// R_j(w + s) - R_j(w), the quadratic part as rb s (w + s/2).
__device__ inline double reg_change(double w, double s, double ra, double rb) {
  return ra * (fabs(w + s) - fabs(w)) + rb * s * (w + 0.5 * s);
}

// Minimum-norm subgradient of F in coordinate j.
__device__ inline double min_norm_subgradient(double g, double w, double ra, double rb) {
  const double G = g + rb * w;  // gradient of the smooth part
  if (w > 0.0) return G + ra;
  if (w < 0.0) return G - ra;
  if (G > ra) return G - ra;
  if (G < -ra) return G + ra;
  return 0.0;
}

// ---------------------------------------------------------------------------
// simple kernels
// ---------------------------------------------------------------------------
__global__ void k_fill(double* a, double v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    a[i] = v;
}

// Kernel bodies that the multi-problem executor also runs take their block
// index (and block count) as arguments; see k_exec.
__device__ __forceinline__ void perm_keys_body(const IterState* it, uint64_t seed, int64_t k,
                                               int64_t p, const double* act, uint32_t* keys,
                                               int32_t* idx, int64_t bid) {
  const int64_t j = bid * (int64_t)kBlock + threadIdx.x;
  if (it) {
    seed = it->seed;
    k = it->k;
  }
  // stream of outer iteration k: output k of the generator seeded with `seed`
  const uint64_t stream = splitmix_out(seed + (uint64_t)(k + 1) * 0x9E3779B97F4A7C15ull);
  if (j < p) {
    const uint64_t state = stream + (uint64_t)(j + 1) * 0x9E3779B97F4A7C15ull;
    uint32_t key = (uint32_t)(splitmix_out(state) >> 32);
    if (act) key = act[j] != 0.0 ? (key < 0xFFFFFFFFu ? key : 0xFFFFFFFEu) : 0xFFFFFFFFu;
    keys[j] = key;
    idx[j] = (int32_t)j;
  }
}

__global__ __launch_bounds__(kBlock) void k_perm_keys(const IterState* it, uint64_t seed,
                                                      int64_t k, int64_t p, const double* act,
                                                      uint32_t* keys, int32_t* idx) {
  perm_keys_body(it, seed, k, p, act, keys, idx, blockIdx.x);
}

// ---------------------------------------------------------------------------
// exclusive scan (int32), two launches: per-block scan with the block
// totals, then add-back of the sum of the earlier blocks' totals (each block
// forms its own).  A block of THREADS threads covers kScanTile items (PER
// = kScanTile / THREADS each): 1024-thread blocks in direct launches,
// kBlock-thread blocks in the multi-problem executor.  Integer sums, so
// every block size gives the same result.
// ---------------------------------------------------------------------------
constexpr int kScanThreads = 1024;
constexpr int kScanTile = 4096;

// Exclusive scan of one value per thread across a THREADS-thread block
// (lds holds THREADS / kWave + 1 ints).
template <int THREADS>
__device__ inline int32_t block_exclusive_scan(int32_t v, int32_t* lds, int32_t* total) {
  const int lane = lane_id(), wv = wave_in_block();
  int32_t x = v;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int32_t y = __shfl_up(x, o, kWave);
    if (lane >= o) x += y;
  }
  if (lane == kWave - 1) lds[wv] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t run = 0;
    for (int k = 0; k < THREADS / kWave; ++k) {
      const int32_t t = lds[k];
      lds[k] = run;
      run += t;
    }
    lds[THREADS / kWave] = run;
  }
  __syncthreads();
  const int32_t r = lds[wv] + x - v;
  *total = lds[THREADS / kWave];
  __syncthreads();
  return r;
}

template <int THREADS>
__device__ __forceinline__ void scan_blocks_body(const int32_t* in, int32_t* out, int64_t m,
                                                 int32_t* block_tot, int64_t bid) {
  constexpr int PER = kScanTile / THREADS;
  __shared__ int32_t lds[THREADS / kWave + 1];
  const int64_t base = bid * kScanTile + (int64_t)threadIdx.x * PER;
  int32_t v[PER];
  int32_t s = 0;
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    v[k] = base + k < m ? in[base + k] : 0;
    s += v[k];
  }
  int32_t tot;
  int32_t run = block_exclusive_scan<THREADS>(s, lds, &tot);
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    if (base + k < m) out[base + k] = run;
    run += v[k];
  }
  if (threadIdx.x == 0) block_tot[bid] = tot;
}

// Whole scan in one block when m <= 16 THREADS: thread t scans a contiguous
// chunk of ceil(m / THREADS) items (in and out may alias: a thread reads its
// whole chunk before the block scan's barriers and writes it afterwards).
template <int THREADS>
__device__ __forceinline__ void scan_small_body(const int32_t* in, int32_t* out, int64_t m) {
  __shared__ int32_t lds[THREADS / kWave + 1];
  const int64_t per = (m + THREADS - 1) / THREADS;
  const int64_t lo = (int64_t)threadIdx.x * per;
  const int64_t hi = lo + per < m ? lo + per : m;
  int32_t v[16];
  int32_t s = 0;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    v[k] = lo + k < hi ? in[lo + k] : 0;
    s += v[k];
  }
  int32_t tot;
  int32_t run = block_exclusive_scan<THREADS>(s, lds, &tot);
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    if (lo + k < hi) out[lo + k] = run;
    run += v[k];
  }
  if (threadIdx.x == 0) out[m] = tot;
}

// Tile bid adds the sum of the tiles before it, which it forms itself from
// the tiles' totals (a few hundred integers: no launch of its own to scan
// them); the last tile also writes the total at out[m].
template <int THREADS>
__device__ __forceinline__ void scan_add_body(int32_t* out, int64_t m, const int32_t* block_tot,
                                              int64_t nb, int64_t bid) {
  __shared__ int32_t lds[THREADS / kWave + 1];
  constexpr int PER = kScanTile / THREADS;
  int32_t s = 0;
  for (int64_t k = threadIdx.x; k < bid; k += THREADS) s += block_tot[k];
  int32_t add;
  (void)block_exclusive_scan<THREADS>(s, lds, &add);
  const int64_t base = bid * kScanTile + (int64_t)threadIdx.x * PER;
#pragma unroll
  for (int k = 0; k < PER; ++k)
    if (base + k < m) out[base + k] += add;
  if (bid == nb - 1 && threadIdx.x == 0) out[m] = add + block_tot[bid];
}

constexpr int64_t kScanSmall = 16 * kScanThreads;

__global__ __launch_bounds__(kScanThreads) void k_scan_blocks(const int32_t* in, int32_t* out,
                                                              int64_t m, int32_t* block_tot) {
  scan_blocks_body<kScanThreads>(in, out, m, block_tot, blockIdx.x);
}

__global__ __launch_bounds__(kScanThreads) void k_scan_small(const int32_t* in, int32_t* out,
                                                             int64_t m) {
  scan_small_body<kScanThreads>(in, out, m);
}

__global__ __launch_bounds__(kScanThreads) void k_scan_add(int32_t* out, int64_t m,
                                                           const int32_t* block_tot, int64_t nb) {
  scan_add_body<kScanThreads>(out, m, block_tot, nb, blockIdx.x);
}

// ---------------------------------------------------------------------------
// stable LSD radix sort of 32-bit keys with int32 payload, 8-bit digits.
// A tile is kSortTile = 2048 keys (256 threads x 8 rounds).  Stability inside a round
// comes from wavefront peer masks built with ballots, across waves and rounds
// from per-digit running offsets in LDS.
// ---------------------------------------------------------------------------
constexpr int kSortThreads = 256;
constexpr int kSortRounds = 8;
constexpr int kSortTile = kSortThreads * kSortRounds;

static_assert(kSortThreads == kBlock, "the executor runs the sort passes in kBlock-thread blocks");

__device__ __forceinline__ void radix_hist_body(const uint32_t* keys, int64_t p, int shift,
                                                int32_t* hist, int64_t ntiles, int64_t bid) {
  __shared__ int32_t cnt[256];
  cnt[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = bid * kSortTile;
  uint32_t k[kSortRounds];
#pragma unroll
  for (int r = 0; r < kSortRounds; ++r) {
    const int64_t i = base + r * kSortThreads + threadIdx.x;
    k[r] = ldz(keys, i < p, i, 0u);
  }
#pragma unroll
  for (int r = 0; r < kSortRounds; ++r) {
    const int64_t i = base + r * kSortThreads + threadIdx.x;
    if (i < p) atomicAdd(&cnt[(k[r] >> shift) & 255u], 1);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * ntiles + bid] = cnt[threadIdx.x];
}

__global__ __launch_bounds__(kSortThreads) void k_radix_hist(const uint32_t* keys, int64_t p,
                                                             int shift, int32_t* hist,
                                                             int64_t ntiles) {
  radix_hist_body(keys, p, shift, hist, ntiles, blockIdx.x);
}

__device__ __forceinline__ void radix_scatter_body(const uint32_t* kin, const int32_t* iin,
                                                   uint32_t* kout, int32_t* iout, int64_t p,
                                                   int shift, const int32_t* offs, int64_t ntiles,
                                                   int64_t bid) {
  __shared__ int32_t base_off[256];
  __shared__ int32_t wcnt[kWavesPerBlock][256];
  base_off[threadIdx.x] = offs[(int64_t)threadIdx.x * ntiles + bid];
  const int lane = lane_id(), wv = wave_in_block();
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int64_t tile = bid * kSortTile;
  for (int r = 0; r < kSortRounds; ++r) {
#pragma unroll
    for (int w = 0; w < kWavesPerBlock; ++w) wcnt[w][threadIdx.x] = 0;
    __syncthreads();
    const int64_t i = tile + r * kSortThreads + threadIdx.x;
    const bool valid = i < p;
    const uint32_t key = valid ? kin[i] : 0u;
    const uint32_t dig = (key >> shift) & 255u;
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (dig >> b) & 1u;
      const uint64_t bal = __ballot(bit);
      peers &= bit ? bal : ~bal;
    }
    const int rank = __popcll(peers & lt_mask);
    const bool leader = valid && ((peers & lt_mask) == 0);
    if (leader) wcnt[wv][dig] = __popcll(peers);
    __syncthreads();
    if (valid) {
      int32_t pos = base_off[dig] + rank;
      for (int w = 0; w < wv; ++w) pos += wcnt[w][dig];
      kout[pos] = key;
      iout[pos] = iin[i];
    }
    __syncthreads();
    int32_t add = 0;
#pragma unroll
    for (int w = 0; w < kWavesPerBlock; ++w) add += wcnt[w][threadIdx.x];
    base_off[threadIdx.x] += add;
    __syncthreads();
  }
}

__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(
    const uint32_t* kin, const int32_t* iin, uint32_t* kout, int32_t* iout, int64_t p, int shift,
    const int32_t* offs, int64_t ntiles) {
  radix_scatter_body(kin, iin, kout, iout, p, shift, offs, ntiles, blockIdx.x);
}

// The scatter pass of a standalone launch with the tile staged in LDS: the
// tile's keys are ranked as in radix_scatter_body, placed in digit order in
// LDS and stored from there, so a digit's run (8 keys of a tile on average)
// is written by consecutive threads.  The same positions, so the
// same output.  (The executor keeps radix_scatter_body: its LDS is shared by
// every task body.)
__global__ __launch_bounds__(kSortThreads) void k_radix_scatter_staged(
    const uint32_t* kin, const int32_t* iin, uint32_t* kout, int32_t* iout, int64_t p, int shift,
    const int32_t* offs, int64_t ntiles) {
  __shared__ int32_t gbase[256];  // output position of the tile's first key of each digit
  __shared__ int32_t lbase[256];  // the same inside the tile's sorted order
  __shared__ int32_t run_off[256];
  __shared__ int32_t wcnt[kWavesPerBlock][256];
  __shared__ int32_t lds_scan[kSortThreads / kWave + 1];
  __shared__ uint32_t s_key[kSortTile];
  __shared__ int32_t s_idx[kSortTile];
  const int64_t bid = blockIdx.x;
  const int lane = lane_id(), wv = wave_in_block();
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int64_t tile = bid * kSortTile;
  const int32_t tcount = (int32_t)(p - tile < kSortTile ? p - tile : kSortTile);
  gbase[threadIdx.x] = offs[(int64_t)threadIdx.x * ntiles + bid];
  wcnt[0][threadIdx.x] = 0;
  uint32_t key[kSortRounds];
  int32_t idx[kSortRounds];
#pragma unroll
  for (int r = 0; r < kSortRounds; ++r) {
    const int64_t i = tile + r * kSortThreads + threadIdx.x;
    const bool valid = i < p;
    key[r] = ldz(kin, valid, i, 0u);
    idx[r] = ldz(iin, valid, i, 0);
  }
  __syncthreads();
  // the tile's digit counts, then their exclusive scan
#pragma unroll
  for (int r = 0; r < kSortRounds; ++r)
    if (r * kSortThreads + (int)threadIdx.x < tcount)
      atomicAdd(&wcnt[0][(key[r] >> shift) & 255u], 1);
  __syncthreads();
  int32_t total;
  const int32_t lb = block_exclusive_scan<kSortThreads>(wcnt[0][threadIdx.x], lds_scan, &total);
  lbase[threadIdx.x] = lb;
  run_off[threadIdx.x] = lb;
#pragma unroll
  for (int r = 0; r < kSortRounds; ++r) {
#pragma unroll
    for (int w = 0; w < kWavesPerBlock; ++w) wcnt[w][threadIdx.x] = 0;
    __syncthreads();
    const bool valid = r * kSortThreads + (int)threadIdx.x < tcount;
    const uint32_t dig = (key[r] >> shift) & 255u;
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (dig >> b) & 1u;
      const uint64_t bal = __ballot(bit);
      peers &= bit ? bal : ~bal;
    }
    const int rank = __popcll(peers & lt_mask);
    const bool leader = valid && ((peers & lt_mask) == 0);
    if (leader) wcnt[wv][dig] = __popcll(peers);
    __syncthreads();
    if (valid) {
      int32_t pos = run_off[dig] + rank;
      for (int w = 0; w < wv; ++w) pos += wcnt[w][dig];
      s_key[pos] = key[r];
      s_idx[pos] = idx[r];
    }
    __syncthreads();
    int32_t add = 0;
#pragma unroll
    for (int w = 0; w < kWavesPerBlock; ++w) add += wcnt[w][threadIdx.x];
    run_off[threadIdx.x] += add;
  }
  __syncthreads();
  for (int32_t e = threadIdx.x; e < tcount; e += kSortThreads) {
    const uint32_t k = s_key[e];
    const uint32_t dg = (k >> shift) & 255u;
    const int64_t g = (int64_t)gbase[dg] + (e - lbase[dg]);
    kout[g] = k;
    iout[g] = s_idx[e];
  }
}

// ---------------------------------------------------------------------------
// gradient / Hessian sweep of a bundle (eq. (11); SVM: eq. (3) and the
// generalised Hessian), the direction (eq. (5)) and its Delta term (eq. (7)),
// over the bundle's nonzeros in partition order (one contiguous range, the
// nonzeros of each slot together).  Wavefront w takes ranges of W nonzeros
// (SweepArgs::W: 64, 128, 256 or 512, the chunk option), lane L the range's
// nonzeros kE L .. kE L + kE - 1 (kE = W / 64): a lane sums its own
// nonzeros per slot in order and finishes the slots that start and end
// inside it; one segmented wavefront scan over the lanes' last runs carries
// runs across lanes, and a slot is finished where it ends.  Slots that cross
// a range boundary leave partials (part[2m]: the part of range m of the slot
// that began before it, part[2m+1]: of the slot that begins in m and goes on)
// and k_sweep_finish completes them and the empty slots, adding partials in
// range order.  Every sum has a fixed order.  (d^T x, the second read of x,
// is formed by row afterwards.)
// ---------------------------------------------------------------------------
// g, h from the summed terms, the direction and Delta's term of slot o.
template <int LOSS>
__device__ inline void finish_slot(const SweepArgs& a, int64_t o, double gs, double hs, double wj,
                                   double C) {
  double g, h;
  if (LOSS == kLogistic) {
    g = C * gs;
    h = C * hs;
  } else {
    g = -2.0 * C * gs;
    h = 2.0 * C * hs;
  }
  if (h <= 0.0) h += a.nu;
  const double dj = newton_dir(g, h, wj, a.ra, a.rb);
  a.g[o] = g;
  a.h[o] = h;
  a.d[o] = dj;
  a.dterm[o] = g * dj + a.gamma * h * dj * dj + reg_change(wj, dj, a.ra, a.rb);
}

// Last slot of a launch's range, clipped to the active features when
// shrinking (the slot order lists them first).
__device__ inline int64_t clipped_hi(int64_t hi, const double* p_active) {
  if (!p_active) return hi;
  const int64_t pa = (int64_t)*p_active;
  return pa < hi ? pa : hi;
}

__device__ inline double lane_pick(double v, int src) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned l2 = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b & 0xffffffffull), src);
  const unsigned h2 = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), src);
  return __longlong_as_double((long long)(((unsigned long long)h2 << 32) | l2));
}

template <int LOSS, int kE>
__device__ __forceinline__ void sweep_ranges_body(const SweepArgs& a, int64_t bid, int64_t nblk) {
  constexpr int kW = kE * kWave;  // nonzeros per range (a.W); kE consecutive per lane
  const int lane = lane_id();
  const int64_t hi = clipped_hi(a.slot_hi, a.p_active);
  if (hi <= a.slot_lo) return;
  const int64_t e0 = a.poff[a.slot_lo], e1 = a.poff[hi];
  // ranges start at e0 rounded down to 4 nonzeros (the first range's
  // nonzeros before e0 belong to the bundle before and are left out), so a
  // lane's nonzeros of a whole range are one aligned vector of each array
  const int64_t e0a = e0 & ~(int64_t)3;
  const int64_t nr = (e1 - e0a + kW - 1) / kW;
  const int64_t nwaves = nblk * kWavesPerBlock;
  const double C = *a.Cp;
  const bool aligned = ((reinterpret_cast<uintptr_t>(a.pslot) | reinterpret_cast<uintptr_t>(a.pri) |
                         reinterpret_cast<uintptr_t>(a.pv)) & 15) == 0;
  for (int64_t m = uniform((bid * kBlock + threadIdx.x) / kWave); m < nr; m += nwaves) {
    const int64_t rb = e0a + m * kW;
    const int64_t re = rb + kW < e1 ? rb + kW : e1;
    const int64_t k0 = rb + (int64_t)lane * kE;
    int32_t sl[kE], row[kE];
    float xv[kE];
    if (kE % 4 == 0 && aligned && rb >= e0 && re - rb == kW) {
#pragma unroll
      for (int q = 0; q < kE / 4; ++q) {
        const int4 s4 = *reinterpret_cast<const int4*>(a.pslot + k0 + 4 * q);
        const int4 r4 = *reinterpret_cast<const int4*>(a.pri + k0 + 4 * q);
        const float4 v4 = *reinterpret_cast<const float4*>(a.pv + k0 + 4 * q);
        sl[4 * q] = s4.x; sl[4 * q + 1] = s4.y; sl[4 * q + 2] = s4.z; sl[4 * q + 3] = s4.w;
        row[4 * q] = r4.x; row[4 * q + 1] = r4.y; row[4 * q + 2] = r4.z; row[4 * q + 3] = r4.w;
        xv[4 * q] = v4.x; xv[4 * q + 1] = v4.y; xv[4 * q + 2] = v4.z; xv[4 * q + 3] = v4.w;
      }
    } else if (kE == 2 && aligned && rb >= e0 && re - rb == kW) {
      const int2 s2 = *reinterpret_cast<const int2*>(a.pslot + k0);
      const int2 r2 = *reinterpret_cast<const int2*>(a.pri + k0);
      const float2 v2 = *reinterpret_cast<const float2*>(a.pv + k0);
      sl[0] = s2.x; sl[kE - 1] = s2.y;
      row[0] = r2.x; row[kE - 1] = r2.y;
      xv[0] = v2.x; xv[kE - 1] = v2.y;
    } else {
#pragma unroll
      for (int u = 0; u < kE; ++u) {
        const int64_t k = k0 + u;
        const bool in = k >= e0 && k < re;
        sl[u] = ldz(a.pslot, in, k, -1);
        row[u] = ldz(a.pri, in, k, 0);
        xv[u] = ldz(a.pv, in, k, 0.0f);
      }
    }
    // slots open at the range's ends
    const int32_t left = rb > e0 ? a.pslot[rb - 1] : -1;
    const int32_t right = re < e1 ? a.pslot[re] : -1;
    double2 rv[kE];
    double wv[kE];
#pragma unroll
    for (int u = 0; u < kE; ++u) {
      rv[u] = ldz(a.rw, sl[u] >= 0, row[u], make_double2(0.0, 0.0));
      wv[u] = ldz(a.pw, sl[u] >= 0, sl[u], 0.0);
    }
    // every operand loaded before the first use (no load sunk into a branch)
#pragma unroll
    for (int u = 0; u < kE; ++u)
      asm volatile("" ::"v"(rv[u].x), "v"(rv[u].y), "v"(wv[u]), "v"(xv[u]));
    // the lane's runs: head (from its first nonzero), complete middles, tail
    const int32_t hk = sl[0];
    const double hw = wv[0];
    int32_t rk = sl[0];
    double rg = 0.0, rh = 0.0;
    if (sl[0] >= 0) weighted_terms<LOSS>(rv[0], (double)xv[0], rg, rh);
    double wk = wv[0], hg = 0.0, hh = 0.0;
    bool whole = true;  // one run covers the lane's nonzeros
#pragma unroll
    for (int u = 1; u < kE; ++u) {
      double tg = 0.0, th = 0.0;
      if (sl[u] >= 0) weighted_terms<LOSS>(rv[u], (double)xv[u], tg, th);
      if (sl[u] == rk) {
        rg += tg;
        rh += th;
      } else {
        if (whole) {
          hg = rg;  // the head run ends inside the lane
          hh = rh;
          whole = false;
        } else if (rk >= 0) {
          finish_slot<LOSS>(a, rk, rg, rh, wk, C);  // starts and ends here
        }
        rk = sl[u];
        rg = tg;
        rh = th;
        wk = wv[u];
      }
    }
    if (whole) {
      hg = rg;
      hh = rh;
    }
    // tail runs carried over the lanes of equal slot
    const int32_t tk = rk;
    double Sg = rg, Sh = rh;
    seg_scan1(Sg, tk);
    seg_scan1(Sh, tk);
    const int32_t pk = __builtin_amdgcn_update_dpp(-1, tk, 0x138, 0xf, 0xf, false);  // lane - 1
    const double pg = dpp_f64<0x138, 0xf, 0xf>(Sg);
    const double ph = dpp_f64<0x138, 0xf, 0xf>(Sh);
    const int32_t nk = next_lane_key(hk);  // the next lane's first slot
    const int last_lane = (int)((re - 1 - rb) / kE);
    double fg = 0.0, fh = 0.0, lg = 0.0, lh = 0.0;
    bool has_f = false, has_l = false;
    if (!whole && hk >= 0) {
      // the head run ends in this lane: add what the previous lanes carried
      const bool carried = lane > 0 && pk == hk;
      const double Hg = hg + (carried ? pg : 0.0), Hh = hh + (carried ? ph : 0.0);
      if (hk == left) {
        fg = Hg;
        fh = Hh;
        has_f = true;
      } else {
        finish_slot<LOSS>(a, hk, Hg, Hh, hw, C);
      }
    }
    if (tk >= 0 && lane <= last_lane) {
      const bool at_end = lane == last_lane;
      const bool cont = at_end ? right == tk : nk == tk;
      if (at_end || !cont) {
        if (tk == left) {  // (also when right-open: a slot through the whole range)
          fg = Sg;
          fh = Sh;
          has_f = true;
        } else if (cont) {
          lg = Sg;
          lh = Sh;
          has_l = true;
        } else {
          finish_slot<LOSS>(a, tk, Sg, Sh, wk, C);
        }
      }
    }
    // the partials (held by the lanes that ended the open runs)
    const uint64_t mf = __ballot(has_f), ml = __ballot(has_l);
    double2 pf = make_double2(0.0, 0.0), pl = make_double2(0.0, 0.0);
    if (mf) {
      const int src = __builtin_ctzll(mf);
      pf = make_double2(lane_pick(fg, src), lane_pick(fh, src));
    }
    if (ml) {
      const int src = __builtin_ctzll(ml);
      pl = make_double2(lane_pick(lg, src), lane_pick(lh, src));
    }
    if (lane == 0) {
      a.part[2 * m] = pf;
      a.part[2 * m + 1] = pl;
    }
  }
}

template <int LOSS, int kE>
__global__ __launch_bounds__(kBlock) void k_sweep_ranges(SweepArgs a) {
  sweep_ranges_body<LOSS, kE>(a, blockIdx.x, gridDim.x);
}

// The body for the range width a.W (64, 128, 256 or 512 nonzeros).
template <int LOSS>
__device__ __forceinline__ void sweep_ranges_any(const SweepArgs& a, int64_t bid, int64_t nblk) {
  switch (a.W) {
    case 64: sweep_ranges_body<LOSS, 1>(a, bid, nblk); break;
    case 128: sweep_ranges_body<LOSS, 2>(a, bid, nblk); break;
    case 512: sweep_ranges_body<LOSS, 8>(a, bid, nblk); break;
    default: sweep_ranges_body<LOSS, 4>(a, bid, nblk); break;
  }
}

// Slots that cross a range boundary and empty slots (g_j = h_j = 0 before
// the floor).  Lane L of a wavefront takes slot base + L: a slot over at
// most kFinishShort + 1 ranges adds its partials in range order itself; a
// longer one (a long column) is summed by the whole wavefront, lanes taking
// every 64th range, then the fixed-order wavefront sum.
constexpr int kFinishShort = 4;

template <int LOSS>
__device__ __forceinline__ void sweep_finish_body(const SweepArgs& a, int64_t bid, int64_t nblk) {
  const int64_t hi = clipped_hi(a.slot_hi, a.p_active);
  if (hi <= a.slot_lo) return;
  const int lane = lane_id();
  const int64_t e0a = a.poff[a.slot_lo] & ~(int64_t)3;  // where the sweep's ranges start
  const double C = *a.Cp;
  const int wsh = __builtin_ctz((unsigned)a.W);  // range index = offset >> wsh (W a power of 2)
  const int64_t nwaves = nblk * kWavesPerBlock;
  for (int64_t base = a.slot_lo + uniform((bid * kBlock + threadIdx.x) / kWave) * kWave; base < hi;
       base += nwaves * kWave) {
    const int64_t o = base + lane;
    const bool valid = o < hi;
    const int64_t k0 = ldz(a.poff, valid, o, (int64_t)0), k1 = ldz(a.poff, valid, o + 1, (int64_t)0);
    const int64_t m1 = (k0 - e0a) >> wsh, m2 = k1 > k0 ? (k1 - 1 - e0a) >> wsh : m1;
    const bool empty = valid && k1 == k0;
    const bool crossing = valid && k1 > k0 && m2 > m1;
    const bool longer = crossing && m2 - m1 > kFinishShort;
    const double wj = ldz(a.pw, valid, o, 0.0);
    if (empty) finish_slot<LOSS>(a, o, 0.0, 0.0, wj, C);
    if (crossing && !longer) {
      double2 t = a.part[2 * m1 + 1];
      double gs = t.x, hs = t.y;
      for (int64_t m = m1 + 1; m <= m2; ++m) {
        t = a.part[2 * m];
        gs += t.x;
        hs += t.y;
      }
      finish_slot<LOSS>(a, o, gs, hs, wj, C);
    }
    for (uint64_t lm = __ballot(longer); lm; lm &= lm - 1) {
      const int src = __builtin_ctzll(lm);
      const int64_t s1 = (int64_t)__builtin_amdgcn_readlane((int)m1, src) , s2 =
          (int64_t)__builtin_amdgcn_readlane((int)m2, src);
      double gs = 0.0, hs = 0.0;
      for (int64_t m = s1 + 1 + lane; m <= s2; m += kWave) {
        const double2 t = a.part[2 * m];
        gs += t.x;
        hs += t.y;
      }
      gs = wave_sum(gs);
      hs = wave_sum(hs);
      if (lane == src) {
        const double2 t = a.part[2 * m1 + 1];
        finish_slot<LOSS>(a, o, t.x + gs, t.y + hs, wj, C);
      }
    }
  }
}

template <int LOSS>
__global__ __launch_bounds__(kBlock) void k_sweep_finish(SweepArgs a) {
  sweep_finish_body<LOSS>(a, blockIdx.x, gridDim.x);
}

// ---------------------------------------------------------------------------
// stopping sweep over X in column order (see StopArgs)
// ---------------------------------------------------------------------------
template <int LOSS>
__device__ inline void stop_finish_one(const StopArgs& a, int64_t j, double gs, double C,
                                       double thr, double wj) {
  const double g = LOSS == kLogistic ? C * gs : -2.0 * C * gs;
  a.sg[j] = fabs(min_norm_subgradient(g, wj, a.ra, a.rb));
  if (a.act) a.act[j] = (wj != 0.0 || fabs(g) >= thr) ? 1.0 : 0.0;
}

// C and the shrinking threshold, read once before any store of the launch
// (so they stay in registers instead of being reloaded behind every store).
struct StopScalars {
  double C, thr;
};
__device__ inline StopScalars stop_scalars(const StopArgs& a) {
  return {*a.Cp, a.act ? *a.thr : 0.0};
}

// Range m of the stopping sweep (one wavefront); lane L holds the range's
// nonzeros 4L .. 4L+3.  In three parts, so that a caller can issue the
// loads of several ranges before it waits for any: the range's columns and
// values (and rows, for the gather), the rows' gradient weights and the
// columns' w, then the sums.
constexpr int kStopE = kStopW / kWave;  // consecutive nonzeros per lane
static_assert(kStopE == 4, "a lane's nonzeros are one 16-byte vector of each array");
struct StopOps {
  int64_t rb, re;
  int32_t col[kStopE], row[kStopE];
  float xv[kStopE];
  double rg[kStopE], wv[kStopE];
  int32_t left, right;
};

template <bool FROM_LDS>
__device__ inline void stop_range_load(const StopArgs& a, int64_t m, StopOps& o) {
  constexpr int kE = kStopE;
  const int lane = lane_id();
  o.rb = m * kStopW;
  o.re = o.rb + kStopW < a.nnz ? o.rb + kStopW : a.nnz;
  const int64_t rb = o.rb, re = o.re;
  const int64_t k0 = rb + (int64_t)lane * kE;
  const bool aligned = ((reinterpret_cast<uintptr_t>(a.ccol) | reinterpret_cast<uintptr_t>(a.v) |
                         (FROM_LDS ? 0 : reinterpret_cast<uintptr_t>(a.ri))) & 15) == 0;
  if (re - rb == kStopW && aligned) {
    // a whole range: 16-byte loads (rb is a multiple of kStopW, so k0 of 4)
    const int4 c4 = *reinterpret_cast<const int4*>(a.ccol + k0);
    const float4 v4 = *reinterpret_cast<const float4*>(a.v + k0);
    o.col[0] = c4.x; o.col[1] = c4.y; o.col[2] = c4.z; o.col[3] = c4.w;
    o.xv[0] = v4.x; o.xv[1] = v4.y; o.xv[2] = v4.z; o.xv[3] = v4.w;
    if (FROM_LDS) {
      o.row[0] = o.row[1] = o.row[2] = o.row[3] = 0;
    } else {
      const int4 r4 = *reinterpret_cast<const int4*>(a.ri + k0);
      o.row[0] = r4.x; o.row[1] = r4.y; o.row[2] = r4.z; o.row[3] = r4.w;
    }
  } else {
#pragma unroll
    for (int u = 0; u < kE; ++u) {
      const int64_t k = k0 + u;
      const bool in = k < re;
      o.col[u] = ldz(a.ccol, in, k, -1);
      o.row[u] = FROM_LDS ? 0 : ldz(a.ri, in, k, 0);
      o.xv[u] = ldz(a.v, in, k, 0.0f);
    }
  }
  // columns open at the range's ends
  o.left = rb > 0 ? a.ccol[rb - 1] : -1;
  o.right = re < a.nnz ? a.ccol[re] : -1;
}

// The rows' gradient weights alone (the first of the two row weights; zero
// where an SVM row has no slack, so the product is the term): gathered, or
// (FROM_LDS) already placed at the nonzero's position; and the columns' w
// (w = 0 when a.w is null: a load of the always valid cache[0], discarded).
template <bool FROM_LDS>
__device__ inline void stop_range_gather(const StopArgs& a, StopOps& o, const double* lgw,
                                         int64_t lbase) {
  constexpr int kE = kStopE;
  const int64_t k0 = o.rb + (int64_t)lane_id() * kE;
  const double* gw = reinterpret_cast<const double*>(a.rw);
  const double* wsrc = a.w ? a.w : a.cache;
#pragma unroll
  for (int u = 0; u < kE; ++u) {
    o.rg[u] = FROM_LDS ? (o.col[u] >= 0 ? lgw[k0 + u - lbase] : 0.0)
                       : ldz(gw, o.col[u] >= 0, 2 * (int64_t)o.row[u], 0.0);
    o.wv[u] = ldz(wsrc, o.col[u] >= 0 && a.w != nullptr, o.col[u], 0.0);
  }
}

// every operand loaded before the first use (the compiler would sink loads
// into the finishing branches and wait for each there)
__device__ inline void stop_range_pin(StopOps& o) {
#pragma unroll
  for (int u = 0; u < kStopE; ++u) asm volatile("" ::"v"(o.rg[u]), "v"(o.wv[u]), "v"(o.xv[u]));
}

template <int LOSS>
__device__ inline void stop_range_sums(const StopArgs& a, int64_t m, const StopScalars& sc,
                                       const StopOps& o) {
  constexpr int kE = kStopE;
  const int lane = lane_id();
  const int64_t rb = o.rb, re = o.re;
  const int32_t* col = o.col;
  const float* xv = o.xv;
  const double* rg = o.rg;
  const double* wv = o.wv;
  const int32_t left = o.left, right = o.right;
  // the lane's runs: head (from its first nonzero), complete middles, tail
  const int32_t hk = col[0];
  const double hw = wv[0];
  int32_t rk = col[0];
  double run = col[0] >= 0 ? rg[0] * (double)xv[0] : 0.0;
  double wk = wv[0], hs = 0.0;
  bool whole = true;  // one run covers the lane's nonzeros
#pragma unroll
  for (int u = 1; u < kE; ++u) {
    const double t = col[u] >= 0 ? rg[u] * (double)xv[u] : 0.0;
    if (col[u] == rk) {
      run += t;
    } else {
      if (whole) {
        hs = run;  // the head run ends inside the lane
        whole = false;
      } else if (rk >= 0) {
        stop_finish_one<LOSS>(a, rk, run, sc.C, sc.thr, wk);  // starts and ends here
      }
      rk = col[u];
      run = t;
      wk = wv[u];
    }
  }
  if (whole) hs = run;
  // tail runs carried over the lanes of equal column
  const int32_t tk = rk;
  double S = run;
  seg_scan1(S, tk);
  const int32_t pk = __builtin_amdgcn_update_dpp(-1, tk, 0x138, 0xf, 0xf, false);  // lane - 1
  const double pS = dpp_f64<0x138, 0xf, 0xf>(S);
  const int32_t nk = next_lane_key(hk);  // the next lane's first column
  const int last_lane = (int)((re - 1 - rb) / kE);
  double pf = 0.0, pl = 0.0;
  if (!whole && hk >= 0) {
    // the head run ends in this lane: add what the previous lanes carried
    const double H = hs + (lane > 0 && pk == hk ? pS : 0.0);
    if (hk == left)
      pf = H;
    else
      stop_finish_one<LOSS>(a, hk, H, sc.C, sc.thr, hw);
  }
  if (tk >= 0 && lane <= last_lane) {
    const bool at_end = lane == last_lane;
    const bool cont = at_end ? right == tk : nk == tk;
    if (at_end || !cont) {
      if (tk == left)
        pf = S;  // (also when right-open: a column through the whole range)
      else if (cont)
        pl = S;
      else
        stop_finish_one<LOSS>(a, tk, S, sc.C, sc.thr, wk);
    }
  }
  // the partials (held by the lanes that ended the open runs)
  const uint64_t mf = __ballot(pf != 0.0), ml = __ballot(pl != 0.0);
  double2 pr = make_double2(0.0, 0.0);
  if (mf) {
    const int src = __builtin_ctzll(mf);
    const unsigned long long b = (unsigned long long)__double_as_longlong(pf);
    const unsigned l2 = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b & 0xffffffffull), src);
    const unsigned h2 = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), src);
    pr.x = __longlong_as_double((long long)(((unsigned long long)h2 << 32) | l2));
  }
  if (ml) {
    const int src = __builtin_ctzll(ml);
    const unsigned long long b = (unsigned long long)__double_as_longlong(pl);
    const unsigned l2 = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b & 0xffffffffull), src);
    const unsigned h2 = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), src);
    pr.y = __longlong_as_double((long long)(((unsigned long long)h2 << 32) | l2));
  }
  if (lane == 0) a.part[m] = pr;
}

template <int LOSS, bool FROM_LDS>
__device__ inline void stop_one_range(const StopArgs& a, int64_t m, const StopScalars& sc,
                                      const double* lgw, int64_t lbase) {
  StopOps o;
  stop_range_load<FROM_LDS>(a, m, o);
  stop_range_gather<FROM_LDS>(a, o, lgw, lbase);
  stop_range_pin(o);
  stop_range_sums<LOSS>(a, m, sc, o);
}

// Wavefront w of the launch takes ranges w, w + nwaves, ... (the rows'
// weights gathered from global memory).
template <int LOSS>
__device__ __forceinline__ void stop_ranges_body(const StopArgs& a, int64_t bid, int64_t nblk) {
  const int64_t nr = (a.nnz + kStopW - 1) / kStopW;
  const int64_t nwaves = nblk * kWavesPerBlock;
  const StopScalars sc = stop_scalars(a);
  for (int64_t m = uniform((bid * kBlock + threadIdx.x) / kWave); m < nr; m += nwaves)
    stop_one_range<LOSS, false>(a, m, sc, nullptr, 0);
}

template <int LOSS>
__global__ __launch_bounds__(kBlock) void k_stop_ranges(StopArgs a) {
  stop_ranges_body<LOSS>(a, blockIdx.x, gridDim.x);
}

// The stopping sweep by tiles of kStopTile consecutive nonzeros (whole
// ranges), one 1024-thread workgroup each, when the tiles' row-sorted lists
// exist (a.srow, a.spos: each tile's nonzeros in row order, with their
// positions in the tile).  The workgroup first gathers the rows' gradient
// weights in row order, so consecutive threads read neighbouring rows (a
// tile touches a sixth of the 100,000 rows of the huge sparse workload, so
// most 128-byte lines serve several nonzeros instead of one), and places
// each at its nonzero's position in LDS; then its wavefronts run the tile's
// ranges as stop_ranges_body does, reading the weights from LDS.  The sums
// and their order are those of stop_ranges_body, so are the results.
// The rows' gradient weights (the first of each row's two) packed into one
// array for the tiles' gathers.
__global__ __launch_bounds__(kBlock) void k_pack_gradient_weights(const double2* rw, int64_t n,
                                                                  double* gwc) {
  for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlock)
    gwc[i] = rw[i].x;
}

constexpr int kStopTileThreads = 1024;
constexpr int kStopTileRounds = 16;
static_assert(kStopTile == kStopTileThreads * kStopTileRounds, "one weight per thread and round");
template <int LOSS>
__global__ __launch_bounds__(kStopTileThreads) void k_stop_tiles(StopArgs a) {
  __shared__ double lgw[kStopTile];
  const int64_t base = (int64_t)blockIdx.x * kStopTile;
  const int64_t tcount = a.nnz - base < kStopTile ? a.nnz - base : kStopTile;
  const double* gw = a.gwc;  // packed: 16 rows a 128-byte line
  {
    int32_t row[kStopTileRounds];
    int32_t pos[kStopTileRounds];
#pragma unroll
    for (int r = 0; r < kStopTileRounds; ++r) {
      const int64_t e = (int64_t)r * kStopTileThreads + threadIdx.x;
      row[r] = ldz(a.srow, e < tcount, base + e, 0);
      pos[r] = (int32_t)ldz(a.spos, e < tcount, base + e, (uint16_t)0);
    }
    double g[kStopTileRounds];
#pragma unroll
    for (int r = 0; r < kStopTileRounds; ++r) {
      const int64_t e = (int64_t)r * kStopTileThreads + threadIdx.x;
      g[r] = ldz(gw, e < tcount, (int64_t)row[r], 0.0);
    }
#pragma unroll
    for (int r = 0; r < kStopTileRounds; ++r) {
      const int64_t e = (int64_t)r * kStopTileThreads + threadIdx.x;
      if (e < tcount) lgw[pos[r]] = g[r];
    }
  }
  __syncthreads();
  const StopScalars sc = stop_scalars(a);
  const int64_t nr = (tcount + kStopW - 1) / kStopW;
  const int64_t m0 = base / kStopW;
  // two ranges at a time, both ranges' loads issued before either is summed
  // (a missing second range repeats the first's loads and is not summed)
  constexpr int kWaves = kStopTileThreads / kWave;
  for (int64_t j = uniform(threadIdx.x / kWave); j < nr; j += 2 * kWaves) {
    const bool two = j + kWaves < nr;
    const int64_t jb = two ? j + kWaves : j;
    StopOps o1, o2;
    stop_range_load<true>(a, m0 + j, o1);
    stop_range_load<true>(a, m0 + jb, o2);
    stop_range_gather<true>(a, o1, lgw, base);
    stop_range_gather<true>(a, o2, lgw, base);
    stop_range_pin(o1);
    stop_range_pin(o2);
    stop_range_sums<LOSS>(a, m0 + j, sc, o1);
    if (two) stop_range_sums<LOSS>(a, m0 + jb, sc, o2);
  }
}

// Columns that cross a range boundary (the partials in range order) and
// empty columns (g_j = 0); one thread per column.
template <int LOSS>
__device__ __forceinline__ void stop_finish_body(const StopArgs& a, int64_t bid, int64_t nblk) {
  const StopScalars sc = stop_scalars(a);
  const int lane = lane_id();
  const int64_t nwaves = nblk * kWavesPerBlock;
  // lane L of a wavefront takes column base + L; long columns are summed by
  // the whole wavefront (as the bundle sweep's finish does)
  for (int64_t base = uniform((bid * kBlock + threadIdx.x) / kWave) * kWave; base < a.p;
       base += nwaves * kWave) {
    const int64_t j = base + lane;
    const bool valid = j < a.p;
    const int64_t k0 = ldz(a.cp, valid, j, (int64_t)0), k1 = ldz(a.cp, valid, j + 1, (int64_t)0);
    const int64_t m1 = k0 / kStopW, m2 = k1 > k0 ? (k1 - 1) / kStopW : m1;
    const bool empty = valid && k1 == k0;
    const bool crossing = valid && k1 > k0 && m2 > m1;
    const bool longer = crossing && m2 - m1 > kFinishShort;
    const double wj = a.w ? ldz(a.w, valid, j, 0.0) : 0.0;
    if (empty) stop_finish_one<LOSS>(a, j, 0.0, sc.C, sc.thr, wj);
    if (crossing && !longer) {
      double gs = a.part[m1].y;
      for (int64_t m = m1 + 1; m <= m2; ++m) gs += a.part[m].x;
      stop_finish_one<LOSS>(a, j, gs, sc.C, sc.thr, wj);
    }
    for (uint64_t lm = __ballot(longer); lm; lm &= lm - 1) {
      const int src = __builtin_ctzll(lm);
      const int64_t s1 = (int64_t)__builtin_amdgcn_readlane((int)m1, src);
      const int64_t s2 = (int64_t)__builtin_amdgcn_readlane((int)m2, src);
      double gs = 0.0;
      for (int64_t m = s1 + 1 + lane; m <= s2; m += kWave) gs += a.part[m].x;
      gs = wave_sum(gs);
      if (lane == src) stop_finish_one<LOSS>(a, j, a.part[m1].y + gs, sc.C, sc.thr, wj);
    }
  }
}

template <int LOSS>
__global__ __launch_bounds__(kBlock) void k_stop_finish(StopArgs a) {
  stop_finish_body<LOSS>(a, blockIdx.x, gridDim.x);
}

// ---------------------------------------------------------------------------
// d^T x by row, the line search (Algorithm 4 with eq. (10)) and the update,
// over the bundle's nonzeros in bundle-row order (see RowsArgs).
//
// d^T x_i = sum_{j in B} d_j x_ij is formed for each touched row by one
// wavefront in a fixed order (a segmented wavefront scan over the row's
// nonzeros in column order, rounds of 64 added in order), so it does not
// depend on timing; no atomics.  The same pass evaluates the first kQGroup
// line-search candidates on the row (the per-sample argument is d^T x_i
// scaled by beta once per rejected candidate, as Algorithm 4 scales its
// retained d^T x_i) and lists the row for the apply.  Per-block partials
// land at part[v * G + block] and are summed in block order by every block
// of the apply, which takes the Armijo decision (eq. (6)) identically.
// ---------------------------------------------------------------------------
// Orders this wavefront's LDS accesses (the queue below is wave-private).
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Loss changes of one row for candidates 0..nq-1 (argument scaled by beta
// once per candidate).
template <int LOSS>
__device__ inline void row_ls_terms(double c, int yi, double dl, double beta, int nq,
                                    double (&acc)[kQGroup], double (&aabs)[kQGroup]) {
  double s = dl;
#pragma unroll
  for (int q = 0; q < kQGroup; ++q) {
    if (q < nq) {
      const double t = loss_delta<LOSS>(c, yi, s);
      acc[q] += t;
      aabs[q] += loss_delta_scale<LOSS>(c, yi, s, t);
      s *= beta;
    }
  }
}

// A wavefront's queue of finished rows in LDS: row, d^T x_i, retained
// quantity and label.
struct RowQueue {
  int32_t row[2 * kWave];
  int32_t y[2 * kWave];
  double dtx[2 * kWave];
  double c[2 * kWave];
};

// n <= 64 queued rows (lane i takes queue entry i): list them for the apply
// and add their line-search terms.
template <int LOSS>
__device__ inline void rows_flush(const RowsArgs& a, const RowQueue& qu, int n, int64_t ubase,
                                  int nq, double (&acc)[kQGroup], double (&aabs)[kQGroup],
                                  double& touched) {
  const int lane = lane_id();
  if (lane < n) {
    const double dl = qu.dtx[lane];
    a.u_row[ubase + lane] = qu.row[lane];
    a.u_dtx[ubase + lane] = dl;
    touched += 1.0;
    row_ls_terms<LOSS>(qu.c[lane], qu.y[lane], dl, a.beta, nq, acc, aabs);
  }
}

// One round of 64 nonzeros of a range: the segmented row sums (carried across
// rounds), and the rows that end in it queued.  Returns the number queued.
__device__ inline int rows_round(RowQueue& qu, int qn, int32_t row, bool owned, double t, double c,
                                 int yi, int32_t next63, int32_t& crow, double& cval) {
  const int lane = lane_id();
  const uint64_t lt_mask = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  const int32_t key = owned ? row : -1;
  seg_scan1(t, key);
  if (crow >= 0 && key == crow) t += cval;
  // the row ends at this nonzero unless the next one is of the same row
  // (for lane 63: next63, the row of the nonzero after the round, < 0 if none)
  int32_t nxt = next_lane_key(key);
  if (lane == kWave - 1) nxt = next63;
  const bool ends = owned && nxt != row;
  const int32_t row63 = __builtin_amdgcn_readlane(key, kWave - 1);
  const bool open63 = __builtin_amdgcn_readlane((int)(owned && !ends), kWave - 1) != 0;
  const unsigned long long tb = (unsigned long long)__double_as_longlong(t);
  const unsigned lo63 = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(tb & 0xffffffffull), kWave - 1);
  const unsigned hi63 = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(tb >> 32), kWave - 1);
  crow = open63 ? row63 : -1;
  cval = open63 ? __longlong_as_double((long long)(((unsigned long long)hi63 << 32) | lo63)) : 0.0;
  // queue the finished rows with d^T x_i != 0 (a zero changes nothing)
  const bool done = ends && t != 0.0;
  const uint64_t m = __ballot(done);
  if (done) {
    const int pos = qn + __popcll(m & lt_mask);
    qu.row[pos] = row;
    qu.y[pos] = yi;
    qu.dtx[pos] = t;
    qu.c[pos] = c;
  }
  return __popcll(m);
}

// Block bx of the G-block launch: wavefront w = bx * 4 + wave takes ranges
// w, w + 4G, ... of the bundle's nonzeros.  The loads of a range's four
// rounds are issued together (rows, slots and values, then the directions
// and the rows' retained quantities and labels), so a range costs two
// dependent round trips to memory.
template <int LOSS, bool EARLY>
__device__ __forceinline__ void rows_dtx_body(const RowsArgs& a, int bx) {
  constexpr int kR = kRangeW / kWave;
  __shared__ RowQueue queue[kWavesPerBlock];
  __shared__ double red[kWavesPerBlock][2 * kQGroup + 2];
  const int64_t hi_act = clipped_hi(a.slot_hi, a.p_active);
  if (hi_act <= a.slot_lo) return;  // no active feature in this bundle: the apply skips it too
  const int lane = lane_id(), wv = wave_in_block();
  const int G = a.G;
  const int nq = a.Q < kQGroup ? a.Q : kQGroup;
  const int64_t e0 = a.poff[a.slot_lo], e1 = a.poff[a.slot_hi];
  const int64_t nr = (e1 - e0 + kRangeW - 1) / kRangeW;
  const int64_t nwaves = (int64_t)G * kWavesPerBlock;
  {
    // a wavefront without a range lists none there (the apply reads its
    // count before it knows the bundle's ranges)
    const int64_t gw = (int64_t)bx * kWavesPerBlock + wv;
    if (gw >= nr && gw < a.u_cap && lane == 0) a.u_cnt[gw] = 0;
  }
  RowQueue& qu = queue[wv];
  // EARLY: the regulariser terms' operands of this thread's first slot,
  // loaded now (they depend on nothing the row sums compute; w from its copy
  // in partition order, which no apply has changed for this bundle's slots).
  // The executor's copy of this body loads them where they are used: the
  // registers they hold across the row sums would cost it occupancy.
  const int64_t Pt = hi_act - a.slot_lo;
  const int64_t r0 = (int64_t)bx * kBlock + threadIdx.x;
  const bool has0 = EARLY && r0 < Pt;
  double wj0 = 0.0, dj0 = 0.0, dt0 = 0.0;
  if (EARLY) {
    wj0 = ldz(a.pw, has0, a.slot_lo + r0, 0.0);
    dj0 = ldz(a.d, has0, a.slot_lo + r0, 0.0);
    dt0 = ldz(a.dterm, has0, a.slot_lo + r0, 0.0);
    asm volatile("" ::"v"(wj0), "v"(dj0), "v"(dt0));
  }
  double acc[kQGroup], aabs[kQGroup];
#pragma unroll
  for (int q = 0; q < kQGroup; ++q) acc[q] = aabs[q] = 0.0;
  double touched = 0.0, nz_d = 0.0;
  for (int64_t r = (int64_t)bx * kWavesPerBlock + wv; r < nr; r += nwaves) {
    const int64_t rb = e0 + r * kRangeW;
    const int64_t re = rb + kRangeW < e1 ? rb + kRangeW : e1;
    // rows owned by this range: those whose first nonzero lies in [rb, re);
    // the range's first row may have started earlier (skip), its last row
    // may continue past re (tail)
    int32_t prow[kR], psl[kR];
    float pv[kR];
#pragma unroll
    for (int u = 0; u < kR; ++u) {
      const int64_t k = rb + u * kWave + lane;
      prow[u] = ldz(a.br_row, k < e1, k, -1);
      psl[u] = ldz(a.br_slot, k < e1, k, -1);
      pv[u] = ldz(a.br_val, k < e1, k, 0.0f);
    }
    const int32_t skip = rb > e0 ? a.br_row[rb - 1] : -1;
    int32_t tail = a.br_row[re - 1];
    if (tail == skip) tail = -1;
    // the row of the nonzero after the last loaded round (< 0: none)
    const int32_t after = rb + kRangeW < e1 ? a.br_row[rb + kRangeW] : -2;
    double pd[kR], pc[kR];
    int py[kR];
#pragma unroll
    for (int u = 0; u < kR; ++u) {
      const bool act = psl[u] >= a.slot_lo && psl[u] < hi_act;
      pd[u] = ldz(a.d, act, psl[u], 0.0);
      pc[u] = ldz(a.cache, prow[u] >= 0, prow[u], 0.0);
      py[u] = (int)ldz(a.y, prow[u] >= 0, prow[u], (int8_t)0);
    }
    // all operands loaded before the rounds use them (no load sunk into a
    // branch and waited for there)
#pragma unroll
    for (int u = 0; u < kR; ++u) asm volatile("" ::"v"(pd[u]), "v"(pc[u]), "v"(py[u]), "v"(pv[u]));
    int qn = 0;            // rows queued in LDS
    int32_t listed = 0;    // rows listed for this range
    int32_t crow = -1;     // row carried into the next round
    double cval = 0.0;
    int64_t s0 = rb;
#pragma unroll
    for (int u = 0; u < kR; ++u, s0 += kWave) {
      if (s0 >= re && crow < 0) break;
      const int64_t k = s0 + lane;
      const bool owned = k < e1 && prow[u] != skip && (k < re || prow[u] == tail);
      const double t = owned ? pd[u] * (double)pv[u] : 0.0;
      nz_d += owned && pd[u] != 0.0 ? 1.0 : 0.0;
      const int32_t n63 = u + 1 < kR ? __builtin_amdgcn_readlane(prow[u + 1], 0) : after;
      qn += rows_round(qu, qn, prow[u], owned, t, pc[u], py[u], n63, crow, cval);
      if (qn >= kWave) {
        wave_lds_sync();
        rows_flush<LOSS>(a, qu, kWave, r * kRangeW + listed, nq, acc, aabs, touched);
        listed += kWave;
        qn -= kWave;
        wave_lds_sync();
        if (lane < qn) {
          qu.row[lane] = qu.row[kWave + lane];
          qu.y[lane] = qu.y[kWave + lane];
          qu.dtx[lane] = qu.dtx[kWave + lane];
          qu.c[lane] = qu.c[kWave + lane];
        }
      }
    }
    // the tail row continues past the loaded rounds (one row only)
    for (; crow >= 0; s0 += kWave) {
      const int64_t k = s0 + lane;
      const int32_t row = k < e1 ? a.br_row[k] : -1;
      const bool owned = k < e1 && row == tail;
      double t = 0.0, c = 0.0;
      int yi = 0;
      if (owned) {
        const int32_t sl = a.br_slot[k];
        if (sl >= a.slot_lo && sl < hi_act) {
          const double dj = a.d[sl];
          t = dj * (double)a.br_val[k];
          nz_d += dj != 0.0 ? 1.0 : 0.0;
        }
        c = a.cache[row];
        yi = (int)a.y[row];
      }
      const int64_t k63 = s0 + kWave - 1;
      const int32_t n63 = k63 + 1 < e1 ? a.br_row[k63 + 1] : -2;
      qn += rows_round(qu, qn, row, owned, t, c, yi, n63, crow, cval);
      if (qn >= kWave) {
        wave_lds_sync();
        rows_flush<LOSS>(a, qu, kWave, r * kRangeW + listed, nq, acc, aabs, touched);
        listed += kWave;
        qn -= kWave;
        wave_lds_sync();
        if (lane < qn) {
          qu.row[lane] = qu.row[kWave + lane];
          qu.y[lane] = qu.y[kWave + lane];
          qu.dtx[lane] = qu.dtx[kWave + lane];
          qu.c[lane] = qu.c[kWave + lane];
        }
      }
    }
    wave_lds_sync();
    rows_flush<LOSS>(a, qu, qn, r * kRangeW + listed, nq, acc, aabs, touched);
    listed += qn;
    if (lane == 0) a.u_cnt[r] = listed;
    wave_lds_sync();
  }
#pragma unroll
  for (int q = 0; q < kQGroup; ++q) {
    const double v = wave_sum(acc[q]);
    const double va = wave_sum(aabs[q]);
    if (lane == 0) {
      red[wv][q] = v;
      red[wv][kQGroup + 2 + q] = va;
    }
  }
  {
    const double v = wave_sum(touched);
    const double z = wave_sum(nz_d);
    if (lane == 0) {
      red[wv][kQGroup] = v;
      red[wv][kQGroup + 1] = z;
    }
  }
  __syncthreads();
  {
    // part rows: q -> loss sum of candidate q; 2Q+1 touched rows; 2Q+2
    // nonzeros with d_j != 0; 2Q+3+q -> rounding scale of the loss changes of
    // candidate q
    const int v = threadIdx.x;
    const double tot = v < 2 * kQGroup + 2
                           ? ((red[0][v] + red[1][v]) + red[2][v]) + red[3][v]
                           : 0.0;
    if (v < nq) a.part[(int64_t)v * G + bx] = tot;
    if (v == kQGroup) a.part[(int64_t)(2 * a.Q + 1) * G + bx] = tot;
    if (v == kQGroup + 1) a.part[(int64_t)(2 * a.Q + 2) * G + bx] = tot;
    if (v >= kQGroup + 2 && v < kQGroup + 2 + nq)
      a.part[(int64_t)(2 * a.Q + 3 + (v - kQGroup - 2)) * G + bx] = tot;
  }
  __syncthreads();
  // Delta and the regulariser change of the bundle coordinates
  double del = 0.0;
#pragma unroll
  for (int q = 0; q < kQGroup; ++q) acc[q] = aabs[q] = 0.0;
  for (int64_t r = r0; r < Pt; r += (int64_t)G * kBlock) {
    const int64_t slot = a.slot_lo + r;
    const bool pre = EARLY && r == r0;
    const double wj = pre ? wj0 : a.pw[slot];
    const double dj = pre ? dj0 : a.d[slot];
    del += pre ? dt0 : a.dterm[slot];
    double al = 1.0;
#pragma unroll
    for (int q = 0; q < kQGroup; ++q) {
      if (q < nq) {
        const double rc = reg_change(wj, al * dj, a.ra, a.rb);
        acc[q] += rc;
        aabs[q] += reg_change_scale(wj, al * dj, a.ra, a.rb);
        al *= a.beta;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < kQGroup; ++q) {
    const double v = wave_sum(acc[q]);
    const double va = wave_sum(aabs[q]);
    if (lane == 0) {
      red[wv][q] = v;
      red[wv][kQGroup + 2 + q] = va;
    }
  }
  {
    const double v = wave_sum(del);
    if (lane == 0) red[wv][kQGroup] = v;
  }
  __syncthreads();
  {
    // part rows: Q+q -> regulariser change of candidate q; 2Q Delta;
    // 3Q+3+q -> rounding scale of the regulariser changes of candidate q
    const int v = threadIdx.x;
    const double tot = v < 2 * kQGroup + 2
                           ? ((red[0][v] + red[1][v]) + red[2][v]) + red[3][v]
                           : 0.0;
    if (v < nq) a.part[(int64_t)(a.Q + v) * G + bx] = tot;
    if (v == kQGroup) a.part[(int64_t)(2 * a.Q) * G + bx] = tot;
    if (v >= kQGroup + 2 && v < kQGroup + 2 + nq)
      a.part[(int64_t)(3 * a.Q + 3 + (v - kQGroup - 2)) * G + bx] = tot;
  }
}

template <int LOSS>
__global__ __launch_bounds__(kBlock) void k_rows_dtx(RowsArgs a) {
  rows_dtx_body<LOSS, true>(a, blockIdx.x);
}

// Sum of row v of the line-search partials, same order in every block.
__device__ inline double ls_total(const double* part, int v, int G, double* lds4) {
  double x = 0.0;
  for (int b = threadIdx.x; b < G; b += kBlock) x += part[(int64_t)v * G + b];
  return block_sum(x, lds4);
}

// ls_total of N partial rows at once: the same sums in the same order (so
// the same bits), with the rows' loads issued together.  ls_load issues this
// thread's first loads (so that other loads can be issued behind them);
// ls_finish adds the rest and reduces.
template <int N>
__device__ inline void ls_load(const double* part, const int (&v)[N], int G, double (&x)[N]) {
  const int b = threadIdx.x;
  double y[N];
#pragma unroll
  for (int k = 0; k < N; ++k) y[k] = ldz(part, b < G, (int64_t)v[k] * G + b, 0.0);
#pragma unroll
  for (int k = 0; k < N; ++k) x[k] = 0.0 + y[k];
}

template <int N>
__device__ inline void ls_finish(const double* part, const int (&v)[N], int G, double (&x)[N],
                                 double (&out)[N], double (*lds)[kWavesPerBlock]) {
  for (int b = threadIdx.x + kBlock; b < G; b += kBlock) {
    double y[N];
#pragma unroll
    for (int k = 0; k < N; ++k) y[k] = part[(int64_t)v[k] * G + b];
#pragma unroll
    for (int k = 0; k < N; ++k) x[k] += y[k];
  }
#pragma unroll
  for (int k = 0; k < N; ++k) x[k] = wave_sum(x[k]);
  if (lane_id() == 0)
#pragma unroll
    for (int k = 0; k < N; ++k) lds[k][wave_in_block()] = x[k];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < N; ++k) out[k] = ((lds[k][0] + lds[k][1]) + lds[k][2]) + lds[k][3];
  __syncthreads();
}

template <int N>
__device__ inline void ls_totals(const double* part, const int (&v)[N], int G, double (&out)[N],
                                 double (*lds)[kWavesPerBlock]) {
  double x[N];
  ls_load(part, v, G, x);
  ls_finish(part, v, G, x, out, lds);
}

// Candidates q >= kQGroup (none of the first group passed: rare), in one
// block: one pass over the listed rows per candidate, in Algorithm 4's
// order, until the test passes.  Returns the accepted q (or -1) with its
// step and objective change.
template <int LOSS>
__device__ inline int rows_more_candidates(const RowsArgs& a, int64_t nr, int64_t hi_act,
                                           double& Dq, double& al, double& dF, double& margin,
                                           double* lds4) {
  const int lane = lane_id(), wv = wave_in_block();
  for (int q = kQGroup; q < a.Q; ++q) {
    double sl = 0.0, sla = 0.0;
    for (int64_t r = wv; r < nr; r += kWavesPerBlock) {
      const int32_t cnt = a.u_cnt[r];
      for (int32_t i = lane; i < cnt; i += kWave) {
        const int32_t row = a.u_row[r * kRangeW + i];
        double s = a.u_dtx[r * kRangeW + i];
        for (int t = 0; t < q; ++t) s *= a.beta;
        const double c = a.cache[row];
        const int yi = (int)a.y[row];
        const double t = loss_delta<LOSS>(c, yi, s);
        sl += t;
        sla += loss_delta_scale<LOSS>(c, yi, s, t);
      }
    }
    double l1 = 0.0, l1a = 0.0;
    for (int64_t slot = a.slot_lo + threadIdx.x; slot < hi_act; slot += kBlock) {
      const double wj = a.pw[slot], sj = al * a.d[slot];
      const double rc = reg_change(wj, sj, a.ra, a.rb);
      l1 += rc;
      l1a += reg_change_scale(wj, sj, a.ra, a.rb);
    }
    const double sL = block_sum(sl, lds4);
    const double L1 = block_sum(l1, lds4);
    const double sLa = block_sum(sla, lds4);
    const double L1a = block_sum(l1a, lds4);
    const double f = L1 + *a.Cp * sL;
    margin = fmin(margin, armijo_margin(f, a.sigma * Dq, L1a + *a.Cp * sLa));
    if (f <= a.sigma * Dq) {
      dF = f;
      return q;
    }
    Dq *= a.beta;
    al *= a.beta;
  }
  return -1;
}

// Armijo decision and accept: every block takes the decision from the
// partials identically, so no block waits for another; then w_B += alpha
// d_B and the retained quantities of the listed rows are updated (e^{w^T x}
// multiplicatively, Algorithm 4; b_i -= y_i alpha d^T x_i).  When no
// candidate of the first group passes, block 0 alone tests the later ones
// and applies the step.
template <int LOSS>
__device__ inline void apply_row(const RowsArgs& a, int32_t row, double s, double c, int yi,
                                 int q_acc) {
  for (int t = 0; t < q_acc; ++t) s *= a.beta;
  store_retained<LOSS>(&a.cache[row], &a.rw[row],
                       LOSS == kLogistic ? c * exp(s) : c - (yi > 0 ? s : -s), yi, a.stats);
}

template <int LOSS, bool EARLY>
__device__ __forceinline__ void rows_apply_body(const RowsArgs& a, int64_t bid, int64_t nblk) {
  __shared__ double lds4[kWavesPerBlock];
  __shared__ double lds7[7][kWavesPerBlock];
  const int64_t hi_act = clipped_hi(a.slot_hi, a.p_active);
  if (hi_act <= a.slot_lo) return;  // no active feature in this bundle: nothing ran
  const double C = *a.Cp;
  const int nq = a.Q < kQGroup ? a.Q : kQGroup;
  constexpr int kR = kRangeW / kWave;
  const int lane = lane_id();
  // Delta, candidate 0's sums and scales, touched rows and nonzeros with
  // d_j != 0, in one pass over the partials.  EARLY: issued with them, before
  // the decision waits for them (the update's operands depend only on what
  // the d^T x launch wrote): the bundle's nonzero range, this thread's first
  // slot of the w update (w from its copy in partition order), then the
  // wavefront's first listed range (count, rows and d^T x, then the rows'
  // retained quantities and labels).  The executor's copy loads them after
  // the decision (registers held across it would cost it occupancy).
  const int first[7] = {2 * a.Q, 0, a.Q, 2 * a.Q + 3, 3 * a.Q + 3, 2 * a.Q + 1, 2 * a.Q + 2};
  double x7[7];
  ls_load(a.part, first, a.G, x7);
  const int64_t e0 = a.poff[a.slot_lo], e1 = a.poff[a.slot_hi];
  const int64_t sl0 = a.slot_lo + bid * kBlock + threadIdx.x;
  const bool own0 = EARLY && sl0 < hi_act;
  const int64_t nr = (e1 - e0 + kRangeW - 1) / kRangeW;
  const int64_t gwave = (bid * kBlock + threadIdx.x) / kWave;
  int32_t f0 = 0;
  double d0 = 0.0, w0 = 0.0;
  int32_t row0[kR];
  double sv0[kR], c0[kR];
  int y0[kR];
#pragma unroll
  for (int u = 0; u < kR; ++u) {
    row0[u] = -1;
    sv0[u] = c0[u] = 0.0;
    y0[u] = 0;
  }
  if (EARLY) {
    f0 = ldz(a.perm, own0, sl0, 0);
    d0 = ldz(a.d, own0, sl0, 0.0);
    w0 = ldz(a.pw, own0, sl0, 0.0);
    // the count depends on nothing the offsets give: the d^T x launch wrote
    // one (0 past the bundle's ranges) for every wavefront of this grid
    const int32_t cnt0 = ldz(a.u_cnt, gwave < a.u_cap, gwave, 0);
#pragma unroll
    for (int u = 0; u < kR; ++u) {
      const int32_t i = lane + u * kWave;
      row0[u] = ldz(a.u_row, i < cnt0, gwave * kRangeW + i, -1);
      sv0[u] = ldz(a.u_dtx, i < cnt0, gwave * kRangeW + i, 0.0);
    }
#pragma unroll
    for (int u = 0; u < kR; ++u) {
      c0[u] = ldz(a.cache, row0[u] >= 0, row0[u], 0.0);
      y0[u] = (int)ldz(a.y, row0[u] >= 0, row0[u], (int8_t)0);
    }
    asm volatile("" ::"v"(f0), "v"(d0), "v"(w0));
#pragma unroll
    for (int u = 0; u < kR; ++u) asm volatile("" ::"v"(sv0[u]), "v"(c0[u]), "v"(y0[u]));
  }
  double tot[7];
  ls_finish(a.part, first, a.G, x7, tot, lds7);
  const double Delta = tot[0];
  double Dq = Delta, al = 1.0, dF = 0.0, margin = INFINITY;
  int q_acc = -1;
  for (int q = 0; q < nq; ++q) {
    const double sL = q == 0 ? tot[1] : ls_total(a.part, q, a.G, lds4);
    const double l1 = q == 0 ? tot[2] : ls_total(a.part, a.Q + q, a.G, lds4);
    const double f = l1 + C * sL;
    if (bid == 0) {  // only block 0 records the margin
      const double sabs = q == 0 ? tot[3] : ls_total(a.part, 2 * a.Q + 3 + q, a.G, lds4);
      const double l1abs = q == 0 ? tot[4] : ls_total(a.part, 3 * a.Q + 3 + q, a.G, lds4);
      margin = fmin(margin, armijo_margin(f, a.sigma * Dq, l1abs + C * sabs));
    }
    if (f <= a.sigma * Dq) {
      q_acc = q;
      dF = f;
      break;
    }
    Dq *= a.beta;
    al *= a.beta;
  }
  const double touched = tot[5];
  const double nz_d = tot[6];
  bool alone = false;
  if (q_acc < 0 && a.Q > nq) {
    if (bid != 0) return;
    alone = true;
    q_acc = rows_more_candidates<LOSS>(a, nr, hi_act, Dq, al, dF, margin, lds4);
  }
  if (bid == 0 && threadIdx.x == 0) {
    a.st->q = q_acc;
    a.st->alpha = q_acc >= 0 ? al : 0.0;
    a.st->dF = dF;
    a.st->delta = Delta;
    atomicAdd(&a.stats->bundles, 1ull);
    atomicAdd(&a.stats->ls_steps, (unsigned long long)(q_acc >= 0 ? q_acc + 1 : a.max_ls));
    if (q_acc < 0) atomicAdd(&a.stats->ls_fail, 1ull);
    atomicAdd(&a.stats->rows_touched, (unsigned long long)touched);
    atomicAdd(&a.stats->nnz_scat_rows, (unsigned long long)nz_d);
    atomicMin(&a.stats->min_margin_bits, (unsigned long long)__double_as_longlong(margin));
  }
  if (q_acc < 0) return;
  // w_B += alpha d_B and the listed rows' retained quantities; block 0 alone
  // when it tested the later candidates (the loaded operands then go unused)
  const int64_t wave = alone ? wave_in_block() : gwave;
  const int64_t nwaves = alone ? kWavesPerBlock : nblk * kWavesPerBlock;
  int64_t r = wave;
  if (EARLY && !alone && r < nr) {
#pragma unroll
    for (int u = 0; u < kR; ++u)
      if (row0[u] >= 0) apply_row<LOSS>(a, row0[u], sv0[u], c0[u], y0[u], q_acc);
    r += nwaves;
  }
  for (; r < nr; r += nwaves) {
    const int32_t cnt = a.u_cnt[r];
    int32_t row[kR];
    double s[kR], c[kR];
    int yi[kR];
#pragma unroll
    for (int u = 0; u < kR; ++u) {
      const int32_t i = lane + u * kWave;
      row[u] = ldz(a.u_row, i < cnt, r * kRangeW + i, -1);
      s[u] = ldz(a.u_dtx, i < cnt, r * kRangeW + i, 0.0);
    }
#pragma unroll
    for (int u = 0; u < kR; ++u) {
      c[u] = ldz(a.cache, row[u] >= 0, row[u], 0.0);
      yi[u] = (int)ldz(a.y, row[u] >= 0, row[u], (int8_t)0);
    }
#pragma unroll
    for (int u = 0; u < kR; ++u) asm volatile("" ::"v"(s[u]), "v"(c[u]), "v"(yi[u]));
#pragma unroll
    for (int u = 0; u < kR; ++u)
      if (row[u] >= 0) apply_row<LOSS>(a, row[u], s[u], c[u], yi[u], q_acc);
  }
  const int64_t tid = alone ? threadIdx.x : bid * kBlock + threadIdx.x;
  const int64_t nthr = alone ? kBlock : nblk * kBlock;
  int64_t sl = a.slot_lo + tid;
  if (!alone && own0) {
    a.w[f0] = w0 + al * d0;
    sl += nthr;
  }
  for (; sl < hi_act; sl += nthr) a.w[a.perm[sl]] = a.pw[sl] + al * a.d[sl];
}

template <int LOSS>
__global__ __launch_bounds__(kBlock) void k_rows_apply(RowsArgs a) {
  rows_apply_body<LOSS, true>(a, blockIdx.x, gridDim.x);
}

// d^T x of the listed rows into a dense vector (pcdn_step's read-back).
__global__ __launch_bounds__(kBlock) void k_rows_scatter(RowsArgs a, double* dense) {
  const int64_t e0 = a.poff[a.slot_lo], e1 = a.poff[a.slot_hi];
  const int64_t nr = (e1 - e0 + kRangeW - 1) / kRangeW;
  for (int64_t r = blockIdx.x; r < nr; r += gridDim.x) {
    const int32_t cnt = a.u_cnt[r];
    for (int32_t i = threadIdx.x; i < cnt; i += kBlock)
      dense[a.u_row[r * kRangeW + i]] = a.u_dtx[r * kRangeW + i];
  }
}

// ---------------------------------------------------------------------------
// bundle-row order: islot, column lengths and offsets in slot order, then a
// stable counting sort of the CSR copy by bundle (8-bit digits, tiles of
// kBrTile nonzeros; stability inside a round from wavefront peer masks built
// with ballots, across waves and rounds from per-digit running offsets)
// ---------------------------------------------------------------------------
constexpr int kBrTile = kSortThreads * kBrRounds;

__global__ void k_fill_i32(int32_t* a, int32_t v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    a[i] = v;
}

__device__ __forceinline__ uint32_t br_digit_of(const BrArgs& a, int32_t slot) {
  const uint32_t b = slot >= 0 ? (uint32_t)slot / (uint32_t)a.P : (uint32_t)a.nb;
  return (b >> a.shift) & 255u;
}

// Digit counts of one tile.  Every round's loads are issued before any is
// used; with islot (pass 0) the slots are also written out (slot_out, in
// source order) for the scatter pass, which then needs no gather.
__device__ __forceinline__ void br_hist_body(const BrArgs& a, int64_t bid) {
  __shared__ int32_t cnt[256];
  cnt[threadIdx.x] = 0;
  const int64_t base = bid * kBrTile;
  int32_t sl[kBrRounds];
#pragma unroll
  for (int r = 0; r < kBrRounds; ++r) {
    const int64_t i = base + r * kSortThreads + threadIdx.x;
    sl[r] = ldz(a.scol, i < a.m, i, 0);
  }
  if (a.islot) {
#pragma unroll
    for (int r = 0; r < kBrRounds; ++r) {
      const int64_t i = base + r * kSortThreads + threadIdx.x;
      sl[r] = ldz(a.islot, i < a.m, sl[r], 0);
    }
#pragma unroll
    for (int r = 0; r < kBrRounds; ++r) {
      const int64_t i = base + r * kSortThreads + threadIdx.x;
      if (i < a.m) a.slot_out[i] = sl[r];
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kBrRounds; ++r) {
    const int64_t i = base + r * kSortThreads + threadIdx.x;
    if (i < a.m) atomicAdd(&cnt[br_digit_of(a, sl[r])], 1);
  }
  __syncthreads();
  a.hist[(int64_t)threadIdx.x * a.ntiles + bid] = cnt[threadIdx.x];
}

__global__ __launch_bounds__(kSortThreads) void k_br_hist(BrArgs a) { br_hist_body(a, blockIdx.x); }

// Scatter of one tile (scol holds slots: the hist pass wrote them).  The
// tile's rows, slots and values are loaded before the ranking rounds.
__device__ __forceinline__ void br_scatter_body(const BrArgs& a, int64_t bid) {
  __shared__ int32_t base_off[256];
  __shared__ int32_t wcnt[kWavesPerBlock][256];
  base_off[threadIdx.x] = a.hist[(int64_t)threadIdx.x * a.ntiles + bid];
  const int lane = lane_id(), wv = wave_in_block();
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int64_t tile = bid * kBrTile;
  int32_t rrow[kBrRounds], rslot[kBrRounds];
  float rval[kBrRounds];
#pragma unroll
  for (int r = 0; r < kBrRounds; ++r) {
    const int64_t i = tile + r * kSortThreads + threadIdx.x;
    const bool valid = i < a.m;
    rrow[r] = ldz(a.srow, valid, i, 0);
    rslot[r] = ldz(a.scol, valid, i, 0);
    rval[r] = ldz(a.sval, valid, i, 0.0f);
  }
#pragma unroll
  for (int r = 0; r < kBrRounds; ++r) {
#pragma unroll
    for (int w = 0; w < kWavesPerBlock; ++w) wcnt[w][threadIdx.x] = 0;
    __syncthreads();
    const int64_t i = tile + r * kSortThreads + threadIdx.x;
    const bool valid = i < a.m;
    const uint32_t dig = valid ? br_digit_of(a, rslot[r]) : 0u;
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (dig >> b) & 1u;
      const uint64_t bal = __ballot(bit);
      peers &= bit ? bal : ~bal;
    }
    const int rank = __popcll(peers & lt_mask);
    const bool leader = valid && ((peers & lt_mask) == 0);
    if (leader) wcnt[wv][dig] = __popcll(peers);
    __syncthreads();
    if (valid) {
      int32_t pos = base_off[dig] + rank;
      for (int w = 0; w < wv; ++w) pos += wcnt[w][dig];
      a.drow[pos] = rrow[r];
      a.dslot[pos] = rslot[r];
      a.dval[pos] = rval[r];
    }
    __syncthreads();
    int32_t add = 0;
#pragma unroll
    for (int w = 0; w < kWavesPerBlock; ++w) add += wcnt[w][threadIdx.x];
    base_off[threadIdx.x] += add;
  }
}

__global__ __launch_bounds__(kSortThreads) void k_br_scatter(BrArgs a) {
  br_scatter_body(a, blockIdx.x);
}

// The scatter pass of a standalone launch, with the tile staged in LDS: each
// nonzero is ranked as in br_scatter_body, but placed at its position in the
// tile's digit-sorted order in LDS, which is then stored in that order, so
// that consecutive threads store consecutive addresses of a digit's run (the
// stores straight from the ranking rounds put a few nonzeros per digit and
// round).  The positions are the same, so the output is too.  (The executor
// keeps br_scatter_body: its LDS is shared by every task body.)
__global__ __launch_bounds__(kSortThreads) void k_br_scatter_staged(BrArgs a) {
  __shared__ int32_t gbase[256];  // output position of the tile's first nonzero of each digit
  __shared__ int32_t lbase[256];  // the same inside the tile's sorted order
  __shared__ int32_t run_off[256];
  __shared__ int32_t wcnt[kWavesPerBlock][256];
  __shared__ int32_t lds_scan[kSortThreads / kWave + 1];
  __shared__ int32_t s_row[kBrTile], s_slot[kBrTile];
  __shared__ float s_val[kBrTile];
  const int64_t bid = blockIdx.x;
  const int lane = lane_id(), wv = wave_in_block();
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int64_t tile = bid * kBrTile;
  const int32_t tcount = (int32_t)(a.m - tile < kBrTile ? a.m - tile : kBrTile);
  gbase[threadIdx.x] = a.hist[(int64_t)threadIdx.x * a.ntiles + bid];
  wcnt[0][threadIdx.x] = 0;
  int32_t rrow[kBrRounds], rslot[kBrRounds];
  float rval[kBrRounds];
  uint32_t dig[kBrRounds];
#pragma unroll
  for (int r = 0; r < kBrRounds; ++r) {
    const int64_t i = tile + r * kSortThreads + threadIdx.x;
    const bool valid = i < a.m;
    rrow[r] = ldz(a.srow, valid, i, 0);
    rslot[r] = ldz(a.scol, valid, i, 0);
    rval[r] = ldz(a.sval, valid, i, 0.0f);
  }
  __syncthreads();
  // the tile's digit counts, then their exclusive scan
#pragma unroll
  for (int r = 0; r < kBrRounds; ++r) {
    const bool valid = r * kSortThreads + (int)threadIdx.x < tcount;
    dig[r] = valid ? br_digit_of(a, rslot[r]) : 0u;
    if (valid) atomicAdd(&wcnt[0][dig[r]], 1);
  }
  __syncthreads();
  int32_t total;
  const int32_t lb = block_exclusive_scan<kSortThreads>(wcnt[0][threadIdx.x], lds_scan, &total);
  lbase[threadIdx.x] = lb;
  run_off[threadIdx.x] = lb;
#pragma unroll
  for (int r = 0; r < kBrRounds; ++r) {
#pragma unroll
    for (int w = 0; w < kWavesPerBlock; ++w) wcnt[w][threadIdx.x] = 0;
    __syncthreads();
    const bool valid = r * kSortThreads + (int)threadIdx.x < tcount;
    const uint32_t d = dig[r];
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t bal = __ballot(bit);
      peers &= bit ? bal : ~bal;
    }
    const int rank = __popcll(peers & lt_mask);
    const bool leader = valid && ((peers & lt_mask) == 0);
    if (leader) wcnt[wv][d] = __popcll(peers);
    __syncthreads();
    if (valid) {
      int32_t pos = run_off[d] + rank;
      for (int w = 0; w < wv; ++w) pos += wcnt[w][d];
      s_row[pos] = rrow[r];
      s_slot[pos] = rslot[r];
      s_val[pos] = rval[r];
    }
    __syncthreads();
    int32_t add = 0;
#pragma unroll
    for (int w = 0; w < kWavesPerBlock; ++w) add += wcnt[w][threadIdx.x];
    run_off[threadIdx.x] += add;
  }
  __syncthreads();
  for (int32_t e = threadIdx.x; e < tcount; e += kSortThreads) {
    const int32_t sl = s_slot[e];
    const uint32_t d = br_digit_of(a, sl);
    const int64_t g = (int64_t)gbase[d] + (e - lbase[d]);
    a.drow[g] = s_row[e];
    a.dslot[g] = sl;
    a.dval[g] = s_val[e];
  }
}

// ---------------------------------------------------------------------------
// Single-workgroup schedule: one 512-thread workgroup runs every bundle of an
// outer iteration of one problem, phase after phase, with workgroup barriers
// as the only synchronisation (no kernel boundary per bundle).  Same
// arithmetic as the multi-kernel path.  Small bundles are bound by the
// latency of dependent memory accesses, so a bundle is arranged to need few:
//  - X has been copied into partition order (k_permute), so a bundle's
//    nonzeros are one contiguous range: thread v takes nonzero v, and a
//    segmented wavefront scan (keys = slot) sums g_j, h_j; slots that cross a
//    64-nonzero chunk are completed from LDS partials in chunk order, so the
//    sums are deterministic;
//  - d^T x is accumulated in 64-bit fixed point: each term d_j x_ij is
//    rounded to a multiple of 2^-e, where 2^-e is set by the bundle's
//    largest |d_j| and the largest row 1-norm of X so that no partial sum can
//    overflow, and integer additions give the same sum in any order: d^T x
//    does not depend on timing;
//  - with bundle-local row ids (k_bundle_rows, at most kNarrowLidCap distinct
//    rows) d^T x is accumulated in LDS by local id, and the thread that first
//    touches a row (an LDS bit per id) records the row, its retained
//    quantity and label, already in its registers, at the row's local id;
//    the line search and the apply then run over the local ids in order and
//    touch global memory only to write the updated retained quantities;
//  - otherwise (more distinct rows, or no ids) d^T x is accumulated in global
//    memory with L2 integer atomics, and the line search and the apply pass
//    over every sample;
//  - candidates are tested one pass at a time in increasing q (Algorithm 4's
//    order), so an accepted unit step costs a single pass.
// ---------------------------------------------------------------------------
constexpr int kNarrowBlock = 512;      // 256 VGPRs per lane: no spills
constexpr int kNarrowWaves = kNarrowBlock / kWave;
constexpr int kNarrowRegRounds = 4;    // rounds of nonzeros loaded together, kept in registers
constexpr int kNarrowChunkCap = 512;   // 64-nonzero chunks with LDS partials
constexpr int kTouchCap = 4096;        // touched rows listed per bundle

__device__ inline double block_sum16(double v, double* lds16) {
  v = wave_sum(v);
  if (lane_id() == 0) lds16[wave_in_block()] = v;
  __syncthreads();
  double r = 0.0;
#pragma unroll
  for (int k = 0; k < kNarrowWaves; ++k) r += lds16[k];
  __syncthreads();
  return r;
}

// Sum of up to four per-thread values over the workgroup in a fixed order
// (wavefront DPP sums, then the waves in index order); every thread gets the
// totals.  Double-buffered LDS: one barrier per call suffices because a buffer
// is rewritten only two calls later, after another barrier.
template <int NV>
__device__ inline void block_sums(double (&v)[NV], double (*red)[kNarrowWaves][6], int& buf) {
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = wave_sum(v[i]);
  if (lane_id() == 0)
#pragma unroll
    for (int i = 0; i < NV; ++i) red[buf][wave_in_block()][i] = v[i];
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kNarrowWaves; ++w) s += red[buf][w][i];
    v[i] = s;
  }
  buf ^= 1;
}

// Fixed-point d^T x: a term in units of 2^-e (sc = 2^e) and back.
__device__ inline unsigned long long fx_term(double dj, float x, double sc) {
  return (unsigned long long)(long long)rint((dj * (double)x) * sc);
}
__device__ inline double fx_value(unsigned long long acc, double isc) {
  return (double)(long long)acc * isc;
}

// Exponent e of the bundle's fixed-point scale: with D = max |d_j| and
// xrow = max_i sum_j |x_ij|, every partial sum of d^T x_i is below
// D xrow < 2^(ilogb(D) + ilogb(xrow) + 2), so units of 2^-e with
// e = 59 - ilogb(D) - ilogb(xrow) keep it below 2^61 (64-bit sums cannot
// overflow, whatever the order); clamped so that 2^e and 2^-e are normal.
__device__ inline int fx_exponent(double D, double xrow) {
  if (!(D > 0.0) || !(D <= 1.7976931348623157e308)) return 0;  // no nonzero (finite) term
  int e = 59 - ilogb(D) - ilogb(xrow > 0.0 ? xrow : 1.0);
  return e < -1000 ? -1000 : (e > 1000 ? 1000 : e);
}

// The global fixed-point d^T x is built with L2 atomics while a stale copy
// of the line may sit in the CU's L1: read it at workgroup scope, which
// bypasses L1 and is served by the L2 of this XCD.  The single-workgroup
// kernel's problem state is touched by no other workgroup while it runs
// (kernel boundaries make it visible to the rest of the GPU), so workgroup
// scope suffices; agent scope would also ask for coherence with the other
// XCDs' L2s and go to the memory side.
__device__ inline unsigned long long load_l2_fx(const double* p) {
  return __hip_atomic_load((const unsigned long long*)p, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Bundle-local row ids for the single-workgroup schedule: one workgroup per
// bundle marks the rows of its nonzeros in an LDS bitmap of the n rows; a
// row's id is the number of marked rows below it (so ids follow the row
// order and do not depend on timing), found from per-word prefix counts.
constexpr int kRowsBlock = 256;

__global__ __launch_bounds__(kRowsBlock) void k_bundle_rows(const int64_t* poff,
                                                            const int32_t* pri, int64_t p_slots,
                                                            int64_t P, int64_t n, uint16_t* plid,
                                                            int32_t* pR) {
  extern __shared__ uint32_t rows_lds[];
  __shared__ uint32_t part[kRowsBlock];
  const int64_t words = (n + 31) >> 5;
  uint32_t* bits = rows_lds;
  uint32_t* pre = rows_lds + words;
  const int64_t t = blockIdx.x;
  const int64_t lo = t * P, hi = lo + P < p_slots ? lo + P : p_slots;
  const int64_t k0 = poff[lo], k1 = poff[hi];
  for (int64_t w = threadIdx.x; w < words; w += kRowsBlock) bits[w] = 0u;
  __syncthreads();
  for (int64_t k = k0 + threadIdx.x; k < k1; k += kRowsBlock) {
    const int32_t r = pri[k];
    atomicOr(&bits[r >> 5], 1u << (r & 31));
  }
  __syncthreads();
  // exclusive prefix of the words' popcounts: thread i covers a contiguous
  // run of words, then an inclusive scan of the runs' counts
  const int64_t per = (words + kRowsBlock - 1) / kRowsBlock;
  const int64_t w0 = threadIdx.x * per, w1 = w0 + per < words ? w0 + per : words;
  uint32_t cnt = 0;
  for (int64_t w = w0; w < w1; ++w) cnt += __popc(bits[w]);
  part[threadIdx.x] = cnt;
  __syncthreads();
  for (int off = 1; off < kRowsBlock; off <<= 1) {
    const uint32_t add = threadIdx.x >= off ? part[threadIdx.x - off] : 0u;
    __syncthreads();
    part[threadIdx.x] += add;
    __syncthreads();
  }
  uint32_t run = part[threadIdx.x] - cnt;
  for (int64_t w = w0; w < w1; ++w) {
    pre[w] = run;
    run += __popc(bits[w]);
  }
  const uint32_t R = part[kRowsBlock - 1];
  __syncthreads();
  if (threadIdx.x == 0) pR[t] = R <= (uint32_t)kNarrowLidCap ? (int32_t)R : -1;
  if (R > (uint32_t)kNarrowLidCap) return;
  for (int64_t k = k0 + threadIdx.x; k < k1; k += kRowsBlock) {
    const int32_t r = pri[k];
    const uint32_t below = bits[r >> 5] & ((1u << (r & 31)) - 1u);
    plid[k] = (uint16_t)(pre[r >> 5] + __popc(below));
  }
}

static_assert(kNarrowLidCap <= kTouchCap, "local row ids index the LDS row lists");

struct NarrowLds {
  double lds16[kNarrowWaves];
  double red[2][kNarrowWaves][6];
  double dmx[kNarrowWaves];             // per-wave max |d_j|
  int32_t any_d;                        // some direction of the bundle is nonzero
  int32_t off[kNarrowMaxP + 1];        // nonzero offsets of the bundle's slots
  int32_t feat[kNarrowMaxP];
  double w[kNarrowMaxP];
  double d[kNarrowMaxP];
  double2 acc[kNarrowMaxP];            // (sum g terms, sum h terms) per slot
  double2 pf[kNarrowChunkCap];         // first segment of each 64-nonzero chunk
  double2 pl[kNarrowChunkCap];         // last segment of each chunk
  // by local row id: the row, its label and retained quantity (written by
  // the row's first toucher), and the fixed-point d^T x
  int32_t t_row[kTouchCap];
  uint32_t t_seen[kTouchCap / 32];     // local row ids already recorded
  int8_t t_y[kTouchCap];
  double t_c[kTouchCap];
  unsigned long long t_acc[kTouchCap];
};

// slot of bundle nonzero v: the largest s with off[s] <= v
__device__ inline int32_t slot_of(const int32_t* off, int32_t nslots, int32_t v) {
  int32_t lo = 0, hi = nslots;  // off[lo] <= v < off[hi]
  while (hi - lo > 1) {
    const int32_t mid = (lo + hi) >> 1;
    if (off[mid] <= v) lo = mid; else hi = mid;
  }
  return lo;
}

// Record a row at its local id (first toucher only).
__device__ inline void list_lid(NarrowLds& L, int32_t lid, int32_t row, double c, int yi) {
  L.t_row[lid] = row;
  L.t_c[lid] = c;
  L.t_y[lid] = (int8_t)yi;
}

// One round of the sweep for bundle nonzero v (slot s, row, value x, the
// row's retained quantity c and label yi): its g, h terms, the segmented
// wavefront sums, and the per-slot or per-chunk record of each segment end.
// Every lane of the wavefront calls it (lanes past nb carry slot -1).
template <int LOSS>
__device__ __forceinline__ void narrow_term(NarrowLds& L, int32_t v, int32_t nb, int32_t ns,
                                            int32_t row, float x, double c, int yi, int32_t s,
                                            double2* pf, double2* pl) {
  (void)row;
  (void)ns;
  const bool valid = v < nb;
  if (!valid) s = -1;
  double g = 0.0, h = 0.0;
  if (valid) grad_hess_term<LOSS>(c, yi, (double)x, g, h);
  // inclusive segmented scan over the wavefront (slots ascend along lanes;
  // lanes past the end carry slot -1 and zero terms)
  seg_scan(g, h, s);
  const bool seg_end = valid && next_lane_key(s) != s;
  if (seg_end) {
    const int32_t m = v / kWave;                 // chunk of this nonzero
    const int32_t cbeg = m * kWave, cend = cbeg + kWave - 1;
    const bool left_open = L.off[s] < cbeg;
    const bool right_open = L.off[s + 1] - 1 > cend;
    if (!left_open && !right_open)
      L.acc[s] = make_double2(g, h);             // the slot lies in this chunk
    else if (left_open)
      pf[m] = make_double2(g, h);                // first segment of chunk m
    else
      pl[m] = make_double2(g, h);                // last segment of chunk m
  }
}

template <int LOSS>
__device__ __forceinline__ void narrow_body(const NarrowArgs& na, NarrowLds& L) {
  const SweepArgs& a = na.sw;
  const int tid = threadIdx.x;
  double n_bundles = 0.0, n_ls = 0.0, n_fail = 0.0, n_touched = 0.0, margin = INFINITY;
  double n_nnz = 0.0, n_slots = 0.0;      // uniform
  double n_scat = 0.0, n_scat_long = 0.0;  // this thread's slots
  const double Cv = *a.Cp;
  int64_t t_end = na.t_end, p_lim = na.p;
  if (na.p_active) {  // shrinking: bundles of the active features only
    const int64_t pa = (int64_t)*na.p_active;
    if (pa < p_lim) p_lim = pa;
    const int64_t te = (p_lim + na.P - 1) / na.P;
    if (te < t_end) t_end = te;
  }
  for (int64_t t = na.t_begin; t < t_end; ++t) {
    const int64_t lo = t * na.P;
    const int64_t hi = lo + na.P < p_lim ? lo + na.P : p_lim;
    const int32_t ns = (int32_t)(hi - lo);
    const int64_t base = na.poff[lo];
    // bundle metadata into LDS; clear the per-slot sums
    for (int32_t s = tid; s <= ns; s += kNarrowBlock) L.off[s] = (int32_t)(na.poff[lo + s] - base);
    for (int32_t s = tid; s < ns; s += kNarrowBlock) {
      L.feat[s] = na.perm[lo + s];
      L.w[s] = na.pw[lo + s];  // no load that waits on perm
      L.acc[s] = make_double2(0.0, 0.0);
    }
    if (tid == 0) L.any_d = 0;
    // distinct rows of the bundle with d^T x kept in LDS (t_row/t_c/t_y/t_acc
    // indexed by local row id), or -1: d^T x in global memory
    const int32_t R = na.pR ? na.pR[t] : -1;
    for (int32_t e = tid; e < R; e += kNarrowBlock) L.t_acc[e] = 0ull;
    for (int32_t e = tid; e < (R + 31) / 32; e += kNarrowBlock) L.t_seen[e] = 0u;
    __syncthreads();
    const int32_t nb = L.off[ns];
    const int32_t nchunks = (nb + kWave - 1) / kWave;
    double2* pf = nchunks <= kNarrowChunkCap ? L.pf : na.part;
    double2* pl = nchunks <= kNarrowChunkCap ? L.pl : na.part + nchunks;
    // 1. sweep: nonzero v = r0 + tid; segmented wavefront sums per slot.
    //    The first kNarrowRegRounds rounds issue all their loads together.
    int32_t rrow[kNarrowRegRounds];
    float rx[kNarrowRegRounds];
    double rc[kNarrowRegRounds];
    int ry[kNarrowRegRounds];
    int32_t rs[kNarrowRegRounds];
    int32_t rl[kNarrowRegRounds];
#pragma unroll
    for (int u = 0; u < kNarrowRegRounds; ++u) {
      const int32_t v = u * kNarrowBlock + tid;
      rrow[u] = ldz(na.pri, v < nb, base + v, 0);
      rx[u] = ldz(na.pv, v < nb, base + v, 0.0f);
      rl[u] = R >= 0 ? (int32_t)ldz(na.plid, v < nb, base + v, (uint16_t)0) : 0;
    }
#pragma unroll
    for (int u = 0; u < kNarrowRegRounds; ++u) {
      const int32_t v = u * kNarrowBlock + tid;
      rs[u] = v < nb ? slot_of(L.off, ns, v) : -1;
      rc[u] = ldz(a.cache, v < nb, rrow[u], 0.0);
      ry[u] = (int)ldz(a.y, v < nb, rrow[u], (int8_t)0);
    }
#pragma unroll
    for (int u = 0; u < kNarrowRegRounds; ++u)
      if (u * kNarrowBlock < nb)
        narrow_term<LOSS>(L, u * kNarrowBlock + tid, nb, ns, rrow[u], rx[u], rc[u], ry[u], rs[u],
                          pf, pl);
    // later rounds in groups of kNarrowRegRounds, each group's loads issued
    // together (two dependent round trips per group)
    for (int32_t g0 = kNarrowRegRounds * kNarrowBlock; g0 < nb;
         g0 += kNarrowRegRounds * kNarrowBlock) {
      int32_t grow[kNarrowRegRounds], gs[kNarrowRegRounds];
      float gx[kNarrowRegRounds];
      double gc[kNarrowRegRounds];
      int gy[kNarrowRegRounds];
#pragma unroll
      for (int u = 0; u < kNarrowRegRounds; ++u) {
        const int32_t v = g0 + u * kNarrowBlock + tid;
        grow[u] = ldz(na.pri, v < nb, base + v, 0);
        gx[u] = ldz(na.pv, v < nb, base + v, 0.0f);
      }
#pragma unroll
      for (int u = 0; u < kNarrowRegRounds; ++u) {
        const int32_t v = g0 + u * kNarrowBlock + tid;
        gs[u] = v < nb ? slot_of(L.off, ns, v) : -1;
        gc[u] = ldz(a.cache, v < nb, grow[u], 0.0);
        gy[u] = (int)ldz(a.y, v < nb, grow[u], (int8_t)0);
      }
#pragma unroll
      for (int u = 0; u < kNarrowRegRounds; ++u)
        if (g0 + u * kNarrowBlock < nb)
          narrow_term<LOSS>(L, g0 + u * kNarrowBlock + tid, nb, ns, grow[u], gx[u], gc[u], gy[u],
                            gs[u], pf, pl);
    }
    __syncthreads();
    // slots spanning several chunks: head (pl) + middle chunks (pf) + tail (pf)
    for (int32_t s = tid; s < ns; s += kNarrowBlock) {
      const int32_t b0 = L.off[s], b1 = L.off[s + 1];
      if (b1 - b0 == 0) continue;
      const int32_t m1 = b0 / kWave, m2 = (b1 - 1) / kWave;
      if (m1 == m2) continue;
      double2 tot = pl[m1];
      for (int32_t m = m1 + 1; m <= m2; ++m) {
        tot.x += pf[m].x;
        tot.y += pf[m].y;
      }
      L.acc[s] = tot;
    }
    __syncthreads();
    // finish each slot: g, h, d (eqs. (4)-(5), (11)), Delta term
    double del = 0.0, dmax = 0.0;
    for (int32_t s = tid; s < ns; s += kNarrowBlock) {
      double g, h;
      if (LOSS == kLogistic) {
        g = Cv * L.acc[s].x;
        h = Cv * L.acc[s].y;
      } else {
        g = -2.0 * Cv * L.acc[s].x;
        h = 2.0 * Cv * L.acc[s].y;
      }
      if (h <= 0.0) h += a.nu;
      const double wj = L.w[s];
      const double dj = newton_dir(g, h, wj, a.ra, a.rb);
      L.d[s] = dj;
      dmax = fmax(dmax, fabs(dj));
      if (dj != 0.0) {
        L.any_d = 1;
        const int32_t len = L.off[s + 1] - L.off[s];
        if (len > na.chunk)
          n_scat_long += (double)len;
        else
          n_scat += (double)len;
      }
      del += g * dj + a.gamma * h * dj * dj + reg_change(wj, dj, a.ra, a.rb);
      a.g[lo + s] = g;
      a.h[lo + s] = h;
      a.d[lo + s] = dj;
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) dmax = fmax(dmax, __shfl_xor(dmax, o, kWave));
    if (lane_id() == 0) L.dmx[wave_in_block()] = dmax;
    __syncthreads();  // publishes L.d; Delta's per-thread part stays in `del`
    if (L.any_d == 0 && !na.dtx_copy) {
      // every direction is zero: no row is touched, Delta = 0, the first
      // candidate passes (eq. (6): 0 <= 0) with dF = 0, and w and the
      // retained quantities stay as they are
      n_bundles += 1.0;
      n_nnz += (double)nb;
      n_slots += (double)ns;
      n_ls += 1.0;
      if (tid == 0 && t == t_end - 1) {
        na.st->q = 0;
        na.st->alpha = 1.0;
        na.st->dF = 0.0;
        na.st->delta = 0.0;
      }
      __syncthreads();
      continue;
    }
    // 2. scatter d_j x_ij into d^T x (fixed point, see above); record the
    //    touched rows with their retained quantity and label by local id.
    //    The register rounds issue every atomic before waiting on any.
    double D = L.dmx[0];
#pragma unroll
    for (int k = 1; k < kNarrowWaves; ++k) D = fmax(D, L.dmx[k]);
    const int fe = fx_exponent(D, na.xrow);
    const double sc = ldexp(1.0, fe), isc = ldexp(1.0, -fe);
    if (R >= 0) {
      // d^T x by local row id with LDS atomics; the first toucher of a row
      // (LDS bit per local id) records it: no global memory traffic
#pragma unroll
      for (int u = 0; u < kNarrowRegRounds; ++u) {
        if (u * kNarrowBlock + tid < nb) {
          const double dj = L.d[rs[u]];
          if (dj != 0.0) {
            atomicAdd(&L.t_acc[rl[u]], fx_term(dj, rx[u], sc));
            const uint32_t bit = 1u << (rl[u] & 31);
            if ((atomicOr(&L.t_seen[rl[u] >> 5], bit) & bit) == 0u)
              list_lid(L, rl[u], rrow[u], rc[u], ry[u]);
          }
        }
      }
      // later rounds in groups, loads of a group issued together
      for (int32_t g0 = kNarrowRegRounds * kNarrowBlock; g0 < nb;
           g0 += kNarrowRegRounds * kNarrowBlock) {
        double gd[kNarrowRegRounds], gc[kNarrowRegRounds];
        int32_t glid[kNarrowRegRounds], grow[kNarrowRegRounds];
        float gx[kNarrowRegRounds];
        int gy[kNarrowRegRounds];
        bool first[kNarrowRegRounds];
#pragma unroll
        for (int u = 0; u < kNarrowRegRounds; ++u) {
          const int32_t v = g0 + u * kNarrowBlock + tid;
          gd[u] = v < nb ? L.d[slot_of(L.off, ns, v)] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kNarrowRegRounds; ++u) {
          const int32_t v = g0 + u * kNarrowBlock + tid;
          const bool on = gd[u] != 0.0;
          glid[u] = (int32_t)ldz(na.plid, on, base + v, (uint16_t)0);
          gx[u] = ldz(na.pv, on, base + v, 0.0f);
          grow[u] = ldz(na.pri, on, base + v, 0);
        }
#pragma unroll
        for (int u = 0; u < kNarrowRegRounds; ++u) {
          first[u] = false;
          if (gd[u] != 0.0) {
            atomicAdd(&L.t_acc[glid[u]], fx_term(gd[u], gx[u], sc));
            const uint32_t bit = 1u << (glid[u] & 31);
            first[u] = (atomicOr(&L.t_seen[glid[u] >> 5], bit) & bit) == 0u;
          }
        }
#pragma unroll
        for (int u = 0; u < kNarrowRegRounds; ++u) {
          gc[u] = ldz(a.cache, first[u], grow[u], 0.0);
          gy[u] = (int)ldz(a.y, first[u], grow[u], (int8_t)0);
        }
#pragma unroll
        for (int u = 0; u < kNarrowRegRounds; ++u)
          if (first[u]) list_lid(L, glid[u], grow[u], gc[u], gy[u]);
      }
    } else {
      unsigned long long* gacc = (unsigned long long*)a.dtx;
#pragma unroll
      for (int u = 0; u < kNarrowRegRounds; ++u) {
        if (u * kNarrowBlock + tid < nb) {
          const double dj = L.d[rs[u]];
          if (dj != 0.0) atomicAdd(&gacc[rrow[u]], fx_term(dj, rx[u], sc));
        }
      }
      for (int32_t g0 = kNarrowRegRounds * kNarrowBlock; g0 < nb;
           g0 += kNarrowRegRounds * kNarrowBlock) {
        double gd[kNarrowRegRounds];
        int32_t grow[kNarrowRegRounds];
        float gx[kNarrowRegRounds];
#pragma unroll
        for (int u = 0; u < kNarrowRegRounds; ++u) {
          const int32_t v = g0 + u * kNarrowBlock + tid;
          gd[u] = v < nb ? L.d[slot_of(L.off, ns, v)] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kNarrowRegRounds; ++u) {
          const int32_t v = g0 + u * kNarrowBlock + tid;
          const bool on = gd[u] != 0.0;
          grow[u] = ldz(na.pri, on, base + v, 0);
          gx[u] = ldz(na.pv, on, base + v, 0.0f);
        }
#pragma unroll
        for (int u = 0; u < kNarrowRegRounds; ++u)
          if (gd[u] != 0.0) atomicAdd(&gacc[grow[u]], fx_term(gd[u], gx[u], sc));
      }
    }
    __syncthreads();
    const bool listed = R >= 0;
    // 3. candidates q = 0, 1, ... until the Armijo test (eq. (6)) holds
    int rbuf = 0;
    double Delta = 0.0, Dq = 0.0, al = 1.0, dF = 0.0;
    int q_acc = -1;
    for (int q = 0; q < na.max_ls; ++q) {
      double sl = 0.0, l1 = 0.0, touched = 0.0, sla = 0.0, l1a = 0.0;
      if (listed) {
        for (int32_t e = tid; e < R; e += kNarrowBlock) {
          const unsigned long long ac = L.t_acc[e];
          if (ac == 0ull) continue;
          touched += 1.0;
          double sv = fx_value(ac, isc);
          for (int u = 0; u < q; ++u) sv *= na.beta;
          const double ld = loss_delta<LOSS>(L.t_c[e], (int)L.t_y[e], sv);
          sl += ld;
          sla += loss_delta_scale<LOSS>(L.t_c[e], (int)L.t_y[e], sv, ld);
        }
      } else {
        // every sample, the loads of kNarrowRegRounds samples issued
        // together; a fixed summation order
        for (int64_t i0 = tid; i0 < na.n; i0 += (int64_t)kNarrowRegRounds * kNarrowBlock) {
          unsigned long long fa[kNarrowRegRounds];
          double fc[kNarrowRegRounds];
          int fy[kNarrowRegRounds];
#pragma unroll
          for (int u = 0; u < kNarrowRegRounds; ++u) {
            const int64_t i = i0 + (int64_t)u * kNarrowBlock;
            fa[u] = i < na.n ? load_l2_fx(&a.dtx[i]) : 0ull;
          }
#pragma unroll
          for (int u = 0; u < kNarrowRegRounds; ++u) {
            const int64_t i = i0 + (int64_t)u * kNarrowBlock;
            fc[u] = fa[u] != 0ull ? a.cache[i] : 0.0;
            fy[u] = fa[u] != 0ull ? (int)a.y[i] : 0;
          }
#pragma unroll
          for (int u = 0; u < kNarrowRegRounds; ++u) {
            if (fa[u] != 0ull) {
              touched += 1.0;
              double sv = fx_value(fa[u], isc);
              for (int k = 0; k < q; ++k) sv *= na.beta;
              const double ld = loss_delta<LOSS>(fc[u], fy[u], sv);
              sl += ld;
              sla += loss_delta_scale<LOSS>(fc[u], fy[u], sv, ld);
            }
          }
        }
      }
      for (int32_t s = tid; s < ns; s += kNarrowBlock) {
        const double rc = reg_change(L.w[s], al * L.d[s], a.ra, a.rb);
        l1 += rc;
        l1a += reg_change_scale(L.w[s], al * L.d[s], a.ra, a.rb);
      }
      double sL, L1, sLa, L1a;
      if (q == 0) {
        double v6[6] = {sl, l1, del, touched, sla, l1a};
        block_sums<6>(v6, L.red, rbuf);
        sL = v6[0];
        L1 = v6[1];
        Delta = v6[2];
        Dq = Delta;
        n_touched += v6[3];
        sLa = v6[4];
        L1a = v6[5];
      } else {
        double v4[4] = {sl, l1, sla, l1a};
        block_sums<4>(v4, L.red, rbuf);
        sL = v4[0];
        L1 = v4[1];
        sLa = v4[2];
        L1a = v4[3];
      }
      const double f = L1 + Cv * sL;
      margin = fmin(margin, armijo_margin(f, na.sigma * Dq, L1a + Cv * sLa));
      if (f <= na.sigma * Dq) {
        q_acc = q;
        dF = f;
        break;
      }
      Dq *= na.beta;
      al *= na.beta;
    }
    n_bundles += 1.0;
    n_nnz += (double)nb;
    n_slots += (double)ns;
    n_ls += q_acc >= 0 ? q_acc + 1 : na.max_ls;
    n_fail += q_acc < 0 ? 1.0 : 0.0;
    // 4. accept: w, retained quantities; clear the global d^T x
    if (na.dtx_copy) {
      if (R >= 0) {
        // the recorded rows' values over zeros
        for (int64_t i = tid; i < na.n; i += kNarrowBlock) na.dtx_copy[i] = 0.0;
        __syncthreads();
        for (int32_t e = tid; e < R; e += kNarrowBlock)
          if (L.t_acc[e] != 0ull) na.dtx_copy[L.t_row[e]] = fx_value(L.t_acc[e], isc);
      } else {
        for (int64_t i = tid; i < na.n; i += kNarrowBlock)
          na.dtx_copy[i] = fx_value(load_l2_fx(&a.dtx[i]), isc);
      }
      __syncthreads();  // copied before any thread clears d^T x below
    }
    if (listed) {
      if (q_acc >= 0) {
        for (int32_t e = tid; e < R; e += kNarrowBlock) {
          const unsigned long long ac = L.t_acc[e];
          if (ac == 0ull) continue;
          double sv = fx_value(ac, isc);
          for (int u = 0; u < q_acc; ++u) sv *= na.beta;
          const int32_t i = L.t_row[e];
          store_retained<LOSS>(&na.cache[i], &na.rw[i],
                               LOSS == kLogistic ? L.t_c[e] * exp(sv)
                                                 : L.t_c[e] - (L.t_y[e] > 0 ? sv : -sv),
                               (int)L.t_y[e], na.stats);
        }
      }
    } else {
      unsigned long long* gacc = (unsigned long long*)a.dtx;
      for (int64_t i0 = tid; i0 < na.n; i0 += (int64_t)kNarrowRegRounds * kNarrowBlock) {
        unsigned long long fa[kNarrowRegRounds];
        double fc[kNarrowRegRounds];
        int fy[kNarrowRegRounds];
#pragma unroll
        for (int u = 0; u < kNarrowRegRounds; ++u) {
          const int64_t i = i0 + (int64_t)u * kNarrowBlock;
          fa[u] = i < na.n ? load_l2_fx(&a.dtx[i]) : 0ull;
        }
#pragma unroll
        for (int u = 0; u < kNarrowRegRounds; ++u) {
          const int64_t i = i0 + (int64_t)u * kNarrowBlock;
          const bool upd = q_acc >= 0 && fa[u] != 0ull;
          fc[u] = upd ? na.cache[i] : 0.0;
          fy[u] = upd ? (int)a.y[i] : 0;
        }
#pragma unroll
        for (int u = 0; u < kNarrowRegRounds; ++u) {
          const int64_t i = i0 + (int64_t)u * kNarrowBlock;
          if (fa[u] == 0ull) continue;
          if (q_acc >= 0) {
            double sv = fx_value(fa[u], isc);
            for (int k = 0; k < q_acc; ++k) sv *= na.beta;
            store_retained<LOSS>(&na.cache[i], &na.rw[i],
                                 LOSS == kLogistic ? fc[u] * exp(sv)
                                                   : fc[u] - (fy[u] > 0 ? sv : -sv),
                                 fy[u], na.stats);
          }
          __hip_atomic_store(&gacc[i], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
      }
    }
    if (q_acc >= 0)
      for (int32_t s = tid; s < ns; s += kNarrowBlock) na.w[L.feat[s]] = L.w[s] + al * L.d[s];
    if (tid == 0 && t == t_end - 1) {
      na.st->q = q_acc;
      na.st->alpha = q_acc >= 0 ? al : 0.0;
      na.st->dF = dF;
      na.st->delta = Delta;
    }
    __syncthreads();
  }
  if (na.stats) {
    n_scat = block_sum16(n_scat, L.lds16);
    n_scat_long = block_sum16(n_scat_long, L.lds16);
  }
  if (tid == 0 && na.stats) {
    atomicAdd(&na.stats->nnz_gh_narrow, (unsigned long long)n_nnz);
    atomicAdd(&na.stats->slots_narrow, (unsigned long long)n_slots);
    atomicAdd(&na.stats->nnz_scat_narrow, (unsigned long long)n_scat);
    atomicAdd(&na.stats->nnz_scat_narrow_split, (unsigned long long)n_scat_long);
    atomicAdd(&na.stats->bundles, (unsigned long long)n_bundles);
    atomicAdd(&na.stats->ls_steps, (unsigned long long)n_ls);
    if (n_fail > 0.0) atomicAdd(&na.stats->ls_fail, (unsigned long long)n_fail);
    atomicAdd(&na.stats->rows_touched, (unsigned long long)n_touched);
    atomicAdd(&na.stats->rows_touched_narrow, (unsigned long long)n_touched);
    atomicMin(&na.stats->min_margin_bits, (unsigned long long)__double_as_longlong(margin));
  }
}

template <int LOSS>
__global__ __launch_bounds__(kNarrowBlock) void k_narrow(NarrowArgs na) {
  __shared__ NarrowLds L;
  narrow_body<LOSS>(na, L);
}

// Independent problems in one launch: workgroup b runs the bundles of
// problem tab[b] (its own data, state and loss).
__global__ __launch_bounds__(kNarrowBlock) void k_narrow_multi(const NarrowArgs* __restrict__ tab) {
  __shared__ NarrowLds L;
  // a private copy: the kernel stores to global memory, so fields read
  // through the table could otherwise be re-read after stores
  const NarrowArgs na = tab[blockIdx.x];
  if (na.loss == kLogistic)
    narrow_body<kLogistic>(na, L);
  else
    narrow_body<kL2Svm>(na, L);
}

// Copy X into partition order: the nonzeros of slot r land at
// [poff[r], poff[r+1]).  A wavefront takes kPermW consecutive output
// positions, lane L the positions 4L .. 4L+3.  The slots that cover them
// are read 64 at a time, from rfirst[range] on (their output offsets and the
// first nonzero of their columns, one slot per lane); a position finds its
// slot by a binary search over the 64 slots' ends (exchanged by lane
// shuffles), gathers its row index and value from the column, and stores
// them with its slot, so the stores are contiguous and every lane has
// nonzeros to move however short the columns are.
constexpr int kPermE = kPermW / kWave;

__device__ inline int64_t shfl64(int64_t x, int src) {
  const int lo = __shfl((int)(uint32_t)(uint64_t)x, src, kWave);
  const int hi = __shfl((int)(uint32_t)((uint64_t)x >> 32), src, kWave);
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo);
}

__device__ __forceinline__ void permute_body(const PermuteArgs& a, int64_t bid, int64_t nblk) {
  const int lane = lane_id();
  const int64_t wave = uniform((bid * kBlock + threadIdx.x) / kWave);
  const int64_t nwaves = nblk * kWavesPerBlock;
  const int64_t N = a.poff[a.p];
  const int64_t nr = (N + kPermW - 1) / kPermW;
  const bool vec = ((reinterpret_cast<uintptr_t>(a.pri) | reinterpret_cast<uintptr_t>(a.pv) |
                     reinterpret_cast<uintptr_t>(a.pslot)) & 15) == 0;
  for (int64_t m = wave; m < nr; m += nwaves) {
    const int64_t q0 = m * kPermW + (int64_t)lane * kPermE;
    int32_t slot[kPermE];
    int64_t src[kPermE];
    bool open[kPermE];
#pragma unroll
    for (int u = 0; u < kPermE; ++u) {
      slot[u] = 0;
      src[u] = 0;
      open[u] = q0 + u < N;
    }
    // windows of 64 slots; a window's slots past the order end nowhere
    // (INT64_MAX), so every position < N is found
    for (int64_t s = uniform(a.rfirst[m]);; s += kWave) {
      const int64_t sw = s + lane;
      const bool in = sw < a.p;
      const int64_t st = in ? a.poff[sw] : INT64_MAX;
      const int64_t en = in ? a.poff[sw + 1] : INT64_MAX;
      const int64_t cs = in ? a.src[sw] : 0;
      bool more = false;
#pragma unroll
      for (int u = 0; u < kPermE; ++u) {
        // i = the number of window slots that end at or before q: slot s + i
        // holds q (its start is <= q, its end > q) unless i == 64
        const int64_t q = q0 + u;
        // (the halving steps count the ends <= q among the first 63; the
        // last end is then tested at i, which is 63 only if all 63 were)
        int i = 0;
#pragma unroll
        for (int step = kWave / 2; step >= 1; step >>= 1)
          if (shfl64(en, i + step - 1) <= q) i += step;
        if (shfl64(en, i) <= q) i += 1;
        const int ic = i < kWave ? i : kWave - 1;
        const int64_t sti = shfl64(st, ic), csi = shfl64(cs, ic);
        if (open[u] && i < kWave) {
          slot[u] = (int32_t)(s + i);
          src[u] = csi + (q - sti);
          open[u] = false;
        }
        more = more || open[u];
      }
      if (__ballot(more) == 0) break;
    }
    int32_t row[kPermE];
    float val[kPermE];
#pragma unroll
    for (int u = 0; u < kPermE; ++u) {
      const bool ok = q0 + u < N;
      row[u] = ldz(a.ri, ok, src[u], 0);
      val[u] = ldz(a.v, ok, src[u], 0.0f);
    }
    if (vec && q0 + kPermE <= N) {
      *reinterpret_cast<int4*>(a.pri + q0) = make_int4(row[0], row[1], row[2], row[3]);
      *reinterpret_cast<float4*>(a.pv + q0) = make_float4(val[0], val[1], val[2], val[3]);
      if (a.pslot)
        *reinterpret_cast<int4*>(a.pslot + q0) = make_int4(slot[0], slot[1], slot[2], slot[3]);
    } else {
#pragma unroll
      for (int u = 0; u < kPermE; ++u) {
        if (q0 + u < N) {
          a.pri[q0 + u] = row[u];
          a.pv[q0 + u] = val[u];
          if (a.pslot) a.pslot[q0 + u] = slot[u];
        }
      }
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_permute(PermuteArgs a) {
  permute_body(a, blockIdx.x, gridDim.x);
}

// Column length of each slot, and w in slot order (pw[r] = w[perm[r]]).
__device__ __forceinline__ void slot_len_body(const SlotLenArgs& a, int64_t bid) {
  const int64_t r = bid * (int64_t)kBlock + threadIdx.x;
  if (r < a.p) {
    const int32_t j = a.perm[r];
    const int64_t k0 = a.cp[j];
    a.len[r] = (int32_t)(a.cp[j + 1] - k0);
    if (a.w) a.pw[r] = a.w[j];
    if (a.src) a.src[r] = k0;
    if (a.islot) a.islot[j] = (int32_t)r;
  }
}

__global__ __launch_bounds__(kBlock) void k_slot_len(SlotLenArgs a) { slot_len_body(a, blockIdx.x); }

__device__ __forceinline__ void widen_body(const WidenArgs& a, int64_t bid) {
  const int64_t r = bid * (int64_t)kBlock + threadIdx.x;
  if (r <= a.m) a.out[r] = a.in[r];
  if (a.rfirst && r < a.m) {  // the ranges whose first position slot r holds
    const int64_t lo = a.in[r], hi = a.in[r + 1];
    for (int64_t k = (lo + kPermW - 1) / kPermW; k * kPermW < hi; ++k) a.rfirst[k] = (int32_t)r;
  }
}

__global__ __launch_bounds__(kBlock) void k_widen(WidenArgs a) { widen_body(a, blockIdx.x); }

// ---------------------------------------------------------------------------
// deterministic sum (two kernels), loss terms, margins
// ---------------------------------------------------------------------------
__device__ __forceinline__ void sum_partial_body(const SumArgs& a, int64_t bid, int64_t nblk) {
  __shared__ double lds4[kWavesPerBlock];
  double s = 0.0;
  for (int64_t i = bid * kBlock + threadIdx.x; i < a.m; i += nblk * kBlock) s += a.x[i];
  s = block_sum(s, lds4);
  if (threadIdx.x == 0) a.part[bid] = s;
}

__device__ __forceinline__ void sum_final_body(const SumArgs& a) {
  __shared__ double lds4[kWavesPerBlock];
  double s = 0.0;
  for (int b = threadIdx.x; b < a.nb; b += kBlock) s += a.part[b];
  s = block_sum(s, lds4);
  if (threadIdx.x == 0) {
    *a.out = s;
    if (a.it) a.it->k += 1;
  }
}

__global__ __launch_bounds__(kBlock) void k_sum_partial(SumArgs a) {
  sum_partial_body(a, blockIdx.x, gridDim.x);
}

__global__ __launch_bounds__(kBlock) void k_sum_final(SumArgs a) { sum_final_body(a); }

// Shrinking's stopping reduction (see StopSumArgs): four values per block in
// a fixed order, then the final level in block order.
__device__ inline double block_max(double v, double* lds4) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
  if (lane_id() == 0) lds4[wave_in_block()] = v;
  __syncthreads();
  double r = lds4[0];
  for (int k = 1; k < kWavesPerBlock; ++k) r = fmax(r, lds4[k]);
  __syncthreads();
  return r;
}

__device__ __forceinline__ void stop_partial_body(const StopSumArgs& a, int64_t bid, int64_t nblk) {
  __shared__ double lds4[kWavesPerBlock];
  double sg = 0.0, mx = 0.0, na = 0.0, nz = 0.0;
  for (int64_t j = bid * kBlock + threadIdx.x; j < a.p; j += nblk * kBlock) {
    const double v = a.sg[j];
    sg += v;
    mx = fmax(mx, v);
    if (a.act[j] != 0.0) {
      na += 1.0;
      nz += (double)(a.cp[j + 1] - a.cp[j]);
    }
  }
  sg = block_sum(sg, lds4);
  mx = block_max(mx, lds4);
  na = block_sum(na, lds4);
  nz = block_sum(nz, lds4);
  if (threadIdx.x == 0) {
    a.part[4 * bid + 0] = sg;
    a.part[4 * bid + 1] = mx;
    a.part[4 * bid + 2] = na;
    a.part[4 * bid + 3] = nz;
  }
}

__device__ __forceinline__ void stop_final_body(const StopSumArgs& a) {
  __shared__ double lds4[kWavesPerBlock];
  double sg = 0.0, mx = 0.0, na = 0.0, nz = 0.0;
  for (int b = threadIdx.x; b < a.nb; b += kBlock) {
    sg += a.part[4 * b + 0];
    mx = fmax(mx, a.part[4 * b + 1]);
    na += a.part[4 * b + 2];
    nz += a.part[4 * b + 3];
  }
  sg = block_sum(sg, lds4);
  mx = block_max(mx, lds4);
  na = block_sum(na, lds4);
  nz = block_sum(nz, lds4);
  if (threadIdx.x == 0) {
    a.scal[0] = sg;
    a.scal[3] = mx;
    a.scal[4] = a.ra - mx / (double)a.n;
    a.scal[5] = na;
    a.scal[6] = nz;
    if (a.it) a.it->k += 1;
  }
}

__global__ __launch_bounds__(kBlock) void k_stop_partial(StopSumArgs a) {
  stop_partial_body(a, blockIdx.x, gridDim.x);
}

__global__ __launch_bounds__(kBlock) void k_stop_final(StopSumArgs a) { stop_final_body(a); }

// ---------------------------------------------------------------------------
// Multi-problem executor: one launch runs one task of each of several
// independent problems.  Block b finds its task i (first[i] <= b <
// first[i+1]) with ballots over the block-offset table and runs the task's
// kernel body on local block b - first[i] of nblk, i.e. with the work split
// of a launch of its own, so every problem gets the same results as alone.
// ---------------------------------------------------------------------------
__device__ inline int task_of_block(const int32_t* first, int count, int b) {
  int i = 0;
  for (int base = 0; base < count; base += kWave) {
    const int k = base + lane_id();
    i += __popcll(__ballot(k < count && first[k + 1] <= b));
  }
  return __builtin_amdgcn_readfirstlane(i);
}

template <int LOSS>
__device__ __forceinline__ void exec_task(const Task& t, int lb) {
  switch (t.kind) {
    case kTaskSweepRanges: sweep_ranges_any<LOSS>(t.u.sw, lb, t.nblk); break;
    case kTaskStopRanges: stop_ranges_body<LOSS>(t.u.so, lb, t.nblk); break;
    case kTaskSweepFinish: sweep_finish_body<LOSS>(t.u.sw, lb, t.nblk); break;
    case kTaskStopFinish: stop_finish_body<LOSS>(t.u.so, lb, t.nblk); break;
    case kTaskRowsDtx: rows_dtx_body<LOSS, false>(t.u.rw, lb); break;
    case kTaskRowsApply: rows_apply_body<LOSS, false>(t.u.rw, lb, t.nblk); break;
    case kTaskSlotLen: slot_len_body(t.u.sl, lb); break;
    case kTaskWiden: widen_body(t.u.wd, lb); break;
    case kTaskPermute: permute_body(t.u.pm, lb, t.nblk); break;
    case kTaskBrHist: br_hist_body(t.u.br, lb); break;
    case kTaskBrScatter: br_scatter_body(t.u.br, lb); break;
    case kTaskSumPartial: sum_partial_body(t.u.sum, lb, t.nblk); break;
    case kTaskSumFinal: sum_final_body(t.u.sum); break;
    case kTaskStopPartial: stop_partial_body(t.u.stop, lb, t.nblk); break;
    case kTaskStopFinal: stop_final_body(t.u.stop); break;
    case kTaskPermKeys:
      perm_keys_body(t.u.pk.it, t.u.pk.seed, t.u.pk.k, t.u.pk.p, t.u.pk.act, t.u.pk.keys,
                     t.u.pk.idx, lb);
      break;
    case kTaskRadixHist:
      radix_hist_body(t.u.rx.kin, t.u.rx.p, t.u.rx.shift, t.u.rx.hist, t.u.rx.ntiles, lb);
      break;
    case kTaskRadixScatter:
      radix_scatter_body(t.u.rx.kin, t.u.rx.iin, t.u.rx.kout, t.u.rx.iout, t.u.rx.p, t.u.rx.shift,
                         t.u.rx.hist, t.u.rx.ntiles, lb);
      break;
    case kTaskScanSmall: scan_small_body<kBlock>(t.u.scan.in, t.u.scan.out, t.u.scan.m); break;
    case kTaskScanBlocks:
      scan_blocks_body<kBlock>(t.u.scan.in, t.u.scan.out, t.u.scan.m, t.u.scan.tmp, lb);
      break;
    case kTaskScanAdd:
      scan_add_body<kBlock>(t.u.scan.out, t.u.scan.m, t.u.scan.tmp, t.u.scan.nb, lb);
      break;
    default: break;
  }
}

// The tables are not written by any task (__restrict__), so task fields
// read once can stay in registers across the bodies' stores.
__global__ __launch_bounds__(kBlock) void k_exec(const Task* __restrict__ tasks,
                                                 const int32_t* __restrict__ first, int count) {
  const int b = blockIdx.x;
  const int i = task_of_block(first, count, b);
  const Task& t = tasks[i];
  const int lb = b - first[i];
  if (t.loss == kLogistic)
    exec_task<kLogistic>(t, lb);
  else
    exec_task<kL2Svm>(t, lb);
}

template <int LOSS>
__global__ void k_loss_terms(const double* cache, const int8_t* y, int64_t n, double* out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) {
    const double c = cache[i];
    if (LOSS == kLogistic) {
      out[i] = y[i] > 0 ? log1p(1.0 / c) : log1p(c);  // log(1 + e^{-y z})
    } else {
      const double b = c > 0.0 ? c : 0.0;
      out[i] = b * b;
    }
  }
}

// Regulariser terms ra |w_j| + (rb/2) w_j^2 of F.
__global__ void k_reg_terms(const double* w, int64_t p, double ra, double rb, double* out) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j < p) out[j] = ra * fabs(w[j]) + 0.5 * rb * w[j] * w[j];
}

// Every row's term weights from its retained quantity and label.
template <int LOSS>
__global__ void k_row_weights(const double* cache, const int8_t* y, int64_t n, double2* rw) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) rw[i] = row_weights<LOSS>(cache[i], (int)y[i]);
}

// Retained quantities from w, one wavefront per row over X in CSR order: the
// margin z_i = sum_j x_ij w_j is summed lane-strided, then by the fixed-order
// wavefront sum, so it does not depend on scheduling; then e^{z_i} (logistic)
// or b_i = 1 - y_i z_i (SVM).
template <int LOSS>
__global__ __launch_bounds__(kBlock) void k_margins_rows(const int64_t* rp, const int32_t* col,
                                                         const float* v, const double* w,
                                                         const int8_t* y, int64_t n,
                                                         double* cache, Stats* stats) {
  const int lane = lane_id();
  const int64_t wave = uniform(((int64_t)blockIdx.x * kBlock + threadIdx.x) / kWave);
  const int64_t nwaves = (int64_t)gridDim.x * kWavesPerBlock;
  for (int64_t i = wave; i < n; i += nwaves) {
    double z = 0.0;
    for (int64_t k = rp[i] + lane; k < rp[i + 1]; k += kWave) z += (double)v[k] * w[col[k]];
    z = wave_sum(z);
    if (lane == 0) {
      const double c = LOSS == kLogistic ? exp(z) : 1.0 - (y[i] > 0 ? z : -z);
      cache[i] = c;
      count_range<LOSS>(c, stats);
    }
  }
}

template <int LOSS>
__global__ void k_cache_from_z(double* zc, const int8_t* y, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) {
    const double z = zc[i];
    zc[i] = LOSS == kLogistic ? exp(z) : 1.0 - (y[i] > 0 ? z : -z);
  }
}

inline int grid_for(int64_t items, int per_block, int cap) {
  int64_t g = (items + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

int permute_grid(int64_t nnz) { return grid_for((nnz + kPermW - 1) / kPermW, kWavesPerBlock, 8192); }

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_fill(double* a, double v, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_fill, dim3(grid_for(n, kBlock, 4096)), dim3(kBlock), 0, s, a, v, n);
  return hipGetLastError();
}

hipError_t launch_perm_keys(const IterState* it, uint64_t seed, int64_t k, int64_t p,
                            const double* act, uint32_t* keys, int32_t* idx, hipStream_t s) {
  hipLaunchKernelGGL(k_perm_keys, dim3(grid_for(p, kBlock, 1 << 30)), dim3(kBlock), 0, s, it,
                     seed, k, p, act, keys, idx);
  return hipGetLastError();
}

int64_t scan_tmp_ints(int64_t m) { return (m + kScanTile - 1) / kScanTile + 1; }
int64_t radix_hist_ints(int64_t p) { return 256 * ((p + kSortTile - 1) / kSortTile) + 1; }

hipError_t launch_scan(const int32_t* in, int32_t* out, int64_t m, int32_t* tmp, hipStream_t s) {
  if (m < 0) return hipErrorInvalidValue;
  if (m <= kScanSmall) {
    hipLaunchKernelGGL(k_scan_small, dim3(1), dim3(kScanThreads), 0, s, in, out, m);
    return hipGetLastError();
  }
  const int64_t nb = (m + kScanTile - 1) / kScanTile;
  hipLaunchKernelGGL(k_scan_blocks, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, out, m,
                     tmp);
  hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nb), dim3(kScanThreads), 0, s, out, m, tmp, nb);
  return hipGetLastError();
}

hipError_t launch_radix_sort(uint32_t* keys0, int32_t* idx0, uint32_t* keys1, int32_t* idx1,
                             int64_t p, int32_t* hist, int32_t* scan_tmp, hipStream_t s) {
  const int64_t ntiles = (p + kSortTile - 1) / kSortTile;
  const int64_t m = 256 * ntiles;
  uint32_t* kin = keys0;
  int32_t* iin = idx0;
  uint32_t* kout = keys1;
  int32_t* iout = idx1;
  for (int pass = 0; pass < 4; ++pass) {
    const int shift = 8 * pass;
    hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)ntiles), dim3(kSortThreads), 0, s, kin, p,
                       shift, hist, ntiles);
    hipError_t e = launch_scan(hist, hist, m, scan_tmp, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_radix_scatter_staged, dim3((unsigned)ntiles), dim3(kSortThreads), 0, s, kin,
                       iin, kout, iout, p, shift, hist, ntiles);
    uint32_t* tk = kin;
    kin = kout;
    kout = tk;
    int32_t* ti = iin;
    iin = iout;
    iout = ti;
  }
  // four passes: the sorted data is back in keys0 / idx0
  return hipGetLastError();
}

namespace {

Task partition_task(int kind, int loss, int64_t nblk) {
  Task t;
  std::memset(&t, 0, sizeof(t));
  t.kind = kind;
  t.loss = loss;
  t.nblk = (int32_t)nblk;
  return t;
}

// The tasks of launch_scan(in, out, m, tmp); kBlock-thread blocks, so the
// one-block scan takes m <= 16 kBlock.
void scan_tasks(int loss, const int32_t* in, int32_t* out, int64_t m, int32_t* tmp,
                std::vector<Task>& v) {
  Task t = partition_task(kTaskScanSmall, loss, 1);
  t.u.scan = ScanArgs{in, out, tmp, m, 0};
  if (m <= 16 * kBlock) {
    v.push_back(t);
    return;
  }
  const int64_t nb = (m + kScanTile - 1) / kScanTile;
  t.u.scan.nb = nb;
  t.kind = kTaskScanBlocks;
  t.nblk = (int32_t)nb;
  v.push_back(t);
  t.kind = kTaskScanAdd;
  t.nblk = (int32_t)nb;
  v.push_back(t);
}

}  // namespace

void partition_tasks(int loss, const IterState* it, uint64_t seed, int64_t p, const double* act,
                     uint32_t* keys0, int32_t* idx0, uint32_t* keys1, int32_t* idx1,
                     int32_t* hist, int32_t* scan_tmp, std::vector<Task>& out) {
  const int64_t pg = grid_for(p, kBlock, 1 << 30);
  Task t = partition_task(kTaskPermKeys, loss, pg);
  t.u.pk = PermKeysArgs{it, seed, 0, p, act, keys0, idx0};
  out.push_back(t);
  // launch_radix_sort's passes
  const int64_t ntiles = (p + kSortTile - 1) / kSortTile;
  uint32_t* kin = keys0;
  int32_t* iin = idx0;
  uint32_t* kout = keys1;
  int32_t* iout = idx1;
  for (int pass = 0; pass < 4; ++pass) {
    t = partition_task(kTaskRadixHist, loss, ntiles);
    t.u.rx = RadixArgs{kin, iin, kout, iout, hist, p, ntiles, 8 * pass};
    out.push_back(t);
    scan_tasks(loss, hist, hist, 256 * ntiles, scan_tmp, out);
    t.kind = kTaskRadixScatter;
    out.push_back(t);
    std::swap(kin, kout);
    std::swap(iin, iout);
  }
}

// One wavefront per range of a bundle of the expected size and at least 256
// wavefronts; a larger bundle (the partition is random) takes several ranges
// per wavefront.  Which wavefront takes a range changes no sum.
int sweep_ranges_grid(double nnz_bundle, int W) {
  const double ranges = nnz_bundle / W + 1.0;
  const int64_t waves = ranges > 256.0 ? (int64_t)ranges : 256;
  return grid_for(waves, kWavesPerBlock, 8192);
}

int sweep_finish_grid(int64_t slots) { return grid_for(slots, kBlock, 4096); }

template <int LOSS>
void launch_sweep_ranges_w(const SweepArgs& a, int grid, hipStream_t s) {
  switch (a.W) {
    case 64: hipLaunchKernelGGL((k_sweep_ranges<LOSS, 1>), dim3(grid), dim3(kBlock), 0, s, a); break;
    case 128: hipLaunchKernelGGL((k_sweep_ranges<LOSS, 2>), dim3(grid), dim3(kBlock), 0, s, a); break;
    case 512: hipLaunchKernelGGL((k_sweep_ranges<LOSS, 8>), dim3(grid), dim3(kBlock), 0, s, a); break;
    default: hipLaunchKernelGGL((k_sweep_ranges<LOSS, 4>), dim3(grid), dim3(kBlock), 0, s, a); break;
  }
}

hipError_t launch_sweep_ranges(int loss, const SweepArgs& a, int grid, hipStream_t s) {
  if (a.W != 64 && a.W != 128 && a.W != 256 && a.W != 512) return hipErrorInvalidValue;
  if (loss == kLogistic)
    launch_sweep_ranges_w<kLogistic>(a, grid, s);
  else
    launch_sweep_ranges_w<kL2Svm>(a, grid, s);
  return hipGetLastError();
}

hipError_t launch_sweep_finish(int loss, const SweepArgs& a, hipStream_t s) {
  const dim3 g(sweep_finish_grid(a.slot_hi - a.slot_lo));
  if (loss == kLogistic)
    hipLaunchKernelGGL(k_sweep_finish<kLogistic>, g, dim3(kBlock), 0, s, a);
  else
    hipLaunchKernelGGL(k_sweep_finish<kL2Svm>, g, dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

int stop_ranges_grid(int64_t nnz) {
  return grid_for((nnz + kStopW - 1) / kStopW, kWavesPerBlock, 8192);
}
int stop_finish_grid(int64_t p) { return grid_for(p, kBlock, 4096); }

hipError_t launch_stop_sweep(int loss, const StopArgs& a, hipStream_t s) {
  const dim3 g1(stop_ranges_grid(a.nnz)), g2(stop_finish_grid(a.p));
  const dim3 gt((unsigned)((a.nnz + kStopTile - 1) / kStopTile));
  const bool tiles = a.srow && a.spos && a.gwc && a.nnz > 0;
  if (tiles)
    hipLaunchKernelGGL(k_pack_gradient_weights, dim3(grid_for(a.n, kBlock, 4096)), dim3(kBlock), 0,
                       s, a.rw, a.n, a.gwc);
  if (loss == kLogistic) {
    if (a.nnz > 0 && tiles)
      hipLaunchKernelGGL(k_stop_tiles<kLogistic>, gt, dim3(kStopTileThreads), 0, s, a);
    else if (a.nnz > 0)
      hipLaunchKernelGGL(k_stop_ranges<kLogistic>, g1, dim3(kBlock), 0, s, a);
    hipLaunchKernelGGL(k_stop_finish<kLogistic>, g2, dim3(kBlock), 0, s, a);
  } else {
    if (a.nnz > 0 && tiles)
      hipLaunchKernelGGL(k_stop_tiles<kL2Svm>, gt, dim3(kStopTileThreads), 0, s, a);
    else if (a.nnz > 0)
      hipLaunchKernelGGL(k_stop_ranges<kL2Svm>, g1, dim3(kBlock), 0, s, a);
    hipLaunchKernelGGL(k_stop_finish<kL2Svm>, g2, dim3(kBlock), 0, s, a);
  }
  return hipGetLastError();
}

int sum_grid(int64_t m) { return grid_for(m, kBlock, kSumGrid); }

// One wavefront per range of an average bundle, at least 128 blocks: a
// bundle with more ranges than wavefronts takes several per wavefront.
int rows_grid(double nnz_bundle) {
  const double ranges = nnz_bundle / kRangeW;
  double g = ranges / kWavesPerBlock;
  if (g < 128) g = 128;
  if (g > kRowsGridMax) g = kRowsGridMax;
  return (int)g;
}

hipError_t launch_rows_dtx(int loss, const RowsArgs& a, hipStream_t s) {
  if (a.G < 1 || a.G > kRowsGridMax) return hipErrorInvalidValue;
  if (loss == kLogistic)
    hipLaunchKernelGGL(k_rows_dtx<kLogistic>, dim3(a.G), dim3(kBlock), 0, s, a);
  else
    hipLaunchKernelGGL(k_rows_dtx<kL2Svm>, dim3(a.G), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_rows_apply(int loss, const RowsArgs& a, hipStream_t s) {
  if (a.G < 1 || a.G > kRowsGridMax) return hipErrorInvalidValue;
  if (loss == kLogistic)
    hipLaunchKernelGGL(k_rows_apply<kLogistic>, dim3(a.G), dim3(kBlock), 0, s, a);
  else
    hipLaunchKernelGGL(k_rows_apply<kL2Svm>, dim3(a.G), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_rows_scatter(const RowsArgs& a, double* dense, hipStream_t s) {
  hipLaunchKernelGGL(k_rows_scatter, dim3(256), dim3(kBlock), 0, s, a, dense);
  return hipGetLastError();
}

// Passes of the bundle-row sort: enough 8-bit digits for bundles 0 .. nb
// (nb = the bundle of features outside the order).
int br_passes(int64_t p_slots, int64_t P) {
  const int64_t nb = (p_slots + P - 1) / P;
  int passes = 1;
  while (passes < 4 && (nb >> (8 * passes)) != 0) ++passes;
  return passes;
}

int64_t br_hist_ints(int64_t nnz) { return 256 * ((nnz + kBrTile - 1) / kBrTile) + 1; }

namespace {

// The launches of the bundle-row order, in order: (kernel kind, block count,
// arguments).  Shared by the direct launcher and the executor's task list.
struct BrStep {
  int kind;  // kTaskSlotLen, kTaskWiden, kTaskPermute, kTaskBrHist, kTaskBrScatter; -1: scan
  int64_t nblk;
  SlotLenArgs sl;
  WidenArgs wd;
  PermuteArgs pm;
  BrArgs br;
  const int32_t* scan_in;
  int32_t* scan_out;
  int64_t scan_m;
};

// Calls f(step) for each launch in order (no host allocation).
template <class F>
void br_steps(const BrPlan& bp, F&& f) {
  const int64_t p_slots = bp.p_slots, P = bp.P, nnz = bp.nnz;
  BrStep st{};
  const int64_t pg = grid_for(p_slots, kBlock, 1 << 30);
  st.kind = kTaskSlotLen;
  st.nblk = pg;
  st.sl = SlotLenArgs{bp.perm, bp.cp, p_slots, bp.len_tmp, bp.w, bp.pw, bp.psrc, bp.islot};
  f(st);
  st = BrStep{};
  st.kind = -1;
  st.scan_in = bp.len_tmp;
  st.scan_out = bp.off32;
  st.scan_m = p_slots;
  f(st);
  st = BrStep{};
  st.kind = kTaskWiden;
  st.nblk = grid_for(p_slots + 1, kBlock, 1 << 30);
  st.wd = WidenArgs{bp.off32, p_slots, bp.poff, bp.rfirst};
  f(st);
  if (nnz == 0) return;
  // X in partition order (the bundle sweep's input)
  st = BrStep{};
  st.kind = kTaskPermute;
  st.nblk = permute_grid(nnz);
  st.pm = PermuteArgs{bp.ri, bp.v, bp.psrc, bp.poff, bp.rfirst, p_slots, bp.pri, bp.pv, bp.pslot};
  f(st);
  const int passes = br_passes(p_slots, P);
  const int64_t ntiles = (nnz + kBrTile - 1) / kBrTile;
  const int32_t nb = (int32_t)((p_slots + P - 1) / P);
  // the last pass writes the br arrays
  const int32_t* srow = bp.rr;
  const int32_t* scol = bp.rc;
  const float* sval = bp.rv;
  for (int pass = 0; pass < passes; ++pass) {
    const bool to_br = ((passes - 1 - pass) % 2) == 0;
    int32_t* drow = to_br ? bp.br_row : bp.bt_row;
    int32_t* dslot = to_br ? bp.br_slot : bp.bt_slot;
    float* dval = to_br ? bp.br_val : bp.bt_val;
    BrArgs b{pass == 0 ? bp.islot : nullptr, srow, scol, sval, drow, dslot, dval, bp.hist,
             nullptr, nnz, ntiles, P, 8 * pass, nb};
    if (pass == 0) b.slot_out = to_br ? bp.bt_slot : bp.br_slot;  // the buffer pass 0 does not write
    st = BrStep{};
    st.kind = kTaskBrHist;
    st.nblk = ntiles;
    st.br = b;
    f(st);
    if (pass == 0) {  // the scatter reads the slots the histogram pass wrote
      b.islot = nullptr;
      b.scol = b.slot_out;
      b.slot_out = nullptr;
    }
    st = BrStep{};
    st.kind = -1;
    st.scan_in = bp.hist;
    st.scan_out = bp.hist;
    st.scan_m = 256 * ntiles;
    f(st);
    st = BrStep{};
    st.kind = kTaskBrScatter;
    st.nblk = ntiles;
    st.br = b;
    f(st);
    srow = drow;
    scol = dslot;
    sval = dval;
  }
}

}  // namespace

hipError_t launch_bundle_row_order(const BrPlan& bp, hipStream_t s) {
  if (bp.P < 1 || bp.p_slots < 1 || bp.p_slots > bp.p) return hipErrorInvalidValue;
  if (bp.p_slots < bp.p)  // features outside the order keep slot -1
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(bp.p, kBlock, 4096)), dim3(kBlock), 0, s,
                       bp.islot, -1, bp.p);
  hipError_t err = hipSuccess;
  br_steps(bp, [&](const BrStep& st) {
    if (err != hipSuccess) return;
    hipError_t e = hipSuccess;
    switch (st.kind) {
      case kTaskSlotLen:
        hipLaunchKernelGGL(k_slot_len, dim3((unsigned)st.nblk), dim3(kBlock), 0, s, st.sl);
        break;
      case kTaskWiden:
        hipLaunchKernelGGL(k_widen, dim3((unsigned)st.nblk), dim3(kBlock), 0, s, st.wd);
        break;
      case kTaskPermute:
        hipLaunchKernelGGL(k_permute, dim3((unsigned)st.nblk), dim3(kBlock), 0, s, st.pm);
        break;
      case kTaskBrHist:
        hipLaunchKernelGGL(k_br_hist, dim3((unsigned)st.nblk), dim3(kSortThreads), 0, s, st.br);
        break;
      case kTaskBrScatter:
        hipLaunchKernelGGL(k_br_scatter_staged, dim3((unsigned)st.nblk), dim3(kSortThreads), 0, s,
                           st.br);
        break;
      default:
        e = launch_scan(st.scan_in, st.scan_out, st.scan_m, bp.scan_tmp, s);
        break;
    }
    err = e;
  });
  if (err != hipSuccess) return err;
  return hipGetLastError();
}

void bundle_row_tasks(int loss, const BrPlan& bp, std::vector<Task>& out) {
  // every feature has a slot in an outer iteration's order (p_slots == p)
  br_steps(bp, [&](const BrStep& st) {
    if (st.kind < 0) {
      scan_tasks(loss, st.scan_in, st.scan_out, st.scan_m, bp.scan_tmp, out);
      return;
    }
    Task t = partition_task(st.kind, loss, st.nblk);
    switch (st.kind) {
      case kTaskSlotLen: t.u.sl = st.sl; break;
      case kTaskWiden: t.u.wd = st.wd; break;
      case kTaskPermute: t.u.pm = st.pm; break;
      default: t.u.br = st.br; break;
    }
    out.push_back(t);
  });
}

hipError_t launch_permute(const int32_t* perm, const int64_t* cp, int64_t p, int64_t nnz,
                          const int32_t* ri, const float* v, int64_t* psrc, int32_t* rfirst,
                          int32_t* len_tmp, int32_t* off32, int32_t* scan_tmp, int64_t* poff,
                          int32_t* pri, float* pv, int32_t* pslot, const double* w, double* pw,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_slot_len, dim3(grid_for(p, kBlock, 1 << 30)), dim3(kBlock), 0, s,
                     SlotLenArgs{perm, cp, p, len_tmp, w, pw, psrc});
  hipError_t e = launch_scan(len_tmp, off32, p, scan_tmp, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_widen, dim3(grid_for(p + 1, kBlock, 1 << 30)), dim3(kBlock), 0, s,
                     WidenArgs{off32, p, poff, rfirst});
  if (nnz > 0)
    hipLaunchKernelGGL(k_permute, dim3(permute_grid(nnz)), dim3(kBlock), 0, s,
                       PermuteArgs{ri, v, psrc, poff, rfirst, p, pri, pv, pslot});
  return hipGetLastError();
}

hipError_t launch_bundle_rows(const int64_t* poff, const int32_t* pri, int64_t p_slots, int64_t P,
                              int64_t n, uint16_t* plid, int32_t* pR, hipStream_t s) {
  const int64_t words = (n + 31) >> 5;
  if (words > kRowsMaxWords || P < 1 || p_slots < 1) return hipErrorInvalidValue;
  const int64_t nbundles = (p_slots + P - 1) / P;
  hipLaunchKernelGGL(k_bundle_rows, dim3((unsigned)nbundles), dim3(kRowsBlock),
                     (size_t)(2 * words * sizeof(uint32_t)), s, poff, pri, p_slots, P, n, plid, pR);
  return hipGetLastError();
}

// Heavy-bundle list: one workgroup walks the bundles 1024 at a time; ballots
// and per-wave counts give each heavy bundle its position, so the list is in
// ascending order.
__global__ __launch_bounds__(1024) void k_heavy_bundles(const int64_t* poff, int64_t p_slots,
                                                        int64_t P, int64_t thresh, int32_t cap,
                                                        int32_t* out) {
  __shared__ int32_t wcnt[1024 / kWave];
  __shared__ int32_t total;
  if (threadIdx.x == 0) total = 0;
  __syncthreads();
  const int lane = lane_id(), wv = threadIdx.x / kWave;
  const int64_t nb = (p_slots + P - 1) / P;
  for (int64_t t0 = 0; t0 < nb; t0 += 1024) {
    const int64_t t = t0 + threadIdx.x;
    bool heavy = false;
    if (t < nb) {
      const int64_t lo = t * P, hi = lo + P < p_slots ? lo + P : p_slots;
      heavy = poff[hi] - poff[lo] >= thresh;
    }
    const uint64_t m = __ballot(heavy);
    if (lane == 0) wcnt[wv] = __popcll(m);
    __syncthreads();
    int32_t pos = total;
    for (int k = 0; k < wv; ++k) pos += wcnt[k];
    pos += __popcll(m & ((1ull << lane) - 1ull));
    if (heavy && pos < cap) out[1 + pos] = (int32_t)t;
    __syncthreads();
    if (threadIdx.x == 0) {
      int32_t sum = 0;
      for (int k = 0; k < 1024 / kWave; ++k) sum += wcnt[k];
      total += sum;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = total < cap ? total : cap;
}

hipError_t launch_heavy_bundles(const int64_t* poff, int64_t p_slots, int64_t P, int64_t thresh,
                                int32_t cap, int32_t* out, hipStream_t s) {
  if (P < 1 || p_slots < 1 || cap < 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_heavy_bundles, dim3(1), dim3(1024), 0, s, poff, p_slots, P, thresh, cap,
                     out);
  return hipGetLastError();
}

hipError_t launch_narrow(int loss, const NarrowArgs& a, hipStream_t s) {
  if (loss == kLogistic)
    hipLaunchKernelGGL(k_narrow<kLogistic>, dim3(1), dim3(kNarrowBlock), 0, s, a);
  else
    hipLaunchKernelGGL(k_narrow<kL2Svm>, dim3(1), dim3(kNarrowBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_exec(const Task* tasks, const int32_t* first, int count, int blocks,
                       hipStream_t s) {
  if (count <= 0 || blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_exec, dim3(blocks), dim3(kBlock), 0, s, tasks, first, count);
  return hipGetLastError();
}

__global__ void k_gather(const double* const* src, double* dst, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) dst[i] = *src[i];
}

hipError_t launch_gather(const double* const* src, double* dst, int count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather, dim3((count + kBlock - 1) / kBlock), dim3(kBlock), 0, s, src, dst,
                     count);
  return hipGetLastError();
}

hipError_t launch_narrow_multi(const NarrowArgs* tab, int count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_narrow_multi, dim3(count), dim3(kNarrowBlock), 0, s, tab);
  return hipGetLastError();
}

hipError_t launch_sum(const double* x, int64_t m, double* part, double* out, IterState* it,
                      hipStream_t s) {
  const int nb = sum_grid(m);
  const SumArgs a{x, m, part, out, it, nb};
  hipLaunchKernelGGL(k_sum_partial, dim3(nb), dim3(kBlock), 0, s, a);
  hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_stop_sum(const StopSumArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_stop_partial, dim3(a.nb), dim3(kBlock), 0, s, a);
  hipLaunchKernelGGL(k_stop_final, dim3(1), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_loss_terms(int loss, const double* cache, const int8_t* y, int64_t n,
                             double* out, hipStream_t s) {
  const dim3 g(grid_for(n, kBlock, 1 << 30));
  if (loss == kLogistic)
    hipLaunchKernelGGL(k_loss_terms<kLogistic>, g, dim3(kBlock), 0, s, cache, y, n, out);
  else
    hipLaunchKernelGGL(k_loss_terms<kL2Svm>, g, dim3(kBlock), 0, s, cache, y, n, out);
  return hipGetLastError();
}

hipError_t launch_reg_terms(const double* w, int64_t p, double ra, double rb, double* out,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_reg_terms, dim3(grid_for(p, kBlock, 1 << 30)), dim3(kBlock), 0, s, w, p,
                     ra, rb, out);
  return hipGetLastError();
}

hipError_t launch_margins_rows(int loss, const int64_t* rp, const int32_t* col, const float* v,
                               const double* w, const int8_t* y, int64_t n, double* cache,
                               Stats* stats, hipStream_t s) {
  const dim3 g(grid_for(n, kWavesPerBlock, 8192));
  if (loss == kLogistic)
    hipLaunchKernelGGL(k_margins_rows<kLogistic>, g, dim3(kBlock), 0, s, rp, col, v, w, y, n,
                       cache, stats);
  else
    hipLaunchKernelGGL(k_margins_rows<kL2Svm>, g, dim3(kBlock), 0, s, rp, col, v, w, y, n,
                       cache, stats);
  return hipGetLastError();
}

hipError_t launch_row_weights(int loss, const double* cache, const int8_t* y, int64_t n,
                              double2* rw, hipStream_t s) {
  const dim3 g(grid_for(n, kBlock, 1 << 30));
  if (loss == kLogistic)
    hipLaunchKernelGGL(k_row_weights<kLogistic>, g, dim3(kBlock), 0, s, cache, y, n, rw);
  else
    hipLaunchKernelGGL(k_row_weights<kL2Svm>, g, dim3(kBlock), 0, s, cache, y, n, rw);
  return hipGetLastError();
}

hipError_t launch_cache_from_z(int loss, double* z_to_cache, const int8_t* y, int64_t n,
                               hipStream_t s) {
  const dim3 g(grid_for(n, kBlock, 1 << 30));
  if (loss == kLogistic)
    hipLaunchKernelGGL(k_cache_from_z<kLogistic>, g, dim3(kBlock), 0, s, z_to_cache, y, n);
  else
    hipLaunchKernelGGL(k_cache_from_z<kL2Svm>, g, dim3(kBlock), 0, s, z_to_cache, y, n);
  return hipGetLastError();
}

}  // namespace pcdn
