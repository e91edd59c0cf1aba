// HIP kernels of the PCDN bundle sweep for gfx950 (CDNA4, 64-wide wavefronts).
//
// The work is sparse gather/scatter at well under one flop per byte, so it is
// bound by memory bandwidth and latency, not by the matrix cores: no MFMA here.
// Every reduction that decides anything (g_j, h_j, the line-search sums, the
// stopping norm) is FP64 and deterministic for a fixed launch shape; the only
// atomics are the FP64 adds that build d^T x_i, whose order can differ in the
// last bit between runs.
#include "pcdn_device.h"

namespace pcdn {

namespace {

// ---------------------------------------------------------------------------
// wavefront / block reductions
// ---------------------------------------------------------------------------
__device__ inline double wave_sum(double v) {
  // xor butterfly: every lane ends with the same bits (a + b == b + a)
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, kWave);
  return v;
}

__device__ inline int lane_id() { return threadIdx.x & (kWave - 1); }
__device__ inline int wave_in_block() { return threadIdx.x / kWave; }

// Sum over a 256-thread block; result valid in thread 0.  Fixed order.
__device__ inline double block_sum(double v, double* lds4) {
  v = wave_sum(v);
  if (lane_id() == 0) lds4[wave_in_block()] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) r = ((lds4[0] + lds4[1]) + lds4[2]) + lds4[3];
  __syncthreads();
  return r;
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
// Gradient / Hessian-diagonal contribution of one nonzero x of sample i with
// retained quantity c_i.  Logistic: with sigma(z) = 1/(1+e^{-z}) and E = e^z,
// s1 = sigma(z) = 1/(1+1/E) and s0 = 1 - sigma(z) = 1/(1+E) (both exact at
// E = 0 and E = inf).  For label y the misclassification weight is
// 1 - tau(y z) = (y > 0 ? s0 : s1) and tau(1 - tau) = s0 s1.
template <int LOSS>
__device__ inline void grad_hess_term(double c, int yi, double x, double& gs, double& hs) {
  if (LOSS == kLogistic) {
    const double s0 = 1.0 / (1.0 + c);
    const double s1 = 1.0 / (1.0 + 1.0 / c);
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

// log(A + B e^t) for A, B >= 0, A + B = 1, t <= 0.
__device__ inline double log_blend(double A, double B, double t) {
  const double u = B * expm1(t);
  return u >= -0.5 ? log1p(u) : log(A + B * exp(t));
}

// Loss change of sample i when its margin w^T x_i grows by a (eq. (10)'s
// summand).  Logistic: log(1+e^{-y(z+a)}) - log(1+e^{-yz}); writing
// m = -y a and tau = tau(y z) it is log(tau + (1 - tau) e^m), evaluated as
// m + log((1 - tau) + tau e^{-m}) when m > 0 so no exponential overflows.
// SVM: max(0, b - y a)^2 - max(0, b)^2.
template <int LOSS>
__device__ inline double loss_delta(double c, int yi, double a) {
  if (LOSS == kLogistic) {
    const double s0 = 1.0 / (1.0 + c);
    const double s1 = 1.0 / (1.0 + 1.0 / c);
    const double tau = yi > 0 ? s1 : s0;
    const double one_minus_tau = yi > 0 ? s0 : s1;
    const double m = yi > 0 ? -a : a;
    if (m <= 0.0) return log_blend(tau, one_minus_tau, m);
    return m + log_blend(one_minus_tau, tau, -m);
  } else {
    const double bn = yi > 0 ? c - a : c + a;
    const double pn = bn > 0.0 ? bn : 0.0;
    const double po = c > 0.0 ? c : 0.0;
    return pn * pn - po * po;
  }
}

// Minimiser of g d + h d^2/2 + |w + d| (eqs. (4)-(5), soft-threshold form).
__device__ inline double newton_dir(double g, double h, double w) {
  const double hw = h * w;
  if (g + 1.0 <= hw) return -(g + 1.0) / h;
  if (g - 1.0 >= hw) return -(g - 1.0) / h;
  return -w;
}

// Minimum-norm subgradient of F in coordinate j.
__device__ inline double min_norm_subgradient(double g, double w) {
  if (w > 0.0) return g + 1.0;
  if (w < 0.0) return g - 1.0;
  if (g > 1.0) return g - 1.0;
  if (g < -1.0) return g + 1.0;
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

__global__ void k_perm_keys(uint64_t stream_seed, int64_t p, uint32_t* keys, int32_t* idx) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j < p) {
    const uint64_t state = stream_seed + (uint64_t)(j + 1) * 0x9E3779B97F4A7C15ull;
    keys[j] = (uint32_t)(splitmix_out(state) >> 32);
    idx[j] = (int32_t)j;
  }
}

// ---------------------------------------------------------------------------
// exclusive scan (int32), three launches: per-block scan, scan of block
// totals, add-back.  A block covers kScanTile items.
// ---------------------------------------------------------------------------
constexpr int kScanThreads = 1024;
constexpr int kScanPer = 4;
constexpr int kScanTile = kScanThreads * kScanPer;

// Exclusive scan of one value per thread across a 1024-thread block.
__device__ inline int32_t block_exclusive_scan(int32_t v, int32_t* lds16, int32_t* total) {
  const int lane = lane_id(), wv = wave_in_block();
  int32_t x = v;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int32_t y = __shfl_up(x, o, kWave);
    if (lane >= o) x += y;
  }
  if (lane == kWave - 1) lds16[wv] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t run = 0;
    for (int k = 0; k < kScanThreads / kWave; ++k) {
      const int32_t t = lds16[k];
      lds16[k] = run;
      run += t;
    }
    lds16[kScanThreads / kWave] = run;
  }
  __syncthreads();
  const int32_t r = lds16[wv] + x - v;
  *total = lds16[kScanThreads / kWave];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_blocks(const int32_t* in, int32_t* out,
                                                              int64_t m, int32_t* block_tot) {
  __shared__ int32_t lds[kScanThreads / kWave + 1];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPer;
  int32_t v[kScanPer];
  int32_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    v[k] = base + k < m ? in[base + k] : 0;
    s += v[k];
  }
  int32_t tot;
  int32_t run = block_exclusive_scan(s, lds, &tot);
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    if (base + k < m) out[base + k] = run;
    run += v[k];
  }
  if (threadIdx.x == 0) block_tot[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_totals(int32_t* block_tot, int64_t nb,
                                                              int32_t* out_total) {
  __shared__ int32_t lds[kScanThreads / kWave + 1];
  const int64_t per = (nb + kScanThreads - 1) / kScanThreads;
  const int64_t lo = (int64_t)threadIdx.x * per;
  const int64_t hi = lo + per < nb ? lo + per : nb;
  int32_t s = 0;
  for (int64_t k = lo; k < hi; ++k) s += block_tot[k];
  int32_t tot;
  int32_t run = block_exclusive_scan(s, lds, &tot);
  for (int64_t k = lo; k < hi; ++k) {
    const int32_t t = block_tot[k];
    block_tot[k] = run;
    run += t;
  }
  if (threadIdx.x == 0) *out_total = tot;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_add(int32_t* out, int64_t m,
                                                           const int32_t* block_tot) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPer;
  const int32_t add = block_tot[blockIdx.x];
#pragma unroll
  for (int k = 0; k < kScanPer; ++k)
    if (base + k < m) out[base + k] += add;
}

// ---------------------------------------------------------------------------
// stable LSD radix sort of 32-bit keys with int32 payload, 8-bit digits.
// A tile is 4096 keys (256 threads x 16 rounds).  Stability inside a round
// comes from wavefront peer masks built with ballots, across waves and rounds
// from per-digit running offsets in LDS.
// ---------------------------------------------------------------------------
constexpr int kSortThreads = 256;
constexpr int kSortRounds = 16;
constexpr int kSortTile = kSortThreads * kSortRounds;

__global__ __launch_bounds__(kSortThreads) void k_radix_hist(const uint32_t* keys, int64_t p,
                                                             int shift, int32_t* hist,
                                                             int64_t ntiles) {
  __shared__ int32_t cnt[256];
  cnt[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  for (int r = 0; r < kSortRounds; ++r) {
    const int64_t i = base + r * kSortThreads + threadIdx.x;
    if (i < p) atomicAdd(&cnt[(keys[i] >> shift) & 255u], 1);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * ntiles + blockIdx.x] = cnt[threadIdx.x];
}

__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(
    const uint32_t* kin, const int32_t* iin, uint32_t* kout, int32_t* iout, int64_t p, int shift,
    const int32_t* offs, int64_t ntiles) {
  __shared__ int32_t base_off[256];
  __shared__ int32_t wcnt[kWavesPerBlock][256];
  base_off[threadIdx.x] = offs[(int64_t)threadIdx.x * ntiles + blockIdx.x];
  const int lane = lane_id(), wv = wave_in_block();
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int64_t tile = (int64_t)blockIdx.x * kSortTile;
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

// ---------------------------------------------------------------------------
// chunk bookkeeping
// ---------------------------------------------------------------------------
__global__ void k_chunk_count(const int32_t* perm, const int64_t* cp, int64_t p, int32_t* nch) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r < p) {
    const int32_t j = perm ? perm[r] : (int32_t)r;
    const int64_t len = cp[j + 1] - cp[j];
    const int64_t c = (len + kChunk - 1) / kChunk;
    nch[r] = (int32_t)(c > 0 ? c : 1);
  }
}

__global__ void k_chunk_fill(const int32_t* cstart, int64_t p, int32_t* chunk_slot) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r < p)
    for (int32_t c = cstart[r]; c < cstart[r + 1]; ++c) chunk_slot[c] = (int32_t)r;
}

// ---------------------------------------------------------------------------
// gradient / Hessian sweep over a bundle's columns (one wavefront per chunk).
// Bundle mode: per-feature g, h, direction d and the Delta term; a feature
// whose column fits one chunk also scatters d_j x^j into d^T x right away
// (the second read of x^j comes from L2).  Split columns leave partial sums;
// the last wavefront to finish a feature combines them in chunk order.
// Stopping mode: |grad^S_j F| per feature, no direction, no scatter.
// ---------------------------------------------------------------------------
constexpr int kUnroll = 4;

template <int LOSS>
__device__ inline void sweep_chunk(const SweepArgs& a, int64_t klo, int64_t khi, int lane,
                                   double& gs, double& hs) {
  for (int64_t k = klo + lane; k < khi; k += (int64_t)kWave * kUnroll) {
    int32_t row[kUnroll];
    float xv[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int64_t kk = k + (int64_t)u * kWave;
      const bool ok = kk < khi;
      row[u] = ok ? a.ri[kk] : -1;
      xv[u] = ok ? a.v[kk] : 0.0f;
    }
    double cv[kUnroll];
    int yv[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      cv[u] = row[u] >= 0 ? a.cache[row[u]] : 0.0;
      yv[u] = row[u] >= 0 ? (int)a.y[row[u]] : 0;
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u)
      if (row[u] >= 0) grad_hess_term<LOSS>(cv[u], yv[u], (double)xv[u], gs, hs);
  }
}

__device__ inline void scatter_chunk(const SweepArgs& a, int64_t klo, int64_t khi, int lane,
                                     double dj) {
  for (int64_t k = klo + lane; k < khi; k += kWave) {
    const int32_t row = a.ri[k];
    unsafeAtomicAdd(&a.dtx[row], dj * (double)a.v[k]);
  }
}

template <int LOSS, bool STOP>
__global__ __launch_bounds__(kBlock) void k_sweep(SweepArgs a) {
  const int lane = lane_id();
  const int64_t wave = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
  const int64_t nwaves = (int64_t)gridDim.x * kWavesPerBlock;
  const int32_t c_lo = a.cstart[a.slot_lo];
  const int32_t c_hi = a.cstart[a.slot_hi];
  unsigned long long nnz_local = 0, nnz_scat = 0;
  for (int64_t c = c_lo + wave; c < c_hi; c += nwaves) {
    const int32_t r = a.chunk_slot[c];
    const int32_t j = a.perm ? a.perm[r] : r;
    const int64_t k0 = a.cp[j], k1 = a.cp[j + 1];
    const int32_t c0 = a.cstart[r];
    const int32_t nch = a.cstart[r + 1] - c0;
    const int64_t klo = k0 + (int64_t)(c - c0) * kChunk;
    const int64_t khi = klo + kChunk < k1 ? klo + kChunk : k1;
    double gs = 0.0, hs = 0.0;
    sweep_chunk<LOSS>(a, klo, khi, lane, gs, hs);
    gs = wave_sum(gs);
    hs = wave_sum(hs);
    nnz_local += (unsigned long long)(khi - klo);
    if (nch > 1) {
      if (lane == 0) a.part[c] = make_double2(gs, hs);
      __threadfence();
      unsigned ticket = 0;
      if (lane == 0) ticket = atomicAdd(&a.cnt[r], 1u);
      ticket = __shfl(ticket, 0, kWave);
      if (ticket != (unsigned)(nch - 1)) continue;
      __threadfence();
      gs = 0.0;
      hs = 0.0;
      for (int32_t q = lane; q < nch; q += kWave) {
        const double2 pq = a.part[c0 + q];
        gs += pq.x;
        hs += pq.y;
      }
      gs = wave_sum(gs);
      hs = wave_sum(hs);
      if (lane == 0) a.cnt[r] = 0u;
    }
    double g, h;
    if (LOSS == kLogistic) {
      g = a.C * gs;
      h = a.C * hs;
    } else {
      g = -2.0 * a.C * gs;
      h = 2.0 * a.C * hs;
    }
    if (h <= 0.0) h += a.nu;
    const double wj = a.w ? a.w[j] : 0.0;
    const int64_t o = r - a.slot_lo;
    if (STOP) {
      if (lane == 0) a.sg[o] = fabs(min_norm_subgradient(g, wj));
    } else {
      const double dj = newton_dir(g, h, wj);
      if (lane == 0) {
        a.g[o] = g;
        a.h[o] = h;
        a.d[o] = dj;
        a.dterm[o] = g * dj + a.gamma * h * dj * dj + (fabs(wj + dj) - fabs(wj));
      }
      if (nch == 1 && dj != 0.0) {
        scatter_chunk(a, klo, khi, lane, dj);
        nnz_scat += (unsigned long long)(khi - klo);
      }
    }
  }
  if (STOP && a.stats && blockIdx.x == 0 && threadIdx.x == 0)
    atomicAdd(&a.stats->stop_sweeps, 1ull);
  if (lane == 0 && a.stats) {
    if (STOP) {
      atomicAdd(&a.stats->nnz_stop, nnz_local);
    } else {
      atomicAdd(&a.stats->nnz_gh, nnz_local);
      if (nnz_scat) atomicAdd(&a.stats->nnz_scat_fused, nnz_scat);
    }
  }
}

// d^T x scatter for columns split over several chunks (their direction is only
// known once every chunk has been summed).
__global__ __launch_bounds__(kBlock) void k_scatter_split(SweepArgs a) {
  const int lane = lane_id();
  const int64_t wave = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
  const int64_t nwaves = (int64_t)gridDim.x * kWavesPerBlock;
  const int32_t c_lo = a.cstart[a.slot_lo];
  const int32_t c_hi = a.cstart[a.slot_hi];
  unsigned long long nnz_scat = 0;
  for (int64_t c = c_lo + wave; c < c_hi; c += nwaves) {
    const int32_t r = a.chunk_slot[c];
    const int32_t c0 = a.cstart[r];
    const int32_t nch = a.cstart[r + 1] - c0;
    if (nch == 1) continue;
    const double dj = a.d[r - a.slot_lo];
    if (dj == 0.0) continue;
    const int32_t j = a.perm ? a.perm[r] : r;
    const int64_t k0 = a.cp[j], k1 = a.cp[j + 1];
    const int64_t klo = k0 + (int64_t)(c - c0) * kChunk;
    const int64_t khi = klo + kChunk < k1 ? klo + kChunk : k1;
    scatter_chunk(a, klo, khi, lane, dj);
    nnz_scat += (unsigned long long)(khi - klo);
  }
  if (lane == 0 && nnz_scat && a.stats) atomicAdd(&a.stats->nnz_scat_split, nnz_scat);
}

// ---------------------------------------------------------------------------
// P-dimensional line search (Algorithm 4 with eq. (10)): every candidate
// q0 .. q0+Q-1 in one pass over the samples.  The per-sample argument is
// d^T x_i scaled by beta once per rejected candidate, as Algorithm 4 scales
// its retained d^T x_i.  The last block to finish reduces the block partials
// in block order and applies the Armijo test in increasing q.
// ---------------------------------------------------------------------------
template <int LOSS>
__global__ __launch_bounds__(kBlock) void k_linesearch(LsArgs a) {
  __shared__ double red[kWavesPerBlock][kQMax];
  __shared__ double lds4[kWavesPerBlock];
  __shared__ bool is_last;
  const int lane = lane_id(), wv = wave_in_block();
  const int stride_blk = 2 * kQMax + 1;
  double acc[kQMax];
#pragma unroll
  for (int q = 0; q < kQMax; ++q) acc[q] = 0.0;
  unsigned long long touched = 0;
  for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < a.n;
       i += (int64_t)gridDim.x * kBlock) {
    const double dl = a.dtx[i];
    if (dl == 0.0) continue;
    ++touched;
    const double c = a.cache[i];
    const int yi = a.y[i];
    double s = dl;
    for (int t = 0; t < a.q0; ++t) s *= a.beta;
#pragma unroll
    for (int q = 0; q < kQMax; ++q) {
      if (q < a.Q) {
        acc[q] += loss_delta<LOSS>(c, yi, s);
        s *= a.beta;
      }
    }
  }
  // block partials of the loss sums
#pragma unroll
  for (int q = 0; q < kQMax; ++q) {
    const double v = wave_sum(acc[q]);
    if (lane == 0) red[wv][q] = v;
  }
  __syncthreads();
  double* mine = a.part + (int64_t)blockIdx.x * stride_blk;
  if (threadIdx.x < kQMax)
    mine[threadIdx.x] = ((red[0][threadIdx.x] + red[1][threadIdx.x]) + red[2][threadIdx.x]) +
                        red[3][threadIdx.x];
  __syncthreads();
  // l1 change of the bundle coordinates per candidate, and Delta
  double del = 0.0;
#pragma unroll
  for (int q = 0; q < kQMax; ++q) acc[q] = 0.0;
  const int64_t Pt = a.slot_hi - a.slot_lo;
  for (int64_t r = blockIdx.x * (int64_t)kBlock + threadIdx.x; r < Pt;
       r += (int64_t)gridDim.x * kBlock) {
    const double wj = a.w[a.perm[a.slot_lo + r]];
    const double dj = a.d[r];
    del += a.dterm[r];
    double al = 1.0;
    for (int t = 0; t < a.q0; ++t) al *= a.beta;
#pragma unroll
    for (int q = 0; q < kQMax; ++q) {
      if (q < a.Q) {
        acc[q] += fabs(wj + al * dj) - fabs(wj);
        al *= a.beta;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < kQMax; ++q) {
    const double v = wave_sum(acc[q]);
    if (lane == 0) red[wv][q] = v;
  }
  __syncthreads();
  if (threadIdx.x < kQMax)
    mine[kQMax + threadIdx.x] = ((red[0][threadIdx.x] + red[1][threadIdx.x]) +
                                 red[2][threadIdx.x]) + red[3][threadIdx.x];
  const double dsum = block_sum(del, lds4);
  if (threadIdx.x == 0) mine[2 * kQMax] = dsum;
  double tsum = block_sum((double)touched, lds4);
  if (threadIdx.x == 0 && tsum > 0.0)
    atomicAdd(&a.stats->rows_touched, (unsigned long long)tsum);
  // last block decides
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) is_last = atomicAdd(a.counter, 1u) == gridDim.x - 1;
  __syncthreads();
  if (!is_last) return;
  __threadfence();
  __shared__ double tot[2 * kQMax + 1];
  if (threadIdx.x < 2 * kQMax + 1) {
    double s = 0.0;
    for (int b = 0; b < (int)gridDim.x; ++b) s += a.part[(int64_t)b * stride_blk + threadIdx.x];
    tot[threadIdx.x] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double Delta = tot[2 * kQMax];
    double Dq = Delta, al = 1.0;
    for (int t = 0; t < a.q0; ++t) {
      Dq *= a.beta;
      al *= a.beta;
    }
    int accepted = -1;
    double dF = 0.0;
    for (int q = 0; q < a.Q; ++q) {
      const double f = tot[kQMax + q] + a.C * tot[q];
      if (f <= a.sigma * Dq) {
        accepted = a.q0 + q;
        dF = f;
        break;
      }
      Dq *= a.beta;
      al *= a.beta;
    }
    a.st->q = accepted;
    a.st->alpha = accepted >= 0 ? al : 0.0;
    a.st->dF = dF;
    a.st->delta = Delta;
    atomicAdd(&a.stats->bundles, 1ull);
    atomicAdd(&a.stats->ls_steps,
              (unsigned long long)(accepted >= 0 ? accepted + 1 : a.max_ls));
    if (accepted < 0) atomicAdd(&a.stats->ls_fail, 1ull);
    atomicAdd(&a.stats->slots, (unsigned long long)Pt);
    *a.counter = 0u;
  }
}

// ---------------------------------------------------------------------------
// accept: w_B += alpha d_B, retained quantities updated on the rows the bundle
// touches (e^{w^T x} multiplicatively, Algorithm 4; b_i -= y_i alpha d^T x_i),
// and d^T x cleared for the next inner iteration.
// ---------------------------------------------------------------------------
template <int LOSS>
__global__ __launch_bounds__(kBlock) void k_apply(ApplyArgs a) {
  const int q = a.st->q;
  const int64_t tid = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  const int64_t nthr = (int64_t)gridDim.x * kBlock;
  for (int64_t i = tid; i < a.n; i += nthr) {
    const double dl = a.dtx[i];
    if (dl == 0.0) continue;
    if (q >= 0) {
      double s = dl;
      for (int t = 0; t < q; ++t) s *= a.beta;
      if (LOSS == kLogistic)
        a.cache[i] *= exp(s);
      else
        a.cache[i] -= a.y[i] > 0 ? s : -s;
    }
    a.dtx[i] = 0.0;
  }
  if (q >= 0) {
    const double alpha = a.st->alpha;
    const int64_t Pt = a.slot_hi - a.slot_lo;
    for (int64_t r = tid; r < Pt; r += nthr) {
      const int32_t j = a.perm[a.slot_lo + r];
      a.w[j] += alpha * a.d[r];
    }
  }
}

// ---------------------------------------------------------------------------
// deterministic sum, loss terms, margins
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_sum(const double* x, int64_t m, double* part,
                                                unsigned* counter, double* out) {
  __shared__ double lds4[kWavesPerBlock];
  __shared__ bool is_last;
  double s = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * kBlock)
    s += x[i];
  s = block_sum(s, lds4);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) is_last = atomicAdd(counter, 1u) == gridDim.x - 1;
  __syncthreads();
  if (!is_last) return;
  __threadfence();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int b = 0; b < (int)gridDim.x; ++b) t += part[b];
    *out = t;
    *counter = 0u;
  }
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

__global__ void k_abs(const double* w, int64_t p, double* out) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j < p) out[j] = fabs(w[j]);
}

__global__ __launch_bounds__(kBlock) void k_margins(const int64_t* cp, const int32_t* ri,
                                                    const float* v, const double* w,
                                                    const int32_t* cstart,
                                                    const int32_t* chunk_slot, int64_t p,
                                                    double* z) {
  const int lane = lane_id();
  const int64_t wave = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
  const int64_t nwaves = (int64_t)gridDim.x * kWavesPerBlock;
  const int32_t c_hi = cstart[p];
  for (int64_t c = wave; c < c_hi; c += nwaves) {
    const int32_t j = chunk_slot[c];
    const double wj = w[j];
    if (wj == 0.0) continue;
    const int64_t klo = cp[j] + (int64_t)(c - cstart[j]) * kChunk;
    const int64_t khi = klo + kChunk < cp[j + 1] ? klo + kChunk : cp[j + 1];
    for (int64_t k = klo + lane; k < khi; k += kWave)
      unsafeAtomicAdd(&z[ri[k]], wj * (double)v[k]);
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

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_fill(double* a, double v, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_fill, dim3(grid_for(n, kBlock, 4096)), dim3(kBlock), 0, s, a, v, n);
  return hipGetLastError();
}

hipError_t launch_perm_keys(uint64_t stream_seed, int64_t p, uint32_t* keys, int32_t* idx,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_perm_keys, dim3(grid_for(p, kBlock, 1 << 30)), dim3(kBlock), 0, s,
                     stream_seed, p, keys, idx);
  return hipGetLastError();
}

int64_t scan_tmp_ints(int64_t m) { return (m + kScanTile - 1) / kScanTile + 1; }

hipError_t launch_scan(const int32_t* in, int32_t* out, int64_t m, int32_t* tmp, hipStream_t s) {
  const int64_t nb = (m + kScanTile - 1) / kScanTile;
  if (nb < 1) {
    hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(kScanThreads), 0, s, tmp, (int64_t)0,
                       out + m);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_scan_blocks, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, out, m,
                     tmp);
  hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(kScanThreads), 0, s, tmp, nb, out + m);
  hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nb), dim3(kScanThreads), 0, s, out, m, tmp);
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
    hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)ntiles), dim3(kSortThreads), 0, s, kin,
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

hipError_t launch_chunks(const int32_t* perm, const int64_t* cp, int64_t p, int32_t* nch,
                         int32_t* cstart, int32_t* chunk_slot, int32_t* tmp, hipStream_t s) {
  hipLaunchKernelGGL(k_chunk_count, dim3(grid_for(p, kBlock, 1 << 30)), dim3(kBlock), 0, s, perm,
                     cp, p, nch);
  hipError_t e = launch_scan(nch, cstart, p, tmp, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_chunk_fill, dim3(grid_for(p, kBlock, 1 << 30)), dim3(kBlock), 0, s,
                     cstart, p, chunk_slot);
  return hipGetLastError();
}

hipError_t launch_sweep(int loss, int stopping_mode, const SweepArgs& a, int grid,
                        hipStream_t s) {
  if (loss == kLogistic) {
    if (stopping_mode)
      hipLaunchKernelGGL((k_sweep<kLogistic, true>), dim3(grid), dim3(kBlock), 0, s, a);
    else
      hipLaunchKernelGGL((k_sweep<kLogistic, false>), dim3(grid), dim3(kBlock), 0, s, a);
  } else {
    if (stopping_mode)
      hipLaunchKernelGGL((k_sweep<kL2Svm, true>), dim3(grid), dim3(kBlock), 0, s, a);
    else
      hipLaunchKernelGGL((k_sweep<kL2Svm, false>), dim3(grid), dim3(kBlock), 0, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_scatter_split(const SweepArgs& a, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_scatter_split, dim3(grid), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_linesearch(int loss, const LsArgs& a, int grid, hipStream_t s) {
  if (loss == kLogistic)
    hipLaunchKernelGGL(k_linesearch<kLogistic>, dim3(grid), dim3(kBlock), 0, s, a);
  else
    hipLaunchKernelGGL(k_linesearch<kL2Svm>, dim3(grid), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_apply(int loss, const ApplyArgs& a, int grid, hipStream_t s) {
  if (loss == kLogistic)
    hipLaunchKernelGGL(k_apply<kLogistic>, dim3(grid), dim3(kBlock), 0, s, a);
  else
    hipLaunchKernelGGL(k_apply<kL2Svm>, dim3(grid), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_sum(const double* a, int64_t m, double* part, unsigned* counter, double* out,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_sum, dim3(kSumGrid), dim3(kBlock), 0, s, a, m, part, counter, out);
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

hipError_t launch_abs(const double* w, int64_t p, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_abs, dim3(grid_for(p, kBlock, 1 << 30)), dim3(kBlock), 0, s, w, p, out);
  return hipGetLastError();
}

hipError_t launch_margins(const int64_t* cp, const int32_t* ri, const float* v, const double* w,
                          const int32_t* id_cstart, const int32_t* id_slot, int64_t p, double* z,
                          int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_margins, dim3(grid), dim3(kBlock), 0, s, cp, ri, v, w, id_cstart, id_slot,
                     p, z);
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
