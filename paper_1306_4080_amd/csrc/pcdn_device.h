// Device-side declarations shared by the PCDN kernels and the host driver.
//
// Layout in HBM (per context):
//   X       : col_ptr int64[p+1], row_idx int32[nnz], val fp32[nnz], y int8[n]
//   state   : w fp64[p], cache fp64[n] (e^{w^T x_i} or b_i), dtx fp64[n]
//             (kept all-zero between inner iterations)
//   bundle  : perm int32[p] (slot -> feature), per-slot g, h, d, dterm fp64
//   chunks  : every feature owns ceil(nnz_j / kChunk) >= 1 work chunks;
//             cstart int32[p+1] is the exclusive scan of chunk counts in slot
//             order and chunk_slot int32[] maps a chunk back to its slot, so a
//             wavefront takes one chunk regardless of column length.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pcdn {

constexpr int kWave = 64;
constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kChunk = 1024;   // nonzeros per wavefront work item
constexpr int kQMax = 32;      // line-search candidates evaluated per pass
constexpr int kLogistic = 0;
constexpr int kL2Svm = 1;

// Cumulative device-side counters (read back by the host at sync points).
struct Stats {
  unsigned long long bundles;        // inner iterations
  unsigned long long ls_steps;       // candidates tested (q + 1, or max_ls on failure)
  unsigned long long ls_fail;        // inner iterations without an accepted step
  unsigned long long nnz_gh;         // nonzeros read by the gradient sweep (bundles)
  unsigned long long nnz_scat_fused; // nonzeros scattered into d^T x by the sweep kernel
  unsigned long long nnz_scat_split; // nonzeros scattered by the split-column kernel
  unsigned long long rows_touched;   // rows with d^T x_i != 0, summed over bundles
  unsigned long long slots;          // features swept (bundles)
  unsigned long long nnz_stop;       // nonzeros read by stopping sweeps
  unsigned long long stop_sweeps;    // stopping sweeps run
  unsigned long long pad[6];
};

// Result of the line search of the current inner iteration.
struct StepState {
  double alpha;   // accepted beta^q (0 if none)
  double delta;   // Delta, eq. (7)
  double dF;      // objective change at the accepted q
  int32_t q;      // accepted q, -1 if none
  int32_t pad;
};

struct SweepArgs {
  const int64_t* cp;
  const int32_t* ri;
  const float* v;
  const int8_t* y;
  const double* cache;
  const double* w;            // nullable: treated as zero
  const int32_t* perm;        // slot -> feature
  const int32_t* cstart;      // slot -> first chunk, p+1 entries
  const int32_t* chunk_slot;  // chunk -> slot
  int64_t slot_lo, slot_hi;   // this launch covers slots [slot_lo, slot_hi)
  double* g;                  // outputs indexed by slot - slot_lo
  double* h;
  double* d;
  double* dterm;              // g d + gamma h d^2 + |w + d| - |w|
  double* sg;                 // stopping mode: |grad^S_j F|
  double2* part;              // split-column partial sums, per chunk
  unsigned* cnt;              // split-column arrival counters, per slot
  double* dtx;                // d^T x accumulator
  Stats* stats;
  double C, gamma, nu;
};

struct LsArgs {
  const double* dtx;
  const double* cache;
  const int8_t* y;
  int64_t n;
  const double* w;
  const int32_t* perm;
  int64_t slot_lo, slot_hi;
  const double* d;
  const double* dterm;
  double* part;        // per block: kQMax line-loss sums, kQMax l1 sums, Delta
  unsigned* counter;   // last-block ticket
  StepState* st;
  Stats* stats;
  double C, sigma, beta;
  int q0, Q, max_ls;
};

struct ApplyArgs {
  double* dtx;
  double* cache;
  const int8_t* y;
  int64_t n;
  double* w;
  const int32_t* perm;
  int64_t slot_lo, slot_hi;
  const double* d;
  const StepState* st;
  double beta;
};

// ---- host-callable launchers (pcdn_kernels.hip) -------------------------
hipError_t launch_fill(double* a, double v, int64_t n, hipStream_t s);
hipError_t launch_perm_keys(uint64_t stream_seed, int64_t p, uint32_t* keys, int32_t* idx,
                            hipStream_t s);
// Stable LSD radix sort of (keys, idx) by the 32-bit keys; results end in keys0/idx0.
// hist needs 256 * ceil(p / 4096) + 1 ints, scan_tmp scan_tmp_ints(256 * ceil(p/4096) + 1).
hipError_t launch_radix_sort(uint32_t* keys0, int32_t* idx0, uint32_t* keys1, int32_t* idx1,
                             int64_t p, int32_t* hist, int32_t* scan_tmp, hipStream_t s);
int64_t scan_tmp_ints(int64_t m);
// Exclusive scan of in[0..m) into out[0..m], out[m] = total (int32).
hipError_t launch_scan(const int32_t* in, int32_t* out, int64_t m, int32_t* tmp, hipStream_t s);
// Chunk bookkeeping for a slot order: nch[r] = max(1, ceil(len(perm[r]) / kChunk)),
// cstart = scan(nch), chunk_slot filled.
hipError_t launch_chunks(const int32_t* perm, const int64_t* cp, int64_t p, int32_t* nch,
                         int32_t* cstart, int32_t* chunk_slot, int32_t* tmp, hipStream_t s);
hipError_t launch_sweep(int loss, int stopping_mode, const SweepArgs& a, int grid, hipStream_t s);
hipError_t launch_scatter_split(const SweepArgs& a, int grid, hipStream_t s);
hipError_t launch_linesearch(int loss, const LsArgs& a, int grid, hipStream_t s);
hipError_t launch_apply(int loss, const ApplyArgs& a, int grid, hipStream_t s);
// Deterministic sum of a[0..m) into *out (two levels, fixed grid).
hipError_t launch_sum(const double* a, int64_t m, double* part, unsigned* counter, double* out,
                      hipStream_t s);
hipError_t launch_loss_terms(int loss, const double* cache, const int8_t* y, int64_t n,
                             double* out, hipStream_t s);
hipError_t launch_abs(const double* w, int64_t p, double* out, hipStream_t s);
// z = X w by scattering every column (atomics), then the retained quantities.
hipError_t launch_margins(const int64_t* cp, const int32_t* ri, const float* v, const double* w,
                          const int32_t* id_cstart, const int32_t* id_slot, int64_t p, double* z,
                          int grid, hipStream_t s);
hipError_t launch_cache_from_z(int loss, double* z_to_cache, const int8_t* y, int64_t n,
                               hipStream_t s);

constexpr int kSumGrid = 256;

}  // namespace pcdn
