/*
 * PCDN reference oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded FP64 implementation of Parallel Coordinate
 * Descent Newton (Bian, Li, Liu, Yang: "Parallel Coordinate Descent Newton
 * Method for Efficient L1-Regularized Loss Minimization", arXiv:1306.4080)
 * for L1-regularised logistic regression and L1-regularised L2-loss SVM,
 * and the paper's concluding generalisation to other separable regularisers
 * (ridge, elastic net).
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
 * load this code.  The GPU library shares no code, header, table or helper with
 * it.  Every routine follows the paper's definitions in the paper's order: sums
 * run in storage order (features in bundle order, samples in index order) with
 * no blocking, fusion or reordering.  fp32 matrix values are read exactly as
 * FP64.
 *
 * Notation: the paper writes s samples and n features; this file writes
 * n samples and p features.  C is the loss weight (the paper's c).
 *
 * Pins: every function here is checked in tests/test_oracle_pins.py against
 * something other than itself (brute force, closed forms, finite differences,
 * high-precision recomputation, an independent CDN, published RNG outputs).
 */
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { ORC_LOGISTIC = 0, ORC_L2SVM = 1 };
enum { ORC_PEN_L1 = 0, ORC_PEN_ELASTIC = 1, ORC_PEN_L2 = 2 };

/* Design matrix in compressed sparse column form plus labels.  Column j holds
 * rows row_idx[col_ptr[j] .. col_ptr[j+1]) with values val[...]; y[i] = +-1. */
typedef struct {
  int64_t n, p;
  const int64_t* col_ptr;
  const int32_t* row_idx;
  const float* val;
  const int8_t* y;
} orc_X;

/* Loss and Armijo parameters (Sec. 2.1; the experiments use sigma = 0.01,
 * gamma = 0, beta = 0.5; nu = 1e-12 is the Hessian floor of Lemma 1(b)'s
 * proof).
 *
 * Regulariser.  Eq. (1) is F(w) = ||w||_1 + C sum_i phi_i.  The conclusion
 * (Sec. 6) extends PCDN to any separable regulariser; this oracle takes
 * R(w) = sum_j [a |w_j| + (b/2) w_j^2] in place of ||w||_1 everywhere it
 * appears: in F, in the one-dimensional subproblem eq. (4), in Delta
 * eq. (7) and in the Armijo test eq. (6).  penalty selects
 *   ORC_PEN_L1      a = 1, b = 0   (eq. (1), the default)
 *   ORC_PEN_ELASTIC a = 1, b = l2  (elastic net)
 *   ORC_PEN_L2      a = 0, b = l2  (ridge).
 * g_j and h_j stay those of the loss term C sum_i phi_i. */
typedef struct {
  int32_t loss;
  int32_t max_ls;
  double C, sigma, beta, gamma, nu;
  int32_t shrink;   /* outer-iteration shrinking (see orc_solve); 0: off */
  int32_t penalty;  /* ORC_PEN_* */
  double l2;        /* b of the elastic-net and ridge penalties */
} orc_par;

/* a and b of R for the parameters. */
static double reg_a(const orc_par* par) { return par->penalty == ORC_PEN_L2 ? 0.0 : 1.0; }
static double reg_b(const orc_par* par) { return par->penalty == ORC_PEN_L1 ? 0.0 : par->l2; }

typedef struct {
  double alpha;   /* accepted step beta^q, 0 when the search failed        */
  double delta;   /* Delta of the Armijo rule, eq. (7), at q = 0            */
  double dF;      /* F(w + alpha d) - F(w) at the accepted q (from caches)  */
  int32_t q;      /* accepted backtracking index, -1 if none of max_ls      */
  int32_t pad;
  double margin;  /* smallest |dF - sigma Delta_q| / S over the candidates
                     tested, S = |sigma Delta_q| + the rounding scales of
                     the terms dF is summed from (see change_scale; +inf
                     when S is 0): how far each Armijo decision was from its
                     threshold on the scale of the rounding errors of its
                     two sides                                              */
} orc_step_info;

typedef struct {
  int32_t outer_iters;
  int32_t converged;
  int64_t bundles;     /* inner iterations run                            */
  int64_t ls_steps;    /* line-search evaluations (q + 1 per inner iter)  */
  int64_t ls_fail;     /* inner iterations whose search found no step     */
  int64_t nnz_swept;   /* sum over inner iterations of nnz of the bundle  */
  double objective;    /* F(w) at exit, from the retained quantities      */
  double subgrad;      /* ||grad^S F(w)||_1 at exit                       */
  double subgrad0;     /* ||grad^S F(0)||_1, the stopping reference       */
  /* how close the decisions came to their thresholds (instrumentation; no
   * decision depends on them): the smallest Armijo margin of any inner
   * iteration (orc_step_info.margin) and the smallest
   * |G_k - eps G0| / (eps G0) of any stopping test after an outer iteration */
  double min_armijo_margin;
  double min_stop_margin;
} orc_info;

/* ------------------------------------------------------------------------ */
/* Counter-based random numbers: SplitMix64 (Steele, Lea, Flood, "Fast       */
/* splittable pseudorandom number generators", OOPSLA 2014).  The generator  */
/* state advances by the golden-ratio increment and each output is the       */
/* state passed through the published 64-bit finaliser.                      */
/* ------------------------------------------------------------------------ */
static uint64_t sm64_finalise(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* The i-th output (i = 0, 1, ...) of a SplitMix64 generator seeded with s. */
uint64_t orc_splitmix64(uint64_t s, uint64_t i) {
  return sm64_finalise(s + (i + 1) * 0x9E3779B97F4A7C15ULL);
}

typedef struct {
  uint32_t key;
  int32_t j;
} key_index;

static int cmp_key_index(const void* a, const void* b) {
  const key_index* x = (const key_index*)a;
  const key_index* y = (const key_index*)b;
  if (x->key != y->key) return x->key < y->key ? -1 : 1;
  return (x->j > y->j) - (x->j < y->j);
}

/* Random disjoint partition of the features for outer iteration k (eq. (8),
 * Algorithm 3): a uniformly random permutation; bundle t is the slice
 * [tP, min((t+1)P, p)).  The paper does not fix the generator; here feature j
 * draws the key (upper 32 bits of) output j of the SplitMix64 stream seeded
 * with output k of the stream seeded with `seed`, and the permutation sorts
 * features by (key, j). */
void orc_permutation(uint64_t seed, int64_t k, int64_t p, int32_t* perm) {
  key_index* a = (key_index*)malloc((size_t)p * sizeof(key_index));
  uint64_t stream = orc_splitmix64(seed, (uint64_t)k);
  for (int64_t j = 0; j < p; ++j) {
    a[j].key = (uint32_t)(orc_splitmix64(stream, (uint64_t)j) >> 32);
    a[j].j = (int32_t)j;
  }
  qsort(a, (size_t)p, sizeof(key_index), cmp_key_index);
  for (int64_t r = 0; r < p; ++r) perm[r] = a[r].j;
  free(a);
}

/* The partition restricted to the active features (shrinking): active
 * features keep their keys (capped at 0xFFFFFFFE), inactive ones take
 * 0xFFFFFFFF, so the active features come first, in the order of the full
 * permutation; returns their count. */
int64_t orc_permutation_active(uint64_t seed, int64_t k, int64_t p, const char* active,
                               int32_t* perm) {
  key_index* a = (key_index*)malloc((size_t)p * sizeof(key_index));
  uint64_t stream = orc_splitmix64(seed, (uint64_t)k);
  int64_t n_act = 0;
  for (int64_t j = 0; j < p; ++j) {
    uint32_t key = (uint32_t)(orc_splitmix64(stream, (uint64_t)j) >> 32);
    if (active[j]) {
      if (key == 0xFFFFFFFFu) key = 0xFFFFFFFEu;
      ++n_act;
    } else {
      key = 0xFFFFFFFFu;
    }
    a[j].key = key;
    a[j].j = (int32_t)j;
  }
  qsort(a, (size_t)p, sizeof(key_index), cmp_key_index);
  for (int64_t r = 0; r < p; ++r) perm[r] = a[r].j;
  free(a);
  return n_act;
}

/* ------------------------------------------------------------------------ */
/* Retained per-sample quantities (Sec. 3.1): e^{w^T x_i} for logistic       */
/* regression, b_i = 1 - y_i w^T x_i for the L2-loss SVM.                    */
/* ------------------------------------------------------------------------ */
void orc_margins(const orc_X* X, const double* w, double* z) {
  for (int64_t i = 0; i < X->n; ++i) z[i] = 0.0;
  for (int64_t j = 0; j < X->p; ++j)
    for (int64_t k = X->col_ptr[j]; k < X->col_ptr[j + 1]; ++k)
      z[X->row_idx[k]] += (double)X->val[k] * w[j];
}

void orc_cache_from_w(const orc_X* X, int32_t loss, const double* w, double* cache) {
  orc_margins(X, w, cache);
  for (int64_t i = 0; i < X->n; ++i) {
    double z = cache[i];
    cache[i] = (loss == ORC_LOGISTIC) ? exp(z) : 1.0 - (double)X->y[i] * z;
  }
}

/* tau(y z) = 1 / (1 + e^{-y z}) and 1 - tau(y z), from E = e^{z}; written so
 * that E = 0 and E = +inf give 0 or 1, never NaN. */
static void lr_tau(double E, int y, double* tau, double* one_minus_tau) {
  double u = (y > 0) ? 1.0 / E : E; /* u = e^{-y z} */
  *tau = 1.0 / (1.0 + u);
  *one_minus_tau = 1.0 / (1.0 + 1.0 / u);
}

/* ------------------------------------------------------------------------ */
/* Gradient and (generalised) Hessian diagonal of L for the features in      */
/* `feats`, from the retained quantities.                                    */
/*   LR (eq. (11)):  g_j = C sum_i (tau(y_i z_i) - 1) y_i x_ij,              */
/*                   h_j = C sum_i tau (1 - tau) x_ij^2.                     */
/*   SVM (eq. (3) differentiated; generalised Hessian in the proof of        */
/*   Lemma 1(b)): g_j = -2C sum_{b_i>0} y_i x_ij b_i,                        */
/*                h_j = 2C sum_{b_i>0} x_ij^2.                               */
/* A Hessian entry h_j <= 0 is raised by nu (proof of Lemma 1(b)).           */
/* ------------------------------------------------------------------------ */
void orc_grad_hess(const orc_X* X, const orc_par* par, const double* cache,
                   const int32_t* feats, int64_t m, double* g, double* h) {
  /* features are independent (the multicore build splits them over threads) */
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t t = 0; t < m; ++t) {
    int64_t j = feats[t];
    double gs = 0.0, hs = 0.0;
    for (int64_t k = X->col_ptr[j]; k < X->col_ptr[j + 1]; ++k) {
      int64_t i = X->row_idx[k];
      double x = (double)X->val[k];
      int y = X->y[i];
      if (par->loss == ORC_LOGISTIC) {
        double tau, omt;
        lr_tau(cache[i], y, &tau, &omt);
        gs += -omt * (double)y * x; /* (tau - 1) y x with 1 - tau formed directly */
        hs += tau * omt * x * x;
      } else {
        double b = cache[i];
        if (b > 0.0) {
          gs += (double)y * x * b;
          hs += x * x;
        }
      }
    }
    if (par->loss == ORC_LOGISTIC) {
      g[t] = par->C * gs;
      h[t] = par->C * hs;
    } else {
      g[t] = -2.0 * par->C * gs;
      h[t] = 2.0 * par->C * hs;
    }
    if (h[t] <= 0.0) h[t] += par->nu;
  }
}

/* Closed-form minimiser over d of g d + h d^2 / 2 + R_j(w + d) (eq. (4) with
 * R_j(u) = a |u| + (b/2) u^2 in place of |u|).  With u = w + d, stationarity
 * reads g + h (u - w) + b u + a sign(u) = 0, so u > 0 exactly when
 * g + a < h w, u < 0 exactly when g - a > h w, and u = 0 otherwise.  For
 * a = 1, b = 0 this is eq. (5) (whose printed case conditions are garbled;
 * minimising eq. (4) gives the rule below). */
double orc_newton_direction_reg(double g, double h, double w, double a, double b) {
  if (g + a <= h * w) return -(g + a + b * w) / (h + b);
  if (g - a >= h * w) return -(g - a + b * w) / (h + b);
  return -w;
}

double orc_newton_direction(double g, double h, double w) {
  return orc_newton_direction_reg(g, h, w, 1.0, 0.0);
}

/* Minimum-norm subgradient component of F at w_j given g_j = grad_j L(w):
 * the gradient of the smooth part is G = g + b w, the nonsmooth part a|w|. */
static double min_norm_subgrad(double g, double w, double a, double b) {
  double G = g + b * w;
  if (w > 0.0) return G + a;
  if (w < 0.0) return G - a;
  if (G < -a) return G + a;
  if (G > a) return G - a;
  return 0.0;
}

/* ||grad^S F(w)||_1 over all p features, with grad L from the retained
 * quantities; `gfull` (nullable) receives grad L. */
double orc_subgrad_l1(const orc_X* X, const orc_par* par, const double* w,
                      const double* cache, double* gfull) {
  int32_t* all = (int32_t*)malloc((size_t)X->p * sizeof(int32_t));
  double* g = (double*)malloc((size_t)X->p * sizeof(double));
  double* h = (double*)malloc((size_t)X->p * sizeof(double));
  for (int64_t j = 0; j < X->p; ++j) all[j] = (int32_t)j;
  orc_grad_hess(X, par, cache, all, X->p, g, h);
  double G = 0.0;
  const double ra = reg_a(par), rb = reg_b(par);
  for (int64_t j = 0; j < X->p; ++j) G += fabs(min_norm_subgrad(g[j], w[j], ra, rb));
  if (gfull) memcpy(gfull, g, (size_t)X->p * sizeof(double));
  free(all);
  free(g);
  free(h);
  return G;
}

/* log(p + q e^x) for p, q >= 0 with p + q = 1 and x <= 0: log1p(q expm1(x))
 * while its argument stays above -1/2, else the log of the (then small) sum. */
static double log_mix(double p, double q, double x) {
  double t = q * expm1(x);
  if (t >= -0.5) return log1p(t);
  return log(p + q * exp(x));
}

/* Per-sample loss change when z_i moves to z_i + a (the summand of the
 * descent condition eq. (10)).
 *   LR:  log(1 + e^{-y(z+a)}) - log(1 + e^{-yz}).  With u = e^{-yz},
 *        tau = tau(yz) = 1/(1+u) and m = -y a this equals
 *        log(tau + (1 - tau) e^m) = m + log((1 - tau) + tau e^{-m}); the first
 *        form is used for m <= 0, the second for m > 0, so that no exponential
 *        overflows (eq. (10) writes the same quantity with e^{(w+beta^q d)^T x}).
 *   SVM: max(0, b - y a)^2 - max(0, b)^2. */
static double loss_change(int32_t loss, double cache, int y, double a) {
  if (loss == ORC_LOGISTIC) {
    double tau, omt;
    lr_tau(cache, y, &tau, &omt);
    double m = -(double)y * a;
    if (m <= 0.0) return log_mix(tau, omt, m);
    return m + log_mix(omt, tau, -m);
  } else {
    double bn = cache - (double)y * a;
    double pn = bn > 0.0 ? bn : 0.0;
    double po = cache > 0.0 ? cache : 0.0;
    return pn * pn - po * po;
  }
}

/* Exported for the pin tests: the per-sample change above. */
/* Instrumentation only (no decision reads it): the size of the rounding
 * error a loss change inherits, as a magnitude.  The logistic change is
 * evaluated directly, so it carries its own relative error plus what an
 * error in its argument a moves it by (the derivative in a lies in [-1, 1]);
 * the squared-hinge change is the difference of two squares, whose sizes it
 * inherits, plus the error of the argument times 2 max(0, b - y a). */
static double loss_change_scale(int32_t loss, double cache, int y, double a, double lc) {
  if (loss == ORC_LOGISTIC) return fabs(lc) + fabs(a);
  double bn = cache - (double)y * a;
  double pn = bn > 0.0 ? bn : 0.0;
  double po = cache > 0.0 ? cache : 0.0;
  return pn * pn + po * po + 2.0 * pn * fabs(a);
}

/* Threads of the multicore build (a timing baseline only: the parity oracle
 * is the single-threaded build, whose sums run in the order written).
 * Returns the number the build will use (1 without OpenMP). */
int32_t orc_set_threads(int32_t n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
  return (int32_t)omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}

double orc_loss_change(int32_t loss, double cache, int32_t y, double a) {
  return loss_change(loss, cache, y, a);
}

/* R(w) = a ||w||_1 + (b/2) ||w||_2^2 */
static double regulariser(const orc_par* par, const double* w, int64_t p) {
  double l1 = 0.0, sq = 0.0;
  for (int64_t j = 0; j < p; ++j) {
    l1 += fabs(w[j]);
    sq += w[j] * w[j];
  }
  return reg_a(par) * l1 + 0.5 * reg_b(par) * sq;
}

/* F(w) = R(w) + C sum_i phi_i (eq. (1) with the regulariser above), from the
 * retained quantities. */
double orc_objective_cache(const orc_X* X, const orc_par* par, const double* w,
                           const double* cache) {
  double s = 0.0;
  for (int64_t i = 0; i < X->n; ++i) {
    if (par->loss == ORC_LOGISTIC) {
      /* log(1 + e^{-y z}) with e^{-y z} = E^{-y} */
      s += (X->y[i] > 0) ? log1p(1.0 / cache[i]) : log1p(cache[i]);
    } else {
      double b = cache[i] > 0.0 ? cache[i] : 0.0;
      s += b * b;
    }
  }
  return regulariser(par, w, X->p) + par->C * s;
}

/* F(w) evaluated from X and w directly (no retained quantities). */
double orc_objective_direct(const orc_X* X, const orc_par* par, const double* w) {
  double* z = (double*)malloc((size_t)X->n * sizeof(double));
  orc_margins(X, w, z);
  double s = 0.0;
  for (int64_t i = 0; i < X->n; ++i) {
    double yz = (double)X->y[i] * z[i];
    if (par->loss == ORC_LOGISTIC) {
      /* log(1 + e^{-yz}) */
      s += (yz >= 0.0) ? log1p(exp(-yz)) : -yz + log1p(exp(yz));
    } else {
      double b = 1.0 - yz;
      if (b > 0.0) s += b * b;
    }
  }
  free(z);
  return regulariser(par, w, X->p) + par->C * s;
}

/* ------------------------------------------------------------------------ */
/* One inner iteration t of Algorithm 3 on bundle B (size P):                */
/*   1. d_j = d(w; j) for every j in B (parallel loop of Algorithm 3);       */
/*   2. Delta by eq. (7) with H = diag(h) and R in place of ||.||_1;         */
/*   3. Algorithm 4: d^T x_i for every sample; for q = 0, 1, ...: test the   */
/*      descent condition eq. (10) with the scaled d^T x_i and Delta; on     */
/*      acceptance w += beta^q d and e^{w^T x_i} *= e^{beta^q d^T x_i}       */
/*      (SVM: b_i -= y_i beta^q d^T x_i); on rejection Delta *= beta and     */
/*      d^T x_i *= beta.                                                     */
/* The search stops after max_ls rejections (the paper's loop is unbounded); */
/* then nothing is updated and q = -1.  Outputs g, h, d (length P) and the   */
/* unscaled dtx (length n) are nullable.                                     */
/* ------------------------------------------------------------------------ */
int32_t orc_step(const orc_X* X, const orc_par* par, double* w, double* cache,
                 const int32_t* bundle, int64_t P, double* g_out, double* h_out,
                 double* d_out, double* dtx_out, orc_step_info* info) {
  double* g = (double*)malloc((size_t)P * sizeof(double));
  double* h = (double*)malloc((size_t)P * sizeof(double));
  double* d = (double*)malloc((size_t)P * sizeof(double));
  double* a = (double*)malloc((size_t)X->n * sizeof(double));

  /* 1. one-dimensional Newton directions */
  const double ra = reg_a(par), rb = reg_b(par);
  orc_grad_hess(X, par, cache, bundle, P, g, h);
  for (int64_t t = 0; t < P; ++t)
    d[t] = orc_newton_direction_reg(g[t], h[t], w[bundle[t]], ra, rb);

  /* 2. Delta (eq. (7)); R_j(w + d) - R_j(w) is formed per coordinate, its
   *    quadratic part as b d (w + d/2) */
  double Delta = 0.0;
  for (int64_t t = 0; t < P; ++t) {
    double wj = w[bundle[t]];
    Delta += g[t] * d[t] + par->gamma * h[t] * d[t] * d[t] + ra * fabs(wj + d[t]) -
             ra * fabs(wj) + rb * d[t] * (wj + 0.5 * d[t]);
  }

  /* 3. Algorithm 4: d^T x_i */
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < X->n; ++i) a[i] = 0.0;
  for (int64_t t = 0; t < P; ++t) {
    int64_t j = bundle[t];
    for (int64_t k = X->col_ptr[j]; k < X->col_ptr[j + 1]; ++k)
      a[X->row_idx[k]] += d[t] * (double)X->val[k];
  }
  if (dtx_out) memcpy(dtx_out, a, (size_t)X->n * sizeof(double));

  double Dq = Delta, alpha = 1.0, dF = 0.0, margin = INFINITY;
  int32_t q_acc = -1;
  for (int32_t q = 0; q < par->max_ls; ++q) {
    double l1 = 0.0, l1abs = 0.0; /* R(w + alpha d) - R(w) */
    for (int64_t t = 0; t < P; ++t) {
      double wj = w[bundle[t]], s = alpha * d[t];
      const double r = ra * fabs(wj + s) - ra * fabs(wj) + rb * s * (wj + 0.5 * s);
      l1 += r;
      /* its rounding scale: the magnitudes it is the difference of */
      l1abs += ra * (fabs(wj + s) + fabs(wj)) + fabs(rb * s) * (fabs(wj) + 0.5 * fabs(s));
    }
    double sL = 0.0, sabs = 0.0;
    /* (the multicore build sums over threads: another summation order) */
#pragma omp parallel for reduction(+ : sL, sabs) schedule(static)
    for (int64_t i = 0; i < X->n; ++i) {
      const double lc = loss_change(par->loss, cache[i], X->y[i], a[i]);
      sL += lc;
      sabs += loss_change_scale(par->loss, cache[i], X->y[i], a[i], lc);
    }
    dF = l1 + par->C * sL;
    const double thr = par->sigma * Dq;
    const double scale = fabs(thr) + l1abs + par->C * sabs;
    if (scale != 0.0 && fabs(dF - thr) / scale < margin) margin = fabs(dF - thr) / scale;
    if (dF <= par->sigma * Dq) {
      q_acc = q;
      break;
    }
    Dq *= par->beta;
    alpha *= par->beta;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < X->n; ++i) a[i] *= par->beta;
  }

  if (q_acc >= 0) {
    for (int64_t t = 0; t < P; ++t) w[bundle[t]] += alpha * d[t];
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < X->n; ++i) {
      if (par->loss == ORC_LOGISTIC)
        cache[i] *= exp(a[i]);
      else
        cache[i] -= (double)X->y[i] * a[i];
    }
  }

  if (info) {
    info->alpha = q_acc >= 0 ? alpha : 0.0;
    info->delta = Delta;
    info->dF = q_acc >= 0 ? dF : 0.0;
    info->q = q_acc;
    info->pad = 0;
    info->margin = margin;
  }
  if (g_out) memcpy(g_out, g, (size_t)P * sizeof(double));
  if (h_out) memcpy(h_out, h, (size_t)P * sizeof(double));
  if (d_out) memcpy(d_out, d, (size_t)P * sizeof(double));
  free(g);
  free(h);
  free(d);
  free(a);
  return q_acc;
}

/* ------------------------------------------------------------------------ */
/* Algorithm 3 with an outer stopping rule.  The paper only says its rule is */
/* similar to newGLMNET's outer condition; this oracle stops after outer     */
/* iteration k when ||grad^S F(w^k)||_1 <= eps ||grad^S F(0)||_1, with the   */
/* gradient recomputed over all features from the retained quantities.  If   */
/* the reference norm is 0, w = 0 is optimal and is returned at once.        */
/* w holds the starting point on entry (the paper starts from 0) and the     */
/* result on exit.  trace_F (nullable, max_outer long) receives F after each  */
/* outer iteration.  Returns 0 when converged, 1 when max_outer was hit.     */
/*                                                                          */
/* Shrinking (par->shrink; the paper's experiments shrink between outer     */
/* iterations, not inside the parallel loop, and give no rule): after outer */
/* iteration k, with the gradient g at w^k, feature j stays active for      */
/* iteration k+1 iff w_j != 0 or |g_j| >= a - M_{k-1}/n, where M_{k-1} is   */
/* the largest |grad^S_j F| over all features after iteration k-1          */
/* (M_{-1} = infinity: the first two iterations use every feature; with     */
/* a = 1 the threshold is LIBLINEAR's CDN rule, and with a = 0, ridge, no   */
/* feature is ever left out).  Iteration k+1 partitions only the active     */
/* features (orc_permutation_active) into bundles of P.  The stopping rule  */
/* is unchanged: it uses all features, and a feature is only left out while */
/* its minimum-norm subgradient is 0.                                       */
/* ------------------------------------------------------------------------ */
int32_t orc_solve(const orc_X* X, const orc_par* par, int64_t P, double eps,
                  uint64_t seed, int32_t max_outer, double* w, orc_info* info,
                  double* trace_F) {
  int64_t n = X->n, p = X->p;
  double* cache = (double*)malloc((size_t)n * sizeof(double));
  double* zero_w = (double*)calloc((size_t)p, sizeof(double));
  int32_t* perm = (int32_t*)malloc((size_t)p * sizeof(int32_t));
  orc_info I;
  memset(&I, 0, sizeof(I));
  I.min_armijo_margin = INFINITY;
  I.min_stop_margin = INFINITY;

  /* reference norm at w = 0, where e^{w^T x} = 1 and b = 1 */
  for (int64_t i = 0; i < n; ++i) cache[i] = 1.0;
  I.subgrad0 = orc_subgrad_l1(X, par, zero_w, cache, NULL);

  int converged = 0;
  if (I.subgrad0 == 0.0) {
    for (int64_t j = 0; j < p; ++j) w[j] = 0.0;
    I.subgrad = 0.0;
    converged = 1;
  } else {
    orc_cache_from_w(X, par->loss, w, cache);
    I.subgrad = orc_subgrad_l1(X, par, w, cache, NULL);
    converged = I.subgrad <= eps * I.subgrad0;
  }

  char* active = (char*)malloc((size_t)p);
  double* gfull = (double*)malloc((size_t)p * sizeof(double));
  for (int64_t j = 0; j < p; ++j) active[j] = 1;
  double M_prev = INFINITY;
  while (!converged && I.outer_iters < max_outer) {
    int64_t p_act = p;
    if (par->shrink)
      p_act = orc_permutation_active(seed, I.outer_iters, p, active, perm);
    else
      orc_permutation(seed, I.outer_iters, p, perm);
    int64_t nb = (p_act + P - 1) / P;
    for (int64_t t = 0; t < nb; ++t) {
      int64_t lo = t * P, hi = lo + P < p_act ? lo + P : p_act;
      orc_step_info si;
      int32_t q = orc_step(X, par, w, cache, perm + lo, hi - lo, NULL, NULL, NULL, NULL, &si);
      if (si.margin < I.min_armijo_margin) I.min_armijo_margin = si.margin;
      I.bundles += 1;
      if (q < 0) {
        I.ls_fail += 1;
        I.ls_steps += par->max_ls;
      } else {
        I.ls_steps += q + 1;
      }
      for (int64_t r = lo; r < hi; ++r)
        I.nnz_swept += X->col_ptr[perm[r] + 1] - X->col_ptr[perm[r]];
    }
    if (trace_F) trace_F[I.outer_iters] = orc_objective_cache(X, par, w, cache);
    I.outer_iters += 1;
    I.subgrad = orc_subgrad_l1(X, par, w, cache, gfull);
    converged = I.subgrad <= eps * I.subgrad0;
    if (eps > 0.0) {
      const double sm = fabs(I.subgrad - eps * I.subgrad0) / (eps * I.subgrad0);
      if (sm < I.min_stop_margin) I.min_stop_margin = sm;
    }
    if (par->shrink) {
      double M = 0.0;
      const double thr = reg_a(par) - M_prev / (double)n;
      for (int64_t j = 0; j < p; ++j) {
        const double v = fabs(min_norm_subgrad(gfull[j], w[j], reg_a(par), reg_b(par)));
        if (v > M) M = v;
        active[j] = (w[j] != 0.0 || fabs(gfull[j]) >= thr) ? 1 : 0;
      }
      M_prev = M;
    }
  }
  free(active);
  free(gfull);

  I.converged = converged;
  I.objective = orc_objective_cache(X, par, w, cache);
  if (info) *info = I;
  free(cache);
  free(zero_w);
  free(perm);
  return converged ? 0 : 1;
}
