/*
 * CPU ORACLE for flow routing -- TEST INFRASTRUCTURE, NOT PART OF THE LIBRARY.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this code.  It shares no code with the GPU library: no headers,
 * no helpers, no tables.  It is deliberately plain and slow, computes in
 * float64 / uint64, and follows the paper (W. Bangerth, "Massively parallel
 * flow routing and drainage area determination") step by step:
 *
 *   local flow routing (Section 2.1; Appendix A for multiple receivers)
 *   -> sort all cells high-to-low (Section 2.1, eq. high-to-low-procedure)
 *   -> in that order, each cell's water is its rain plus the shares of its
 *      donors (a row of (I - W^T) q = r, Section 2.2), every donor being
 *      higher and so already final
 *   -> mass balance check: water leaving through sinks equals total rain
 *      (Section 4, verification paragraph).
 *
 * The result is the unique solution q of (I - W^T) q = r (Section 2.2,
 * eq. linear-system / Aw=f), W[i][k] being the fraction of cell i's water
 * given to cell k.  The adjoint solves (I - W) rbar = qbar by the same sweep
 * in reverse (low-to-high) order.
 *
 * Readings of points the paper leaves open (all stated here, once):
 *  - grid: row-major, row 0 first; neighbour k = 0..7 in row-major window
 *    order (-1,-1) (-1,0) (-1,+1) (0,-1) (0,+1) (+1,-1) (+1,0) (+1,+1), where
 *    row -1 is the previous row in memory; off-grid neighbours do not exist.
 *  - "lower" is strict: z_k < z_i.  A cell with no lower neighbour (boundary
 *    outlet, pit or flat) is a sink and keeps its water.
 *  - D8 "steepest downhill gradient" (Section 2.1): slope = drop / distance,
 *    cell size 1, distance sqrt(2) on diagonals, evaluated in float32 as
 *    s_k = fl(fl(z_i - z_k) * c_k), c_k = 1 (cardinal) or fl(1/sqrt 2)
 *    (diagonal); argmax over lower k, ties to the lowest k.  Because this
 *    float decision picks an integer, it is taken in float32, the GPU's
 *    precision.  D4 uses the four cardinal neighbours only.
 *  - MFD (Appendix A): fraction f_k = s_k^p / sum_j s_j^p over strictly lower
 *    neighbours, s_k = (z_i - z_k) / d_k in float64, d_k = 1 or sqrt(2),
 *    p = 1.1 by default (Freeman-type slope-power partition).
 *  - The high-to-low listing sorts pairs by src; it assumes a high-to-low
 *    numbering, so here cells are sorted by elevation, descending, equal
 *    elevations by ascending index.  Any order of equal elevations gives the
 *    same result because equal cells never exchange water.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_SINK 0xFF
#define OR_D8 0
#define OR_MFD 1
#define OR_D4 2

static const int NB_DR[8] = {-1, -1, -1, 0, 0, 1, 1, 1};
static const int NB_DC[8] = {-1, 0, 1, -1, 1, -1, 0, 1};
static const int NB_DIAG[8] = {1, 0, 1, 0, 0, 1, 0, 1};
/* float32 nearest to 1/sqrt(2): bit pattern 0x3F3504F3 */
static const float INV_SQRT2_F = 0x1.6a09e6p-1f;

/* Neighbour k of cell (r, c), or -1 when it lies off the grid. */
static inline int64_t neighbour(int64_t nr, int64_t nc, int64_t r, int64_t c, int k) {
  const int64_t rr = r + NB_DR[k], cc = c + NB_DC[k];
  if (rr < 0 || rr >= nr || cc < 0 || cc >= nc) return -1;
  return rr * nc + cc;
}

/* ---------------------------------------------------------------------------
 * Local flow routing, single receiver (Section 2.1): D8 or D4 direction code
 * 0..7 of the steepest strictly lower neighbour, OR_SINK if there is none.
 */
static uint8_t single_receiver(const float* z, int64_t nr, int64_t nc, int64_t r, int64_t c,
                               int rule) {
  const float zi = z[r * nc + c];
  int best = -1;
  float best_s = 0.0f;
  for (int k = 0; k < 8; ++k) {
    if (rule == OR_D4 && NB_DIAG[k]) continue;
    const int64_t j = neighbour(nr, nc, r, c, k);
    if (j < 0) continue;
    const float zk = z[j];
    if (!(zk < zi)) continue;
    const float drop = zi - zk;
    const float s = NB_DIAG[k] ? drop * INV_SQRT2_F : drop;
    if (best < 0 || s > best_s) {
      best = k;
      best_s = s;
    }
  }
  return best < 0 ? (uint8_t)OR_SINK : (uint8_t)best;
}

int or_receivers(const float* z, int64_t nr, int64_t nc, int rule, uint8_t* code) {
  if (!z || !code || nr < 0 || nc < 0 || (rule != OR_D8 && rule != OR_D4)) return -2;
  for (int64_t r = 0; r < nr; ++r)
    for (int64_t c = 0; c < nc; ++c) code[r * nc + c] = single_receiver(z, nr, nc, r, c, rule);
  return 0;
}

/* Receiver cell of cell i under direction code cd, or -1 for a sink. */
static inline int64_t code_target(int64_t nc, int64_t i, uint8_t cd) {
  if (cd == OR_SINK) return -1;
  return i + (int64_t)NB_DR[cd] * nc + NB_DC[cd];
}

/* ---------------------------------------------------------------------------
 * Local flow routing, multiple receivers (Appendix A): lower-neighbour mask
 * (bit k set when neighbour k is strictly lower) and fractions f_k.
 * frac32 != 0 evaluates the same law in float32 arithmetic (used only to
 * separate fraction rounding from accumulation rounding in error reports).
 */
static int mfd_split(const float* z, int64_t nr, int64_t nc, int64_t r, int64_t c, double p,
                     int frac32, int64_t nb[8], double f[8]) {
  const int64_t i = r * nc + c;
  int m = 0;
  double w[8], sum = 0.0;
  float w32[8], sum32 = 0.0f;
  for (int k = 0; k < 8; ++k) {
    const int64_t j = neighbour(nr, nc, r, c, k);
    if (j < 0 || !(z[j] < z[i])) continue;
    nb[m] = j;
    if (frac32) {
      const float s = NB_DIAG[k] ? (z[i] - z[j]) * INV_SQRT2_F : (z[i] - z[j]);
      w32[m] = powf(s, (float)p);
      sum32 += w32[m];
    } else {
      const double s = ((double)z[i] - (double)z[j]) / (NB_DIAG[k] ? sqrt(2.0) : 1.0);
      w[m] = pow(s, p);
      sum += w[m];
    }
    ++m;
  }
  for (int t = 0; t < m; ++t) f[t] = frac32 ? (double)(w32[t] / sum32) : w[t] / sum;
  return m;
}

int or_mfd_fractions(const float* z, int64_t nr, int64_t nc, double p, int frac32, uint8_t* mask,
                     double* frac /* 8 per cell, slot k for neighbour k, or NULL */) {
  if (!z || nr < 0 || nc < 0) return -2;
  for (int64_t r = 0; r < nr; ++r) {
    for (int64_t c = 0; c < nc; ++c) {
      const int64_t i = r * nc + c;
      int64_t nb[8];
      double f[8];
      const int m = mfd_split(z, nr, nc, r, c, p, frac32, nb, f);
      uint8_t bits = 0;
      if (frac) memset(frac + 8 * i, 0, 8 * sizeof(double));
      int t = 0;
      for (int k = 0; k < 8 && t < m; ++k) {
        if (neighbour(nr, nc, r, c, k) == nb[t]) {
          bits |= (uint8_t)(1u << k);
          if (frac) frac[8 * i + k] = f[t];
          ++t;
        }
      }
      if (mask) mask[i] = bits;
    }
  }
  return 0;
}

/* ---------------------------------------------------------------------------
 * High-to-low order (Section 2.1): sort keys pack a descending float key in
 * the high 32 bits and the cell index in the low 32 bits, so one ascending
 * sort of the keys gives elevation descending, index ascending.
 */
static int cmp_u64(const void* a, const void* b) {
  const uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
  return (x > y) - (x < y);
}

int or_order(const float* z, int64_t n, int64_t* order /* n entries, output */) {
  if (!z || !order || n < 0 || n > ((int64_t)1 << 32)) return -2;
  uint64_t* key = (uint64_t*)order; /* sorted in place, then unpacked */
  for (int64_t i = 0; i < n; ++i) {
    float v = z[i];
    if (v == 0.0f) v = 0.0f; /* -0 and +0 are the same elevation */
    uint32_t u;
    memcpy(&u, &v, sizeof u);
    u = (u & 0x80000000u) ? ~u : (u | 0x80000000u); /* ascending with v */
    key[i] = ((uint64_t)(~u) << 32) | (uint64_t)(uint32_t)i;
  }
  qsort(key, (size_t)n, sizeof(uint64_t), cmp_u64);
  for (int64_t t = 0; t < n; ++t) order[t] = (int64_t)(key[t] & 0xFFFFFFFFu);
  return 0;
}

/* ---------------------------------------------------------------------------
 * Global flow routing (Section 2.1; Section 2.2: q solves (I - W^T) q = r).
 * Row i of that system reads q_i = r_i + sum over donors d of f_{d->i} q_d,
 * the donors being the neighbours that give i (part of) their water.  Every
 * donor is strictly higher than i, so taking the cells from high to low
 * (Section 2.1) finds each donor's value final when it is needed.
 */

/* Share of donor d's water that goes to cell i (0 when none): D8/D4 codes
 * (code != NULL) or MFD fractions from z. */
static double share(const uint8_t* code, const float* z, int64_t nr, int64_t nc, double p, int frac32,
                    int64_t d, int64_t i) {
  if (code) return code_target(nc, d, code[d]) == i ? 1.0 : 0.0;
  int64_t nb[8];
  double f[8];
  const int m = mfd_split(z, nr, nc, d / nc, d % nc, p, frac32, nb, f);
  for (int t = 0; t < m; ++t)
    if (nb[t] == i) return f[t];
  return 0.0;
}

/* Sum over the donors of i of share * x[donor], neighbours taken in order
 * k = 0..7.  frac != NULL: the MFD fractions of every cell, precomputed
 * (slot 8 d + j for neighbour j of d; neighbour k of i sees i as its
 * neighbour 7 - k). */
static double donor_sum(const uint8_t* code, const float* z, int64_t nr, int64_t nc, double p, int frac32,
                        const double* frac, const double* x, int64_t i) {
  double s = 0.0;
  for (int k = 0; k < 8; ++k) {
    const int64_t d = neighbour(nr, nc, i / nc, i % nc, k);
    if (d < 0) continue;
    const double f = frac ? frac[8 * d + (7 - k)] : share(code, z, nr, nc, p, frac32, d, i);
    if (f != 0.0) s += f * x[d];
  }
  return s;
}

static uint64_t donor_count(const uint8_t* code, int64_t nr, int64_t nc, const uint64_t* cnt, int64_t i) {
  uint64_t s = 0;
  for (int k = 0; k < 8; ++k) {
    const int64_t d = neighbour(nr, nc, i / nc, i % nc, k);
    if (d >= 0 && code_target(nc, d, code[d]) == i) s += cnt[d];
  }
  return s;
}

/*
 * Single receiver (D8/D4 codes): q in float64 and/or exact cell counts
 * (unit rain); rain == NULL means unit rain (drainage area, Section 1).
 */
int or_accumulate_single(const uint8_t* code, int64_t nr, int64_t nc, const int64_t* order,
                         const float* rain, double* q, uint64_t* counts) {
  if (!code || !order || nr < 0 || nc < 0) return -2;
  const int64_t n = nr * nc;
  for (int64_t t = 0; t < n; ++t) {
    const int64_t i = order[t];
    if (q) q[i] = (rain ? (double)rain[i] : 1.0) + donor_sum(code, NULL, nr, nc, 0.0, 0, NULL, q, i);
    if (counts) counts[i] = 1 + donor_count(code, nr, nc, counts, i);
  }
  return 0;
}

/* Multiple receivers (Appendix A): every cell's fractions computed from z
 * once, up front. */
int or_accumulate_mfd(const float* z, int64_t nr, int64_t nc, double p, int frac32,
                      const int64_t* order, const float* rain, double* q) {
  if (!z || !order || !q || nr < 0 || nc < 0) return -2;
  const int64_t n = nr * nc;
  double* frac = (double*)malloc((size_t)(8 * n + 1) * sizeof(double));
  if (!frac) return -2;
  or_mfd_fractions(z, nr, nc, p, frac32, NULL, frac);
  for (int64_t t = 0; t < n; ++t) {
    const int64_t i = order[t];
    q[i] = (rain ? (double)rain[i] : 1.0) + donor_sum(NULL, z, nr, nc, p, frac32, frac, q, i);
  }
  free(frac);
  return 0;
}

/*
 * Adjoint (transpose) solves: (I - W) rbar = qbar.  Row i of I - W couples i
 * to its receivers only, which are lower and therefore come later in the
 * high-to-low order, so the sweep runs that order backwards:
 * rbar[i] = qbar[i] + sum_k f_k * rbar[k].
 */
int or_adjoint_single(const uint8_t* code, int64_t nr, int64_t nc, const int64_t* order,
                      const double* qbar, double* rbar) {
  if (!code || !order || !qbar || !rbar || nr < 0 || nc < 0) return -2;
  const int64_t n = nr * nc;
  for (int64_t i = 0; i < n; ++i) rbar[i] = qbar[i];
  for (int64_t t = n - 1; t >= 0; --t) {
    const int64_t i = order[t];
    const int64_t k = code_target(nc, i, code[i]);
    if (k >= 0) rbar[i] += rbar[k];
  }
  return 0;
}

int or_adjoint_mfd(const float* z, int64_t nr, int64_t nc, double p, const int64_t* order,
                   const double* qbar, double* rbar) {
  if (!z || !order || !qbar || !rbar || nr < 0 || nc < 0) return -2;
  const int64_t n = nr * nc;
  for (int64_t i = 0; i < n; ++i) rbar[i] = qbar[i];
  for (int64_t t = n - 1; t >= 0; --t) {
    const int64_t i = order[t];
    int64_t nb[8];
    double f[8];
    const int m = mfd_split(z, nr, nc, i / nc, i % nc, p, 0, nb, f);
    double acc = rbar[i];
    for (int s = 0; s < m; ++s) acc += f[s] * rbar[nb[s]];
    rbar[i] = acc;
  }
  return 0;
}

/*
 * Product y = A x with A = I - W^T (Section 2.2, eq. linear-system; Appendix
 * A for fractions), row by row: y_i = x_i - sum over donors d of
 * f_{d->i} x_d.  Used for the residual r - A q.
 */
int or_apply_A_single(const uint8_t* code, int64_t nr, int64_t nc, const double* x, double* y) {
  if (!code || !x || !y || nr < 0 || nc < 0) return -2;
  const int64_t n = nr * nc;
  for (int64_t i = 0; i < n; ++i) y[i] = x[i] - donor_sum(code, NULL, nr, nc, 0.0, 0, NULL, x, i);
  return 0;
}

int or_apply_A_mfd(const float* z, int64_t nr, int64_t nc, double p, const double* x, double* y) {
  if (!z || !x || !y || nr < 0 || nc < 0) return -2;
  const int64_t n = nr * nc;
  double* frac = (double*)malloc((size_t)(8 * n + 1) * sizeof(double));
  if (!frac) return -2;
  or_mfd_fractions(z, nr, nc, p, 0, NULL, frac);
  for (int64_t i = 0; i < n; ++i) y[i] = x[i] - donor_sum(NULL, z, nr, nc, p, 0, frac, x, i);
  free(frac);
  return 0;
}

/*
 * Mass balance (Section 4 verification): out[0] = water leaving through
 * sinks (cells with no receiver), out[1] = total rain.
 */
int or_mass_single(const uint8_t* code, int64_t n, const float* rain, const double* q,
                   double out[2]) {
  if (!code || !q || !out || n < 0) return -2;
  double s = 0.0, t = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    if (code[i] == OR_SINK) s += q[i];
    t += rain ? (double)rain[i] : 1.0;
  }
  out[0] = s;
  out[1] = t;
  return 0;
}

int or_mass_mfd(const float* z, int64_t nr, int64_t nc, const float* rain, const double* q,
                double out[2]) {
  if (!z || !q || !out || nr < 0 || nc < 0) return -2;
  double s = 0.0, t = 0.0;
  for (int64_t r = 0; r < nr; ++r) {
    for (int64_t c = 0; c < nc; ++c) {
      const int64_t i = r * nc + c;
      int lower = 0;
      for (int k = 0; k < 8; ++k) {
        const int64_t j = neighbour(nr, nc, r, c, k);
        if (j >= 0 && z[j] < z[i]) lower = 1;
      }
      if (!lower) s += q[i];
      t += rain ? (double)rain[i] : 1.0;
    }
  }
  out[0] = s;
  out[1] = t;
  return 0;
}

/* ---------------------------------------------------------------------------
 * The paper's parallel scheme on one machine: block Richardson iteration
 * (Section 3.3 "I+X" and "(I-X)(I+X)" schemes; Appendix B iteration).
 *
 * The grid is split into blocks of br x bc cells, the paper's per-process
 * subdomains.  D is the part of A = I - W^T that couples cells of one block;
 * the routing pairs that cross a block boundary form the transfer rho (the
 * water a cell passes to a receiver in another block), so A = D - rho and
 * X = D^{-1} R with R = -rho.  Applying D^{-1} is the per-block high-to-low
 * push (the global order restricted to pairs inside a block); applying rho
 * moves each cell's current water across the boundary to its receiver.
 *
 *   scheme 0 (I+X):        w <- D^{-1} (r + rho w)        (Appendix B form)
 *   scheme 1 ((I-X)(I+X)): w <- w + (I - X) (D^{-1} r - (I + X) w)
 *
 * from w = 0, alongside the same iteration on integers (see below).  *iters is the first iteration count l >= 1 whose iterate
 * equals the next one, i.e. the number of iterations after which the
 * solution is exact.  The error of scheme 0 is multiplied by -X each
 * iteration and that of scheme 1 by X^2; X^(C+1) = 0 when flow paths cross
 * block boundaries at most C times, so scheme 0 needs C+1 iterations (the
 * paper's claim) and scheme 1 ceil((C+1)/2).  code != NULL: single receiver
 * (D8/D4 codes); code == NULL: MFD fractions from z with exponent p.
 * q (float64) and counts (exact, unit rain; single receivers only)
 * receive the final iterate; either may be NULL.  Returns 0, -2 on bad arguments, -3 when max_iter
 * iterations do not converge.
 */
static int64_t block_of(int64_t nc, int64_t br, int64_t bc, int64_t i) {
  const int64_t nbc = (nc + bc - 1) / bc;
  return (i / nc / br) * nbc + (i % nc) / bc;
}

/* Whether the pair i -> k belongs to D: both cells in one block. */
static int in_d(int64_t nc, int64_t br, int64_t bc, int64_t i, int64_t k) {
  return block_of(nc, br, bc, k) == block_of(nc, br, bc, i);
}

/* y = rho x (inside == 0) or y = D^{-1} x (inside == 1), in float64 and in
 * uint64 (wrap-around arithmetic: the (I-X)(I+X) scheme subtracts), row by
 * row as in the direct solve: (rho x)_i sums the shares of the donors of i
 * in other blocks; D y = x is solved from high to low with
 * y_i = x_i + the shares of the donors of i in its own block.  Counts use
 * share 1 for every pair (for MFD: the number of flow paths). */
static void block_apply(const uint8_t* code, const float* z, int64_t nr, int64_t nc, double p,
                        const int64_t* order, int64_t br, int64_t bc, int inside,
                        const double* x, const uint64_t* xc, double* y, uint64_t* yc) {
  const int64_t n = nr * nc;
  for (int64_t t = 0; t < n; ++t) {
    const int64_t i = inside ? order[t] : t;
    const double* src = inside ? y : x;
    const uint64_t* srcc = inside ? yc : xc;
    double s = 0.0;
    uint64_t sc = 0;
    for (int k = 0; k < 8; ++k) {
      const int64_t d = neighbour(nr, nc, i / nc, i % nc, k);
      if (d < 0 || in_d(nc, br, bc, d, i) != inside) continue;
      const double f = share(code, z, nr, nc, p, 0, d, i);
      if (f == 0.0) continue;
      s += f * src[d];
      sc += srcc[d];
    }
    y[i] = inside ? x[i] + s : s;
    yc[i] = inside ? xc[i] + sc : sc;
  }
}

int or_block_richardson(const uint8_t* code, const float* z, int64_t nr, int64_t nc, double p,
                        const int64_t* order, const float* rain, int64_t br, int64_t bc,
                        int scheme, int max_iter, double* q, uint64_t* counts, int* iters) {
  if ((!code && !z) || !order || !iters || nr < 0 || nc < 0 || br < 1 || bc < 1 || max_iter < 1 ||
      (scheme != 0 && scheme != 1))
    return -2;
  const size_t n = (size_t)(nr * nc) + 1;
  double* w = (double*)calloc(n, sizeof(double));  /* current iterate */
  double* b = (double*)malloc(n * sizeof(double));  /* D^{-1} r */
  double* nx = (double*)malloc(n * sizeof(double)); /* next iterate */
  double* t1 = (double*)malloc(n * sizeof(double));
  double* t2 = (double*)malloc(n * sizeof(double));
  uint64_t* wc = (uint64_t*)calloc(n, sizeof(uint64_t));
  uint64_t* bcn = (uint64_t*)malloc(n * sizeof(uint64_t));
  uint64_t* nxc = (uint64_t*)malloc(n * sizeof(uint64_t));
  uint64_t* u1 = (uint64_t*)malloc(n * sizeof(uint64_t));
  uint64_t* u2 = (uint64_t*)malloc(n * sizeof(uint64_t));
  int rc = -3;
  if (!w || !b || !nx || !t1 || !t2 || !wc || !bcn || !nxc || !u1 || !u2) {
    rc = -2;
  } else {
    const int64_t m = nr * nc;
    for (int64_t i = 0; i < m; ++i) {
      t1[i] = rain ? (double)rain[i] : 1.0;
      u1[i] = 1;
    }
    block_apply(code, z, nr, nc, p, order, br, bc, 1, t1, u1, b, bcn); /* b = D^{-1} r */
    *iters = 0;
    for (int l = 1; l <= max_iter + 1; ++l) {
      if (scheme == 0) {
        /* next = D^{-1} (r + rho w) */
        block_apply(code, z, nr, nc, p, order, br, bc, 0, w, wc, t1, u1);
        for (int64_t i = 0; i < m; ++i) {
          t1[i] += rain ? (double)rain[i] : 1.0;
          u1[i] += 1;
        }
        block_apply(code, z, nr, nc, p, order, br, bc, 1, t1, u1, nx, nxc);
      } else {
        /* res = b - (I + X) w = b - w + D^{-1} rho w  (into t1/u1) */
        block_apply(code, z, nr, nc, p, order, br, bc, 0, w, wc, t2, u2);
        block_apply(code, z, nr, nc, p, order, br, bc, 1, t2, u2, t1, u1);
        for (int64_t i = 0; i < m; ++i) {
          t1[i] = b[i] - w[i] + t1[i];
          u1[i] = bcn[i] - wc[i] + u1[i];
        }
        /* next = w + (I - X) res = w + res + D^{-1} rho res */
        block_apply(code, z, nr, nc, p, order, br, bc, 0, t1, u1, t2, u2);
        block_apply(code, z, nr, nc, p, order, br, bc, 1, t2, u2, nx, nxc);
        for (int64_t i = 0; i < m; ++i) {
          nx[i] = w[i] + t1[i] + nx[i];
          nxc[i] = wc[i] + u1[i] + nxc[i];
        }
      }
      /* The iterate is exact once the next one equals it, decided on the
       * integer iterate: exact cell counts for single receivers; for MFD the
       * same recurrence with every fraction replaced by 1 counts flow paths
       * (modulo 2^64), which stops changing exactly when no path with more
       * crossings is left.  (Comparing the float iterate instead would stop
       * early wherever the last crossing carries water below the rounding
       * of its receiver's total.) */
      int same = l > 1;
      for (int64_t i = 0; same && i < m; ++i) same = nxc[i] == wc[i];
      if (same) {
        *iters = l - 1;
        rc = 0;
        break;
      }
      memcpy(w, nx, (size_t)m * sizeof(double));
      memcpy(wc, nxc, (size_t)m * sizeof(uint64_t));
    }
    if (rc == 0) {
      if (q) memcpy(q, w, (size_t)m * sizeof(double));
      if (counts && code)
        for (int64_t i = 0; i < m; ++i) counts[i] = (uint64_t)wc[i];
    }
  }
  free(w);
  free(b);
  free(nx);
  free(t1);
  free(t2);
  free(wc);
  free(bcn);
  free(nxc);
  free(u1);
  free(u2);
  return rc;
}

/* ------------------------------------------------------------------------
 * Depression filling before routing (Section 4, where the DEM is filled by
 * the priority-flood method of Barnes et al. 2014 so that all water reaches
 * the domain boundary; Section 5 names this sequential step a bottleneck).
 *
 * Definition.  With next(x) the next float32 above x (eps = 1) or x itself
 * (eps = 0), the filled surface F is the solution of
 *     F(c) = z(c)                                     on the grid boundary,
 *     F(c) = max(z(c), min over neighbours n of next(F(n)))   elsewhere,
 * neighbours being the 8 (conn = 8) or the 4 cardinal (conn = 4) cells.  It
 * equals the lowest, over paths from c to the boundary, of the path's cost,
 * the cost growing along the path from the boundary as f <- max(z, next(f)).
 * With eps = 1 every interior cell then has a strictly lower neighbour, so
 * the strict-descent rules route every cell to the boundary.
 *
 * Method (priority flood): seed all boundary cells with F = z, then pop the
 * open cell of lowest F (ties by index) and give each neighbour not yet
 * reached F = max(z, next(F(popped))).  Because the cost is monotone in
 * F(popped), the first time a cell is reached fixes its value (Dijkstra's
 * argument).  Elevation -0 is read as +0.
 * ------------------------------------------------------------------------ */
typedef struct {
  float v;
  int64_t i;
} heap_item;

static int heap_less(heap_item a, heap_item b) { return a.v < b.v || (a.v == b.v && a.i < b.i); }

static void heap_push(heap_item* h, int64_t* n, heap_item x) {
  int64_t k = (*n)++;
  while (k > 0) {
    const int64_t p = (k - 1) / 2;
    if (!heap_less(x, h[p])) break;
    h[k] = h[p];
    k = p;
  }
  h[k] = x;
}

static heap_item heap_pop(heap_item* h, int64_t* n) {
  const heap_item top = h[0];
  const heap_item last = h[--(*n)];
  int64_t k = 0;
  for (;;) {
    int64_t c = 2 * k + 1;
    if (c >= *n) break;
    if (c + 1 < *n && heap_less(h[c + 1], h[c])) ++c;
    if (!heap_less(h[c], last)) break;
    h[k] = h[c];
    k = c;
  }
  if (*n > 0) h[k] = last;
  return top;
}

int or_fill_depressions(const float* z, int64_t nr, int64_t nc, int conn, int eps, float* out) {
  if (!z || !out || nr < 0 || nc < 0 || (conn != 8 && conn != 4) || (eps != 0 && eps != 1)) return -2;
  const int64_t m = nr * nc;
  for (int64_t i = 0; i < m; ++i)
    if (!isfinite(z[i])) return -5;
  if (m == 0) return 0;
  uint8_t* done = (uint8_t*)calloc((size_t)m, 1);
  heap_item* h = (heap_item*)malloc((size_t)m * sizeof(heap_item));
  if (!done || !h) {
    free(done);
    free(h);
    return -2;
  }
  int64_t n = 0;
  for (int64_t r = 0; r < nr; ++r)
    for (int64_t c = 0; c < nc; ++c)
      if (r == 0 || c == 0 || r == nr - 1 || c == nc - 1) {
        const int64_t i = r * nc + c;
        out[i] = z[i] + 0.0f; /* -0 -> +0 */
        done[i] = 1;
        heap_item x = {out[i], i};
        heap_push(h, &n, x);
      }
  while (n > 0) {
    const heap_item t = heap_pop(h, &n);
    const int64_t r = t.i / nc, c = t.i % nc;
    const float up = eps ? nextafterf(t.v, INFINITY) : t.v;
    for (int k = 0; k < 8; ++k) {
      if (conn == 4 && NB_DIAG[k]) continue;
      const int64_t j = neighbour(nr, nc, r, c, k);
      if (j < 0 || done[j]) continue;
      const float zj = z[j] + 0.0f;
      out[j] = zj > up ? zj : up;
      done[j] = 1;
      heap_item x = {out[j], j};
      heap_push(h, &n, x);
    }
  }
  free(done);
  free(h);
  return 0;
}
