/*
 * Seeded synthetic inputs for flow routing: elevation grids (DEMs), rainfall
 * grids and random draws for tests.  This file holds no routing arithmetic;
 * it is shared by the GPU library's tests/benchmarks and by the CPU oracle's
 * tests, and by nothing else.
 *
 * Stand-in for the paper's Colorado DEM (Section 4, which uses a depression-
 * filled Copernicus GLO-90 model at 3585x2049, 14337x8193 and 57345x32769
 * points): a fractal surface with a planar tilt, so that long trunk rivers
 * cross the whole grid, plus small noise.
 *
 * Random numbers: SplitMix64 (Steele, Lea, Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014) used counter-style: the value
 * for (seed, stream, index) is the SplitMix64 output mixer applied to
 *   key(seed, stream) + (index + 1) * GOLDEN,
 *   key(seed, stream) = mix(seed * GOLDEN + mix(stream + 1)).
 * Every draw is a pure function of its coordinates, so any subset of a grid
 * can be regenerated independently, in any order, by any number of threads.
 *
 * Layout: every grid is row-major, row 0 first in memory, float32.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define GOLDEN 0x9E3779B97F4A7C15ULL

static inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

static inline uint64_t stream_key(uint64_t seed, uint64_t stream) {
  return mix64(seed * GOLDEN + mix64(stream + 1));
}

static inline uint64_t draw_u64(uint64_t key, uint64_t index) {
  return mix64(key + (index + 1) * GOLDEN);
}

/* Uniform double in [0,1) with 53 random bits. */
static inline double draw_unit(uint64_t key, uint64_t index) {
  return (double)(draw_u64(key, index) >> 11) * 0x1.0p-53;
}

/* Stream numbers used by the DEM recipe. */
enum { ST_FRACTAL = 0, ST_NOISE = 1, ST_RAIN = 2 };

uint64_t syn_u64(uint64_t seed, uint64_t stream, uint64_t index) {
  return draw_u64(stream_key(seed, stream), index);
}

/* out[i] = uniform [0,1) double for index start+i. */
void syn_uniform(uint64_t seed, uint64_t stream, int64_t start, int64_t n, double* out) {
  const uint64_t key = stream_key(seed, stream);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) out[i] = draw_unit(key, (uint64_t)(start + i));
}

/* Raw 64-bit draws. */
void syn_u64_array(uint64_t seed, uint64_t stream, int64_t start, int64_t n, uint64_t* out) {
  const uint64_t key = stream_key(seed, stream);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) out[i] = draw_u64(key, (uint64_t)(start + i));
}

/* Smallest k >= 1 with 2^k >= m - 1. */
static int lattice_order(int64_t m) {
  int k = 1;
  while (((int64_t)1 << k) < m - 1) ++k;
  return k;
}

/*
 * Diamond-square fractal (Fournier, Fussell, Carpenter 1982) with Hurst
 * exponent H on a (2^k+1)^2 lattice, 2^k >= max(nrows, ncols) - 1, cropped to
 * the top-left nrows x ncols corner and min-max normalised to [0, 1].
 *   corners: U(-1, 1);
 *   level l = 1..k (step s = 2^(k-l+1), half step h = s/2):
 *     diamond step: each square centre = mean of its 4 corners + d_l,
 *     square step:  each edge midpoint = mean of its in-lattice neighbours at
 *                   distance h (3 on the lattice border, else 4) + d_l,
 *   d_l = U(-1, 1) * 2^(-H l).
 * The draw for lattice point p is stream 0, index p (row-major lattice index),
 * so every point is drawn exactly once.
 * Returns 0, or -1 if memory could not be allocated.
 */
int syn_fractal(uint64_t seed, int64_t nrows, int64_t ncols, double hurst, double* out) {
  const int64_t m = nrows > ncols ? nrows : ncols;
  const int k = lattice_order(m < 2 ? 2 : m);
  const int64_t L = ((int64_t)1 << k) + 1;
  double* g = (double*)malloc((size_t)L * (size_t)L * sizeof(double));
  if (!g) return -1;
  const uint64_t key = stream_key(seed, ST_FRACTAL);
#define G(r, c) g[(int64_t)(r) * L + (c)]
#define U11(r, c) (2.0 * draw_unit(key, (uint64_t)((int64_t)(r) * L + (c))) - 1.0)
  const int64_t e = L - 1;
  G(0, 0) = U11(0, 0);
  G(0, e) = U11(0, e);
  G(e, 0) = U11(e, 0);
  G(e, e) = U11(e, e);
  for (int l = 1; l <= k; ++l) {
    const int64_t s = (int64_t)1 << (k - l + 1);
    const int64_t h = s >> 1;
    const double amp = pow(2.0, -hurst * (double)l);
    /* diamond step: centres of the s x s squares */
#pragma omp parallel for schedule(static)
    for (int64_t r = h; r < L; r += s) {
      for (int64_t c = h; c < L; c += s) {
        const double mean = 0.25 * (G(r - h, c - h) + G(r - h, c + h) + G(r + h, c - h) + G(r + h, c + h));
        G(r, c) = mean + amp * U11(r, c);
      }
    }
    /* square step: edge midpoints, i.e. points with (r/h + c/h) odd */
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < L; r += h) {
      const int64_t c0 = ((r / h) % 2 == 0) ? h : 0;
      for (int64_t c = c0; c < L; c += s) {
        double sum = 0.0;
        int cnt = 0;
        if (r - h >= 0) { sum += G(r - h, c); ++cnt; }
        if (r + h < L) { sum += G(r + h, c); ++cnt; }
        if (c - h >= 0) { sum += G(r, c - h); ++cnt; }
        if (c + h < L) { sum += G(r, c + h); ++cnt; }
        G(r, c) = sum / (double)cnt + amp * U11(r, c);
      }
    }
  }
  double lo = INFINITY, hi = -INFINITY;
#pragma omp parallel for reduction(min : lo) reduction(max : hi) schedule(static)
  for (int64_t r = 0; r < nrows; ++r) {
    for (int64_t c = 0; c < ncols; ++c) {
      const double v = G(r, c);
      if (v < lo) lo = v;
      if (v > hi) hi = v;
    }
  }
  const double span = (hi > lo) ? (hi - lo) : 1.0;
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < nrows; ++r) {
    for (int64_t c = 0; c < ncols; ++c) out[r * ncols + c] = (G(r, c) - lo) / span;
  }
#undef G
#undef U11
  free(g);
  return 0;
}

/*
 * The benchmark DEM: z = fractal(H) + tilt * row + U[0, noise), evaluated in
 * double precision and rounded once to float32 (round-to-nearest-even).
 * Noise draws: stream 1, index = row-major cell index.  Water drains toward
 * row 0.  Returns 0, or -1 on allocation failure.
 */
int syn_dem(uint64_t seed, int64_t nrows, int64_t ncols, double hurst, double tilt, double noise,
            float* z) {
  const int64_t n = nrows * ncols;
  double* f = (double*)malloc((size_t)n * sizeof(double));
  if (!f) return -1;
  if (syn_fractal(seed, nrows, ncols, hurst, f) != 0) {
    free(f);
    return -1;
  }
  const uint64_t key = stream_key(seed, ST_NOISE);
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < nrows; ++r) {
    for (int64_t c = 0; c < ncols; ++c) {
      const int64_t i = r * ncols + c;
      const double v = f[i] + tilt * (double)r + noise * draw_unit(key, (uint64_t)i);
      z[i] = (float)v;
    }
  }
  free(f);
  return 0;
}

/*
 * Rainfall U[0,1) with 24 random bits: r = k * 2^-24, k = top 24 bits of the
 * draw (stream 2, index = cell), so every value is exact in float32.
 */
void syn_rain(uint64_t seed, int64_t n, float* r) {
  const uint64_t key = stream_key(seed, ST_RAIN);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) r[i] = (float)(draw_u64(key, (uint64_t)i) >> 40) * 0x1.0p-24f;
}
