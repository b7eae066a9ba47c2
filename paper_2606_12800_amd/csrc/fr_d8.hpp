// Row-sweep single-receiver path: tiles, sweeps and helpers shared by the
// phase A, phase B (forest) and phase C translation units.  See
// fr_d8_a.hip for the method.
#pragma once

#include <math.h>

#include <type_traits>

#include "fr_internal.hpp"

namespace fr {
namespace {

constexpr int TW = D8_TW;
constexpr uint32_t NONE = 0xFFFFFFFFu;

struct ff {
  float hi, lo;
};
__device__ __forceinline__ ff ff_two_sum(float a, float b) {
  const float s = a + b;
  const float bb = s - a;
  return {s, (a - (s - bb)) + (b - bb)};
}
__device__ __forceinline__ ff ff_fast(float a, float b) {
  const float s = a + b;
  return {s, b - (s - a)};
}
__device__ __forceinline__ ff ff_add(ff x, ff y) {
  const ff s = ff_two_sum(x.hi, y.hi);
  return ff_fast(s.hi, s.lo + (x.lo + y.lo));
}

// Lane i receives lane i-1's value (lane 0 receives `edge`), or lane i+1's
// (lane 63 receives `edge`): wavefront-wide DPP shifts.
__device__ __forceinline__ uint32_t from_left(uint32_t x, uint32_t edge) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)edge, (int)x, 0x138, 0xF, 0xF, false);
}
__device__ __forceinline__ uint32_t from_right(uint32_t x, uint32_t edge) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)edge, (int)x, 0x130, 0xF, 0xF, false);
}
__device__ __forceinline__ uint32_t from_left(uint32_t x) { return from_left(x, 0u); }
__device__ __forceinline__ uint32_t from_right(uint32_t x) { return from_right(x, 0u); }
__device__ __forceinline__ float from_left(float x) {
  return __uint_as_float(from_left(__float_as_uint(x), 0u));
}
__device__ __forceinline__ float from_right(float x) {
  return __uint_as_float(from_right(__float_as_uint(x), 0u));
}
__device__ __forceinline__ uint64_t from_left(uint64_t x) {
  return ((uint64_t)from_left((uint32_t)(x >> 32), 0u) << 32) | from_left((uint32_t)x, 0u);
}
__device__ __forceinline__ uint64_t from_right(uint64_t x) {
  return ((uint64_t)from_right((uint32_t)(x >> 32), 0u) << 32) | from_right((uint32_t)x, 0u);
}
__device__ __forceinline__ double from_left(double x) {
  return __longlong_as_double((long long)from_left((uint64_t)__double_as_longlong(x)));
}
__device__ __forceinline__ double from_right(double x) {
  return __longlong_as_double((long long)from_right((uint64_t)__double_as_longlong(x)));
}

__device__ __forceinline__ void set_status(int32_t* st, int32_t code) {
  if (st) atomicCAS(st, 0, code);
}

constexpr int W = 4;            // columns per lane
static_assert(TW == 64 * W, "a tile row is one wavefront of W-column lanes");

struct Tile {
  int r0, c0;  // cell indices fit in int32: the library caps grids at 2^31 - 1 cells
  int th, tw;
  bool border;  // touches the grid border (codes may point off the grid)
};

// Workgroups are dispatched round-robin over the XCDs; give each XCD a
// contiguous run of tiles so that horizontally adjacent tiles, which share
// halo columns, share an L2.
__device__ __forceinline__ Tile tile_of(const D8Params& P, int b) {
  const int ntiles = P.ntr * P.ntc;
  const int q = ntiles / 8;
  const int t = (b < 8 * q) ? (b % 8) * q + b / 8 : b;
  Tile T;
  const int tr = t / P.ntc, tc = t - (t / P.ntc) * P.ntc;
  T.r0 = tr * P.th;
  T.c0 = tc * TW;
  T.th = min(P.th, (int)P.nrows - T.r0);
  T.tw = min(TW, (int)P.ncols - T.c0);
  T.border = T.r0 == 0 || T.c0 == 0 || T.r0 + T.th == (int)P.nrows || T.c0 + T.tw == (int)P.ncols;
  return T;
}

// Rain source of a launch: none (unit rain), float32 or float64.
enum RainKind { RAIN_UNIT = 0, RAIN_F32 = 1, RAIN_F64 = 2 };

// Rows whose loads are in flight ahead of a sweep.  Every load is issued
// unconditionally (addresses clamped into the grid, rows and columns outside
// it replaced after arrival) into a ring of registers indexed by the
// unrolled step, so the wait for a row's data never waits for the rows
// behind it.
constexpr int PF_ROWS = 8;

// One grid row as seen by a lane: the W codes of its columns packed in a
// dword (byte j = column 4*lane + j of the tile) and the codes just left and
// right of them.  Off-grid cells read as sinks.
struct Row {
  uint32_t w, l, r;
  __device__ __forceinline__ uint32_t code(int j) const { return (w >> (8 * j)) & 0xFFu; }
  __device__ __forceinline__ uint32_t left(int j) const { return j == 0 ? l : code(j - 1); }
  __device__ __forceinline__ uint32_t right(int j) const { return j == W - 1 ? r : code(j + 1); }
};

// Raw codes of one row for one lane, as loaded.
struct CodeIn {
  uint32_t w;     // own codes (unaligned rows: the first code only)
  uint32_t side;  // lane 0: the column left of the tile; lane 63: right of it
  uint32_t b[W - 1];  // unaligned rows: codes 1..3, combined only when used
};

template <bool VEC>
__device__ __forceinline__ CodeIn load_codes(const D8Params& P, const Tile& T, int r, int lane) {
  const int nr = (int)P.nrows, nc = (int)P.ncols;
  const uint8_t* row = P.code + (size_t)min(max(r, 0), nr - 1) * (size_t)nc;
  const int c = T.c0 + W * lane;
  CodeIn x;
  if (VEC) {
    x.w = *reinterpret_cast<const uint32_t*>(row + min(c, nc - W));
  } else {
    x.w = row[min(c, nc - 1)];
#pragma unroll
    for (int j = 1; j < W; ++j) x.b[j - 1] = row[min(c + j, nc - 1)];
  }
  // Lane 0 reads the column left of the tile, lane 63 the one right of it
  // (c - 1 and c + W); the others re-read their own first column.  Written
  // as arithmetic so that no lane branches.
  const int sc = c + (lane == 0 ? -1 : 0) + (lane == 63 ? W : 0);
  x.side = row[min(max(sc, 0), nc - 1)];
  return x;
}

// The row at grid row r from its loaded codes.  A tile away from the grid
// border only ever touches rows and columns inside the grid.
template <bool BORDER, bool VEC>
__device__ __forceinline__ Row expand_row(const CodeIn& x, const D8Params& P, const Tile& T, int r, int lane) {
  uint32_t w = x.w, side = x.side;
  if (!VEC) w |= (x.b[0] << 8) | (x.b[1] << 16) | (x.b[2] << 24);
  if (BORDER) {
    const int nr = (int)P.nrows, nc = (int)P.ncols;
    const int c = T.c0 + W * lane;
    const bool row_ok = r >= 0 && r < nr;
    uint32_t oob = 0;
#pragma unroll
    for (int j = 0; j < W; ++j) oob |= (c + j >= nc) ? (0xFFu << (8 * j)) : 0u;
    w = row_ok ? (w | oob) : 0xFFFFFFFFu;
    const bool side_ok = row_ok && (lane == 0 ? T.c0 > 0 : T.c0 + TW < nc);
    side = side_ok ? side : (uint32_t)SINK;
  }
  Row y;
  y.w = w;
  y.l = from_left(w, 0xFFFFFFFFu) >> 24;
  y.r = from_right(w, 0xFFFFFFFFu) & 0xFFu;
  if (lane == 0) y.l = side;
  if (lane == 63) y.r = side;
  return y;
}

// Rain of the lane's W cells of grid row r (clamped address; values of
// columns beyond the grid are never used).
template <int RAIN, bool VEC>
struct RainIn {
  using RT = typename std::conditional<RAIN == RAIN_F64, double, float>::type;
  RT v[W];
};

template <int RAIN, bool VEC>
__device__ __forceinline__ RainIn<RAIN, VEC> load_rain(const D8Params& P, const Tile& T, int r, int lane) {
  RainIn<RAIN, VEC> x;
  if (RAIN == RAIN_UNIT) {
#pragma unroll
    for (int j = 0; j < W; ++j) x.v[j] = 1;
    return x;
  }
  const int nr = (int)P.nrows, nc = (int)P.ncols;
  const size_t rb = (size_t)min(max(r, 0), nr - 1) * (size_t)nc;
  const int c = T.c0 + W * lane;
  if (VEC && RAIN == RAIN_F32) {
    const float4 q = *reinterpret_cast<const float4*>(P.rain32 + rb + min(c, nc - W));
    x.v[0] = q.x;
    x.v[1] = q.y;
    x.v[2] = q.z;
    x.v[3] = q.w;
  } else if (VEC) {
    const double* p = P.rain64 + rb + min(c, nc - W);
    const double2 a = *reinterpret_cast<const double2*>(p);
    const double2 b = *reinterpret_cast<const double2*>(p + 2);
    x.v[0] = a.x;
    x.v[1] = a.y;
    x.v[2] = b.x;
    x.v[3] = b.y;
  } else {
#pragma unroll
    for (int j = 0; j < W; ++j) {
      const size_t g = rb + (size_t)min(c + j, nc - 1);
      if (RAIN == RAIN_F32) x.v[j] = P.rain32[g];
      else x.v[j] = (typename RainIn<RAIN, VEC>::RT)P.rain64[g];
    }
  }
  return x;
}

// Classification of the cell in row r, tile column k = W*lane + j.
struct Cell {
  bool sink;  // no receiver (also malformed codes, columns off the grid)
  bool down;  // receiver in row r-1 inside the tile: followed by the sweep
  bool exit;  // receiver across a cut edge
};

template <bool BORDER>
__device__ __forceinline__ Cell classify(const D8Params& P, const Tile& T, int r, int k, uint32_t cd, bool bottom) {
  Cell x;
  bool bad = false;
  if (BORDER) {
    // A code whose receiver lies off the grid is malformed.
    const int dr = cd <= 2u ? -1 : (cd <= 4u ? 0 : 1);
    const int dc = (cd == 0u || cd == 3u || cd == 5u) ? -1 : ((cd == 1u || cd == 6u) ? 0 : 1);
    const int rr = r + dr, cc = T.c0 + k + dc;
    bad = cd <= 7u && (rr < 0 || rr >= (int)P.nrows || cc < 0 || cc >= (int)P.ncols);
  }
  x.sink = cd > 7u || bad || (BORDER && k >= T.tw);
  const int tk = k + (int)cd - 1;  // target column of a down-row code
  x.down = !x.sink && cd <= 2u && !bottom && tk >= 0 && tk < (BORDER ? T.tw : TW);
  x.exit = !x.sink && !x.down;
  return x;
}

// Donors of the cell (row r, tile column k) that reach it over a cut edge,
// as a bit mask in neighbour order (bit n: neighbour n of the cell gives it
// water).  above = row r+1, here = row r, below = row r-1.  `rare` says
// whether any same-row or towards-higher-row donor can exist in this row.
__device__ __forceinline__ uint32_t cut_donors(const Row& above, const Row& here, const Row& below, int j,
                                               int k, bool top, bool rare, int tw) {
  uint32_t m = 0;
  if (rare) {
    m |= (uint32_t)(below.left(j) == 7) << 0;
    m |= (uint32_t)(below.code(j) == 6) << 1;
    m |= (uint32_t)(below.right(j) == 5) << 2;
    m |= (uint32_t)(here.left(j) == 4) << 3;
    m |= (uint32_t)(here.right(j) == 3) << 4;
  }
  m |= (uint32_t)(above.left(j) == 2 && (top || k == 0)) << 5;
  m |= (uint32_t)(above.code(j) == 1 && top) << 6;
  m |= (uint32_t)(above.right(j) == 0 && (top || k == tw - 1)) << 7;
  return k < tw ? m : 0u;
}

// Can a same-row (codes 3, 4 in `here`) or towards-higher-row (codes 5, 6, 7
// in `below`) donor exist anywhere in this wavefront's row?  Uniform.
__device__ __forceinline__ bool rare_donors(const Row& here, const Row& below) {
  bool any = false;
#pragma unroll
  for (int j = 0; j < W; ++j) {
    const uint32_t h = here.code(j), b = below.code(j);
    any |= (h == 3 || h == 4) || (b >= 5 && b <= 7);
  }
  any |= here.l == 4 || here.r == 3 || below.l == 7 || below.r == 5;
  return __ballot(any) != 0;
}

// Unused slots at the end of a wavefront's last exit chunk are holes
// (ex_cell = NONE) that the forest skips.

__device__ __forceinline__ void exit_holes(const D8Params& P, uint32_t from, uint32_t to, int lane) {
  for (uint32_t h = from + (uint32_t)lane; h < to; h += 64)
    if (h < P.cap) P.ex_cell[h] = NONE;
}


// ---------------------------------------------------------------------------
// 128-bit fixed point for the exit forest.  A value x is held as the integer
// floor(x / 2^E) (two's complement), E = e_max + ceil(log2(n + 1)) + 2 - 126
// with every exit's local sum below 2^e_max in magnitude, so no sum of the n
// exits' values reaches 2^124 units.  Bits below one unit (2^E, at most
// 2^-124 of the largest possible total) are dropped from each term, the
// same way in every run.
using u128 = unsigned __int128;
using i128 = __int128;

__device__ __forceinline__ int ceil_log2_p1(uint32_t n) { return n == 0 ? 0 : 32 - __clz((int)n); }

// The tile path's exit totals: one 16-byte record per exit (the total's
// bits -- float-float hi | lo << 32, or float64 -- then the count) in the
// third fixed-point buffer, which the work-queue forest leaves unused.
__device__ __forceinline__ unsigned __int128* tile_total_rec(const D8Params& P, uint32_t i) { return P.ex_fx[2] + i; }

template <int VK>
__device__ __forceinline__ int fx_exponent(const D8Params& P, uint32_t n) {
  int e = 0;
  if (VK == VK_FF) {
    const float m = __uint_as_float(P.ctl->loc_max_f);
    if (m > 0.0f && isfinite(m)) (void)frexpf(m, &e);  // m < 2^e
  } else {
    const double m = __longlong_as_double((long long)P.ctl->loc_max_d);
    if (m > 0.0 && isfinite(m)) (void)frexp(m, &e);
  }
  return e + ceil_log2_p1(n) + 2 - 126;
}

// m * 2^sh units, floored.  By the choice of E, sh <= 100 for a float32
// term (|m| < 2^24) and sh <= 71 for a float64 term (|m| < 2^53).
__device__ __forceinline__ i128 fx_scale(int64_t m, int sh) {
  if (sh >= 0) return sh <= 100 ? (i128)((u128)(i128)m << sh) : (i128)0;
  return sh > -64 ? (i128)(m >> (-sh)) : (i128)(m < 0 ? -1 : 0);
}

__device__ __forceinline__ i128 fx_from(float x, int E) {
  if (!(x != 0.0f) || !isfinite(x)) return 0;  // non-finite input is reported elsewhere
  int e = 0;
  const float f = frexpf(x, &e);                 // x = f 2^e, 1/2 <= |f| < 1
  return fx_scale((int64_t)(f * 16777216.0f), e - 24 - E);
}

__device__ __forceinline__ i128 fx_from(double x, int E) {
  if (!(x != 0.0) || !isfinite(x)) return 0;
  int e = 0;
  const double f = frexp(x, &e);
  return fx_scale((int64_t)(f * 9007199254740992.0), e - 53 - E);
}

__device__ __forceinline__ int top_bit(u128 u) {
  const uint64_t h = (uint64_t)(u >> 64), l = (uint64_t)u;
  return h ? 127 - __clzll((long long)h) : 63 - __clzll((long long)l);
}

// The leading `bits` bits of u (u != 0) as an integer m and its exponent s:
// u = m 2^s + rest, 0 <= rest < 2^s.
__device__ __forceinline__ uint64_t fx_lead(u128 u, int bits, int* s, u128* rest) {
  const int sh = top_bit(u) - (bits - 1);
  *s = sh;
  if (sh <= 0) {
    *rest = 0;
    return (uint64_t)(u << (-sh));
  }
  const uint64_t m = (uint64_t)(u >> sh);
  *rest = u - ((u128)m << sh);
  return m;
}

// Back to float-float: the leading 24 bits, then the next 24 (truncated:
// relative error below 2^-47).
__device__ __forceinline__ ff fx_to_ff(i128 v, int E) {
  if (v == 0) return {0.0f, 0.0f};
  const bool neg = v < 0;
  const u128 u = neg ? (u128)0 - (u128)v : (u128)v;
  int s1 = 0, s2 = 0;
  u128 r1 = 0, r2 = 0;
  const uint64_t m1 = fx_lead(u, 24, &s1, &r1);
  float hi = ldexpf((float)m1, s1 + E), lo = 0.0f;
  if (r1 != 0) lo = ldexpf((float)fx_lead(r1, 24, &s2, &r2), s2 + E);
  if (neg) {
    hi = -hi;
    lo = -lo;
  }
  return ff_fast(hi, lo);
}

__device__ __forceinline__ double fx_to_double(i128 v, int E) {
  if (v == 0) return 0.0;
  const bool neg = v < 0;
  const u128 u = neg ? (u128)0 - (u128)v : (u128)v;
  int s1 = 0, s2 = 0;
  u128 r1 = 0, r2 = 0;
  const uint64_t m1 = fx_lead(u, 53, &s1, &r1);
  double d = ldexp((double)m1, s1 + E);
  if (r1 != 0) d += ldexp((double)fx_lead(r1, 53, &s2, &r2), s2 + E);
  return neg ? -d : d;
}

// Exact 128-bit atomic addition from two 64-bit ones: the low word's
// carries reach the high word once each, whatever the interleaving.
__device__ __forceinline__ void atomic_add_fx(u128* p, u128 x) {
  unsigned long long* w = reinterpret_cast<unsigned long long*>(p);
  const unsigned long long xl = (unsigned long long)x, xh = (unsigned long long)(x >> 64);
  const unsigned long long old = atomicAdd(w, xl);
  const unsigned long long h = xh + ((old + xl < old) ? 1ull : 0ull);
  if (h) atomicAdd(w + 1, h);
}

// Rows and columns of the block of tiles holding tile T (block iterations).
struct Block {
  int64_t r0, r1, c0, c1;
};
__device__ __forceinline__ Block block_of(const D8Params& P, const Tile& T) {
  const int64_t bh = (int64_t)P.th * P.bt_r, bw = (int64_t)TW * P.bt_c;
  Block B;
  B.r0 = (T.r0 / bh) * bh;
  B.r1 = B.r0 + bh;
  B.c0 = (T.c0 / bw) * bw;
  B.c1 = B.c0 + bw;
  return B;
}
__device__ __forceinline__ bool in_block(const Block& B, int64_t r, int64_t c) {
  return r >= B.r0 && r < B.r1 && c >= B.c0 && c < B.c1;
}

// Value carried down a sweep: float-float water, float64 water, count.
template <typename CT>
struct Val {
  ff f;
  double d;
  CT n;
};

// s + (cond ? x : 0), float-float with one renormalisation per call site.
__device__ __forceinline__ void acc_ff(float& s, float& e, bool cond, float xh, float xl) {
  xh = cond ? xh : 0.0f;
  xl = cond ? xl : 0.0f;
  const ff t = ff_two_sum(s, xh);
  s = t.hi;
  e += t.lo + xl;
}

// What a sweep hands back besides its stores.
struct SweepOut {
  double mass[2] = {0.0, 0.0};  // phase C: {sum over sinks, sum of rain} of the lane's cells
  float lmax_f = 0.0f;          // phase A: largest |local sum| of the lane's exits
  double lmax_d = 0.0;
  bool nonfinite = false, badcode = false, changed = false;
};

// Top-down sweep over the tile (rows r0+th-1 .. r0), one wavefront, W
// columns per lane.  A cell's value is its rain, plus (phase C) the totals of
// its cut donors, plus the values of its donors in the row above inside the
// tile, which the previous step left in registers.  Codes and rain stream
// through a ring of registers PF rows ahead; no LDS.
//   UP   (phase A): record every exit with its local value (local counts of
//                   one tile fit in 32 bits).
//   DOWN (phase C): write the final water / counts and the mass balance.
//   ITER (block iterations): donors in other blocks give their water of the
//                   previous iterate (both phases); the forest covers only
//                   cut donors inside the block; the new iterate is compared
//                   with the previous one.
template <bool UP, int VK, bool CNT, int RAIN, bool VEC, bool BORDER, bool ITER>
__device__ __forceinline__ void sweep(const D8Params& P, const Tile& T, SweepOut& out, float* xq32 = nullptr,
                                      double* xq64 = nullptr, uint64_t* xcnt = nullptr) {
  using CT = typename std::conditional<UP, uint32_t, uint64_t>::type;
  using V = Val<CT>;
  // Rows in flight: fewer in phase A, whose kernel must stay within 128
  // VGPRs for four wavefronts per SIMD.
  constexpr int PF = !VEC ? 4 : (UP ? 6 : PF_ROWS);
  const int lane = threadIdx.x & 63;
  const int k0 = W * lane;  // first tile column of this lane
  const int c = T.c0 + k0;
  const int nc = (int)P.ncols;
  const int rtop = T.r0 + T.th - 1;
  const int tw = BORDER ? T.tw : TW;
  const bool lane_in = !BORDER || c < nc;
  // Phase C reads the forest's totals (of n_ex exits).
  const uint32_t n_ex = UP ? 0u : min(*P.n_exits, P.cap);
  Block B{};
  if (ITER) B = block_of(P, T);
  const bool nosrc = ITER && P.it_nosrc;
  const bool prev = ITER && !P.it_first;
  double m_sink = 0.0, m_rain = 0.0;
  bool nf = false, bad = false, chg = false;
  float lmf = 0.0f;
  double lmd = 0.0;
  V pv[W];
#pragma unroll
  for (int j = 0; j < W; ++j) pv[j] = V{};
  uint32_t ex_base = 0, ex_used = 0, ex_size = 0;  // the wavefront's exit chunk (uniform)
  Row above = expand_row<BORDER, VEC>(load_codes<VEC>(P, T, rtop + 1, lane), P, T, rtop + 1, lane);
  Row here = expand_row<BORDER, VEC>(load_codes<VEC>(P, T, rtop, lane), P, T, rtop, lane);
  // Slot i of the ring holds, for step s = i (mod PF): the codes of row
  // rtop - s - 1 (the row below) and the rain of row rtop - s.
  CodeIn cq[PF];
  RainIn<RAIN, VEC> rq[PF];
#pragma unroll
  for (int i = 0; i < PF; ++i) {
    cq[i] = load_codes<VEC>(P, T, rtop - i - 1, lane);
    rq[i] = load_rain<RAIN, VEC>(P, T, rtop - i, lane);
  }
  for (int s0 = 0; s0 < T.th; s0 += PF) {
#pragma unroll
    for (int i = 0; i < PF; ++i) {
      const int s = s0 + i;
      const int r = rtop - s;
      if (s < T.th) {  // uniform
        const Row below = expand_row<BORDER, VEC>(cq[i], P, T, r - 1, lane);
        const size_t g = (size_t)r * (size_t)nc + (size_t)c;
        const bool top = s == 0;
        const bool bottom = r == T.r0;
        const bool rare = (!UP || ITER) && rare_donors(here, below);
        // Values of the row above at the columns left and right of this lane.
        V lv, rv;
        if (VK == VK_FF) {
          lv.f = {from_left(pv[W - 1].f.hi), from_left(pv[W - 1].f.lo)};
          rv.f = {from_right(pv[0].f.hi), from_right(pv[0].f.lo)};
        }
        if (VK == VK_F64) {
          lv.d = from_left(pv[W - 1].d);
          rv.d = from_right(pv[0].d);
        }
        if (CNT) {
          lv.n = from_left(pv[W - 1].n);
          rv.n = from_right(pv[0].n);
        }
        V nv[W];
        bool exits[W], sinks[W];
        uint32_t cut[W];
#pragma unroll
        for (int j = 0; j < W; ++j) {
          const int k = k0 + j;
          const uint32_t cd = here.code(j);
          const Cell x = classify<BORDER>(P, T, r, k, cd, bottom);
          exits[j] = x.exit;
          sinks[j] = x.sink;
          const bool d5 = !top && k > 0 && above.left(j) == 2;
          const bool d6 = !top && above.code(j) == 1;
          const bool d7 = !top && k + 1 < tw && above.right(j) == 0;
          const V& a5 = j == 0 ? lv : pv[j == 0 ? 0 : j - 1];
          const V& a7 = j == W - 1 ? rv : pv[j == W - 1 ? 0 : j + 1];
          const auto rain = rq[i].v[j];
          if ((UP || ITER) && RAIN != RAIN_UNIT) nf |= !isfinite(rain);
          if (ITER && !UP) bad |= (!BORDER || k < tw) && cd != SINK && x.sink;
          V v;
          if (VK == VK_FF) {
            float sh = (float)rain, se = RAIN == RAIN_F64 ? (float)((double)rain - (double)(float)rain) : 0.0f;
            acc_ff(sh, se, d5, a5.f.hi, a5.f.lo);
            acc_ff(sh, se, d6, pv[j].f.hi, pv[j].f.lo);
            acc_ff(sh, se, d7, a7.f.hi, a7.f.lo);
            v.f = ff_fast(sh, se);
          }
          if (VK == VK_F64)
            v.d = (nosrc ? 0.0 : (double)rain) + (d5 ? a5.d : 0.0) + (d6 ? pv[j].d : 0.0) + (d7 ? a7.d : 0.0);
          if (CNT)
            v.n = (CT)(nosrc ? 0 : 1) + (d5 ? a5.n : (CT)0) + (d6 ? pv[j].n : (CT)0) + (d7 ? a7.n : (CT)0);
          cut[j] = (UP && !ITER) ? 0u : cut_donors(above, here, below, j, k, top, rare, tw);
          nv[j] = v;
        }
        if ((!UP || ITER) && __ballot((cut[0] | cut[1] | cut[2] | cut[3]) != 0u)) {
          // Donors across cut edges (sparse: the top row, the outer columns
          // and rare rows): the forest total of a donor inside the block
          // (phase C), the previous iterate of a donor in another block.
#pragma unroll
          for (int j = 0; j < W; ++j) {
            uint32_t m = cut[j];
            while (m) {
              const int n = __builtin_ctz(m);
              m &= m - 1;
              const size_t gj = (size_t)((int64_t)(g + j) + (int64_t)nb_dr(n) * nc + nb_dc(n));
              const bool other = ITER && !in_block(B, r + nb_dr(n), c + j + nb_dc(n));
              if (other) {
                if (prev) {
                  if (VK == VK_F64) nv[j].d += P.it_q64[gj];
                  if (CNT) nv[j].n += (CT)P.it_cnt[gj];
                }
                continue;
              }
              if (UP) continue;  // phase A: the forest adds donors inside the block
              const uint32_t nd = P.node_of[gj];
              if (nd >= n_ex) {  // inconsistent bookkeeping: never follow it
                set_status(P.status, FR_ERR_BADCODE);
                continue;
              }
              if (VK == VK_FF) nv[j].f = ff_add(nv[j].f, ff{P.tot_hi[nd], P.tot_lo[nd]});
              if (VK == VK_F64) nv[j].d += P.tot_d[nd];
              if (CNT) nv[j].n += (CT)P.ex_cnt[0][nd];
            }
          }
        }
        if (UP && __ballot(exits[0] || exits[1] || exits[2] || exits[3])) {
          // Record exits in consecutive slots of the wavefront's chunk; a
          // new chunk (one atomic) when the row does not fit, the rest of
          // the old one left as holes.
          uint64_t em[W];
          uint32_t ne = 0;
#pragma unroll
          for (int j = 0; j < W; ++j) {
            em[j] = __ballot(exits[j]);
            ne += (uint32_t)__popcll(em[j]);
          }
          // The row's exits fill the rest of the current chunk first; the
          // others go to a new chunk (one atomic, at least D8_EXIT_CHUNK
          // slots), so only a wavefront's last chunk leaves holes.
          const uint32_t avail = ex_size - ex_used;  // uniform
          const uint32_t first = ex_base + ex_used;
          uint32_t nb = 0, want = 0;
          if (ne > avail) {
            want = ne - avail > D8_EXIT_CHUNK ? ne - avail : D8_EXIT_CHUNK;
            if (lane == 0) nb = atomicAdd(P.n_exits, want);
            nb = __shfl(nb, 0, 64);
          }
          const uint64_t lower = lane == 0 ? 0ull : (~0ull >> (64 - lane));
          uint32_t off = 0;  // exits of this row before column j, over all lanes
#pragma unroll
          for (int j = 0; j < W; ++j) {
            if (exits[j]) {
              const uint32_t t = off + (uint32_t)__popcll(em[j] & lower);
              const uint32_t idx = t < avail ? first + t : nb + (t - avail);
              if (idx < P.cap) {
                P.node_of[g + j] = idx;
                P.ex_cell[idx] = (uint32_t)(g + j);
                if (VK == VK_FF) {
                  P.ex_hi[idx] = nv[j].f.hi;
                  P.ex_lo[idx] = nv[j].f.lo;
                  lmf = fmaxf(lmf, fabsf(nv[j].f.hi));
                }
                if (VK == VK_F64) {
                  P.ex_d[idx] = nv[j].d;
                  lmd = fmax(lmd, fabs(nv[j].d));
                }
                if (CNT) P.ex_cnt[0][idx] = (uint64_t)nv[j].n;
              }
            }
            off += (uint32_t)__popcll(em[j]);
          }
          if (ne > avail) {
            ex_base = nb;
            ex_size = want;
            ex_used = ne - avail;
          } else {
            ex_used += ne;
          }
        }
        if (!UP && lane_in) {
          if (VEC) {
            if (VK == VK_FF) {
              float4 o;
              o.x = nv[0].f.hi + nv[0].f.lo;
              o.y = nv[1].f.hi + nv[1].f.lo;
              o.z = nv[2].f.hi + nv[2].f.lo;
              o.w = nv[3].f.hi + nv[3].f.lo;
              *reinterpret_cast<float4*>(P.q32 + g) = o;
            }
            if (VK == VK_F64) {
              *reinterpret_cast<double2*>(P.q64 + g) = make_double2(nv[0].d, nv[1].d);
              *reinterpret_cast<double2*>(P.q64 + g + 2) = make_double2(nv[2].d, nv[3].d);
            }
            if (CNT) {
              ulonglong2 a, b;
              a.x = nv[0].n;
              a.y = nv[1].n;
              b.x = nv[2].n;
              b.y = nv[3].n;
              *reinterpret_cast<ulonglong2*>(P.cnt + g) = a;
              *reinterpret_cast<ulonglong2*>(P.cnt + g + 2) = b;
            }
          }
        }
        if (!UP && !VEC) {
          // Rows not aligned to 4 cells: exchange the row through LDS so
          // that each store instruction writes 64 consecutive cells.
          const size_t g0 = (size_t)r * (size_t)nc + (size_t)T.c0;
#pragma unroll
          for (int j = 0; j < W; ++j) {
            if (VK == VK_FF) xq32[k0 + j] = nv[j].f.hi + nv[j].f.lo;
            if (VK == VK_F64) xq64[k0 + j] = nv[j].d;
            if (CNT) xcnt[k0 + j] = nv[j].n;
          }
          __syncthreads();
#pragma unroll
          for (int j = 0; j < W; ++j) {
            const int kk = 64 * j + lane;
            if (!BORDER || T.c0 + kk < nc) {
              if (VK == VK_FF) P.q32[g0 + kk] = xq32[kk];
              if (VK == VK_F64) P.q64[g0 + kk] = xq64[kk];
              if (CNT) P.cnt[g0 + kk] = xcnt[kk];
            }
          }
          __syncthreads();
        }
        if (ITER && !UP && prev && P.it_detect) {
          // Whether this iterate differs from the previous one here.
#pragma unroll
          for (int j = 0; j < W; ++j) {
            if (BORDER && c + j >= nc) continue;
            if (CNT) chg |= nv[j].n != P.it_cnt[g + j];
            else if (VK == VK_F64) chg |= __double_as_longlong(nv[j].d) != __double_as_longlong(P.it_q64[g + j]);
          }
        }
        if (!UP && !ITER && VK != VK_NONE) {
#pragma unroll
          for (int j = 0; j < W; ++j)
            if (!BORDER || c + j < nc) m_rain += (double)rq[i].v[j];
          if (__ballot(sinks[0] || sinks[1] || sinks[2] || sinks[3])) {
#pragma unroll
            for (int j = 0; j < W; ++j) {
              if (sinks[j] && (!BORDER || c + j < nc))
                m_sink += VK == VK_FF ? (double)nv[j].f.hi + (double)nv[j].f.lo : nv[j].d;
            }
          }
        }
#pragma unroll
        for (int j = 0; j < W; ++j) pv[j] = nv[j];
        above = here;
        here = below;
      }
      // Refill the slot for step s + PF.
      cq[i] = load_codes<VEC>(P, T, r - PF - 1, lane);
      rq[i] = load_rain<RAIN, VEC>(P, T, r - PF, lane);
    }
  }
  if (UP) exit_holes(P, ex_base + ex_used, ex_base + ex_size, lane);
  out.nonfinite |= nf;
  out.badcode |= bad;
  out.changed |= chg;
  out.mass[0] = m_sink;
  out.mass[1] = m_rain;
  out.lmax_f = lmf;
  out.lmax_d = lmd;
}

// Bottom-up sweep (rows r0 .. r0+th-1): the root of every inlet -- the exit
// or sink where its path through the tile ends.
template <bool VEC, bool BORDER>
__device__ __forceinline__ void root_sweep(const D8Params& P, const Tile& T, bool* badcode) {
  const int lane = threadIdx.x & 63;
  const int k0 = W * lane;
  const int nc = (int)P.ncols;
  const int tw = BORDER ? T.tw : TW;
  Row below = expand_row<BORDER, VEC>(load_codes<VEC>(P, T, T.r0 - 1, lane), P, T, T.r0 - 1, lane);
  Row here = expand_row<BORDER, VEC>(load_codes<VEC>(P, T, T.r0, lane), P, T, T.r0, lane);
  uint32_t rp[W];  // roots of the row below
#pragma unroll
  for (int j = 0; j < W; ++j) rp[j] = NONE;
  bool bad = false;
  // Slot i holds, for step s = i (mod PF_ROWS), the codes of row r0 + s + 1.
  CodeIn cq[PF_ROWS];
#pragma unroll
  for (int i = 0; i < PF_ROWS; ++i) cq[i] = load_codes<VEC>(P, T, T.r0 + i + 1, lane);
  for (int s0 = 0; s0 < T.th; s0 += PF_ROWS) {
#pragma unroll
    for (int i = 0; i < PF_ROWS; ++i) {
      const int s = s0 + i;
      const int r = T.r0 + s;
      if (s < T.th) {  // uniform
        const Row above = expand_row<BORDER, VEC>(cq[i], P, T, r + 1, lane);
        const bool top = s == T.th - 1;
        const bool bottom = s == 0;
        const bool rare = rare_donors(here, below);
        const uint32_t left = from_left(rp[W - 1], NONE), right = from_right(rp[0], NONE);
        const uint32_t base = (uint32_t)((size_t)r * (size_t)nc + (size_t)(T.c0 + k0));
        uint32_t nr[W];
        bool inlet[W];
#pragma unroll
        for (int j = 0; j < W; ++j) {
          const int k = k0 + j;
          const uint32_t cd = here.code(j);
          const Cell x = classify<BORDER>(P, T, r, k, cd, bottom);
          if (BORDER) bad |= k < tw && cd != SINK && x.sink;
          else bad |= cd > 7u && cd != SINK;
          const uint32_t rl = j == 0 ? left : rp[j == 0 ? 0 : j - 1];
          const uint32_t rr = j == W - 1 ? right : rp[j == W - 1 ? 0 : j + 1];
          nr[j] = x.down ? (cd == 0u ? rl : (cd == 1u ? rp[j] : rr)) : base + j;
          // Inlets: the top row, the two outer columns, and rows where a
          // same-row / towards-higher-row donor exists.
          inlet[j] = (top || rare || k == 0 || k == tw - 1) && cut_donors(above, here, below, j, k, top, rare, tw);
        }
        if (__ballot(inlet[0] || inlet[1] || inlet[2] || inlet[3])) {
#pragma unroll
          for (int j = 0; j < W; ++j)
            if (inlet[j]) P.root_of[base + j] = nr[j];
        }
#pragma unroll
        for (int j = 0; j < W; ++j) rp[j] = nr[j];
        below = here;
        here = above;
      }
      cq[i] = load_codes<VEC>(P, T, r + PF_ROWS + 1, lane);
    }
  }
  if (bad) *badcode = true;
}

// May a same-row or towards-higher-row donor exist in this wavefront's row?
// As rare_donors, from one bit per code value: bit (code & 31) of a lane's
// four codes.  Malformed codes may alias a donor code and answer "yes",
// which only sends the row through the general donor test.
__device__ __forceinline__ bool rare_donors_bits(const Row& here, const Row& below) {
  uint32_t hb = 0, bb = 0;
#pragma unroll
  for (int j = 0; j < W; ++j) {
    hb |= 1u << ((here.w >> (8 * j)) & 31u);
    bb |= 1u << ((below.w >> (8 * j)) & 31u);
  }
  const bool any = ((hb & 0x18u) | (bb & 0xE0u)) != 0u || here.l == 4u || here.r == 3u || below.l == 7u ||
                   below.r == 5u;
  return __ballot(any) != 0;
}

// root_sweep for a tile away from the grid border, with the per-cell logic
// in straight-line integer form: a cell's root is its receiver's root when
// the receiver is in the row below inside the tile, else the cell itself.
// Outside rows with a rare donor and the tile's top row, only the two outer
// columns can be inlets (water across the tile's side edges).
template <bool VEC>
__device__ __forceinline__ void root_sweep_interior(const D8Params& P, const Tile& T, bool* badcode) {
  const int lane = threadIdx.x & 63;
  const int k0 = W * lane;
  const int nc = (int)P.ncols;
  Row below = expand_row<false, VEC>(load_codes<VEC>(P, T, T.r0 - 1, lane), P, T, T.r0 - 1, lane);
  Row here = expand_row<false, VEC>(load_codes<VEC>(P, T, T.r0, lane), P, T, T.r0, lane);
  uint32_t rp[W];  // roots of the row below
#pragma unroll
  for (int j = 0; j < W; ++j) rp[j] = NONE;
  uint32_t bad = 0;
  CodeIn cq[PF_ROWS];
#pragma unroll
  for (int i = 0; i < PF_ROWS; ++i) cq[i] = load_codes<VEC>(P, T, T.r0 + i + 1, lane);
  for (int s0 = 0; s0 < T.th; s0 += PF_ROWS) {
#pragma unroll
    for (int i = 0; i < PF_ROWS; ++i) {
      const int s = s0 + i;
      const int r = T.r0 + s;
      if (s < T.th) {  // uniform
        const Row above = expand_row<false, VEC>(cq[i], P, T, r + 1, lane);
        const bool top = s == T.th - 1;
        const bool bottom = s == 0;
        const uint32_t base = (uint32_t)((size_t)r * (size_t)nc + (size_t)(T.c0 + k0));
        // A code 0 in column 0 or 2 in column TW - 1 leaves the tile: the
        // cell is its own root, as the DPP edge values say.
        const uint32_t left = from_left(rp[W - 1], base), right = from_right(rp[0], base + (W - 1));
        uint32_t nr[W];
#pragma unroll
        for (int j = 0; j < W; ++j) {
          const uint32_t cd = here.code(j);
          bad |= (uint32_t)(((cd + 1u) & 0xFFu) > 8u);  // neither 0..7 nor the sink code
          const uint32_t rl = j == 0 ? left : rp[j == 0 ? 0 : j - 1];
          const uint32_t rr = j == W - 1 ? right : rp[j == W - 1 ? 0 : j + 1];
          uint32_t v = base + j;
          v = cd == 0u ? rl : v;
          v = cd == 1u ? rp[j] : v;
          v = cd == 2u ? rr : v;
          nr[j] = bottom ? base + j : v;
        }
        if (top || rare_donors_bits(here, below)) {  // uniform
          bool inlet[W];
#pragma unroll
          for (int j = 0; j < W; ++j) inlet[j] = cut_donors(above, here, below, j, k0 + j, top, true, TW) != 0u;
          if (__ballot(inlet[0] || inlet[1] || inlet[2] || inlet[3])) {
#pragma unroll
            for (int j = 0; j < W; ++j)
              if (inlet[j]) P.root_of[base + j] = nr[j];
          }
        } else {
          if (lane == 0 && above.l == 2u) P.root_of[base] = nr[0];
          if (lane == 63 && above.r == 0u) P.root_of[base + W - 1] = nr[W - 1];
        }
#pragma unroll
        for (int j = 0; j < W; ++j) rp[j] = nr[j];
        below = here;
        here = above;
      }
      cq[i] = load_codes<VEC>(P, T, r + PF_ROWS + 1, lane);
    }
  }
  if (bad) *badcode = true;
}



}  // namespace

// Launches a phase A / phase C kernel for the value kind, the rain source
// and the row alignment of the grid (float4 / dword row loads when
// ncols % 4 == 0).
template <template <int, bool, int, bool, bool> class K, int VK, bool CNT, bool ITER>
void d8_sweep_launch(const D8Params& P, hipStream_t s) {
  const bool vec = (P.ncols % 4) == 0;
  const int rain = P.rain64 ? RAIN_F64 : (P.rain32 ? RAIN_F32 : RAIN_UNIT);
  if constexpr (VK == VK_NONE) {
    if (vec) K<VK, CNT, RAIN_UNIT, true, ITER>::launch(P, s);
    else K<VK, CNT, RAIN_UNIT, false, ITER>::launch(P, s);
  } else {
    if (rain == RAIN_UNIT) {
      if (vec) K<VK, CNT, RAIN_UNIT, true, ITER>::launch(P, s);
      else K<VK, CNT, RAIN_UNIT, false, ITER>::launch(P, s);
    } else if (rain == RAIN_F32) {
      if (vec) K<VK, CNT, RAIN_F32, true, ITER>::launch(P, s);
      else K<VK, CNT, RAIN_F32, false, ITER>::launch(P, s);
    } else {
      if (vec) K<VK, CNT, RAIN_F64, true, ITER>::launch(P, s);
      else K<VK, CNT, RAIN_F64, false, ITER>::launch(P, s);
    }
  }
}

template <template <int, bool, int, bool, bool> class K>
hipError_t d8_sweep_dispatch(ValKind vk, bool cnt, bool iter, const D8Params& P, hipStream_t s) {
  if (iter) {
    // Block iterations: float64 water and/or counts.
    if (vk == VK_FF) return hipErrorInvalidValue;
    if (vk == VK_F64) {
      if (cnt) d8_sweep_launch<K, VK_F64, true, true>(P, s);
      else d8_sweep_launch<K, VK_F64, false, true>(P, s);
    } else {
      d8_sweep_launch<K, VK_NONE, true, true>(P, s);
    }
  } else if (vk == VK_FF) {
    if (cnt) d8_sweep_launch<K, VK_FF, true, false>(P, s);
    else d8_sweep_launch<K, VK_FF, false, false>(P, s);
  } else if (vk == VK_F64) {
    if (cnt) d8_sweep_launch<K, VK_F64, true, false>(P, s);
    else d8_sweep_launch<K, VK_F64, false, false>(P, s);
  } else {
    d8_sweep_launch<K, VK_NONE, true, false>(P, s);
  }
  return hipGetLastError();
}

}  // namespace fr
