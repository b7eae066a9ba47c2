// Single-receiver (D8 / D4) accumulation by row sweeps plus a reduced exit
// forest.
//
// The water at a cell is its rain plus the water of every cell upstream of it
// (Section 2.1; the unique solution of (I - W^T) q = r, Section 2.2).  On
// tilted terrain nearly every receiver lies in the previous row (row - 1), so
// a sweep over the rows in decreasing index order visits donors before
// receivers -- it is the paper's high-to-low order restricted to that edge
// class, and like the paper's per-process solves (Section 2.4, Section 3.3)
// the grid is cut into blocks whose solves are independent:
//
//   A. Each tile (th rows x 256 columns) is swept by one wavefront, four
//      columns per lane.  Edges from row r+1 to row r inside the tile are
//      followed in registers (cross-lane shifts); every other edge --
//      leaving the tile, within a row, or toward a higher row index -- is
//      "cut".  A top-down sweep yields each cut cell's (exit's) local
//      upstream sum; a bottom-up sweep (its own kernel) yields, for every
//      cell that receives over a cut edge (inlet), the exit or sink where its
//      in-tile path ends (its root).
//   B. The exits form a forest: exit e drains into exit root(receiver(e)),
//      or nowhere when that root is a sink.  Subtree sums over this forest are
//      computed by pointer doubling in ceil(log2(depth)) rounds.  These stand
//      in for the paper's C + 1 block iterations across block boundaries
//      (Section 3.3, Appendix B), collapsed to a logarithmic number of rounds.
//   C. Each tile is swept again with the totals of its cut donors added: the
//      result is final.  The float64 mass balance is reduced in the same pass.
//
// The same top-down sweep, fed the previous iterate's water across cut edges
// instead of forest totals, is one of the paper's block iterations (k_d8_iter).
//
// Numerics: float32 water uses float-float (hi, lo) sums throughout; the
// exit forest adds hi with float atomics and folds each addition's exact
// rounding error into lo.  Counts are exact uint64.
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

// Exit-list slots reserved per atomic in phase A; unused slots of a chunk
// are holes (ex_cell = NONE) that the forest skips.
constexpr uint32_t EXIT_CHUNK = 32;

__device__ __forceinline__ void exit_holes(const D8Params& P, uint32_t from, uint32_t to, int lane) {
  for (uint32_t h = from + (uint32_t)lane; h < to; h += 64)
    if (h < P.cap) P.ex_cell[h] = NONE;
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

// Top-down sweep over the tile (rows r0+th-1 .. r0), one wavefront, W
// columns per lane.  A cell's value is its rain, plus (phase C) the totals of
// its cut donors, plus the values of its donors in the row above inside the
// tile, which the previous step left in registers.  Codes and rain stream
// through a ring of registers PF rows ahead; no LDS.
//   UP   (phase A): record every exit with its local value (local counts of
//                   one tile fit in 32 bits).
//   DOWN (phase C): write the final water / counts and the mass balance.
//   ITER (block iterations, phase C form): cut donors give their water of
//                   the previous iterate; the tile sweep is the block solve.
template <bool UP, int VK, bool CNT, int RAIN, bool VEC, bool BORDER, bool ITER = false>
__device__ __forceinline__ void sweep(const D8Params& P, const Tile& T, double* mass, bool* nonfinite,
                                      float* xq32 = nullptr, double* xq64 = nullptr, uint64_t* xcnt = nullptr,
                                      bool* badcode = nullptr, bool* changed = nullptr) {
  using CT = typename std::conditional<UP, uint32_t, uint64_t>::type;
  using V = Val<CT>;
  // Rows in flight: fewer in phase A, whose kernel must stay within 128
  // VGPRs for four wavefronts per SIMD.
  constexpr int PF = !VEC ? 4 : (UP ? 6 : PF_ROWS);
  const int lane = threadIdx.x;
  const int k0 = W * lane;  // first tile column of this lane
  const int c = T.c0 + k0;
  const int nc = (int)P.ncols;
  const int rtop = T.r0 + T.th - 1;
  const int tw = BORDER ? T.tw : TW;
  const bool lane_in = !BORDER || c < nc;
  double m_sink = 0.0, m_rain = 0.0;
  bool nf = false, bad = false, chg = false;
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
        const bool rare = !UP && rare_donors(here, below);
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
          if (ITER) bad |= (!BORDER || k < tw) && cd != SINK && x.sink;
          V v;
          if (VK == VK_FF) {
            float sh = (float)rain, se = RAIN == RAIN_F64 ? (float)((double)rain - (double)(float)rain) : 0.0f;
            acc_ff(sh, se, d5, a5.f.hi, a5.f.lo);
            acc_ff(sh, se, d6, pv[j].f.hi, pv[j].f.lo);
            acc_ff(sh, se, d7, a7.f.hi, a7.f.lo);
            v.f = ff_fast(sh, se);
          }
          const bool nosrc = ITER && P.it_nosrc;
          if (VK == VK_F64)
            v.d = (nosrc ? 0.0 : (double)rain) + (d5 ? a5.d : 0.0) + (d6 ? pv[j].d : 0.0) + (d7 ? a7.d : 0.0);
          if (CNT)
            v.n = (CT)(nosrc ? 0 : 1) + (d5 ? a5.n : (CT)0) + (d6 ? pv[j].n : (CT)0) + (d7 ? a7.n : (CT)0);
          cut[j] = UP ? 0u : cut_donors(above, here, below, j, k, top, rare, tw);
          nv[j] = v;
        }
        if (ITER && !P.it_first && __ballot((cut[0] | cut[1] | cut[2] | cut[3]) != 0u)) {
          // Water of the previous iterate across cut edges.
#pragma unroll
          for (int j = 0; j < W; ++j) {
            uint32_t m = cut[j];
            while (m) {
              const int n = __builtin_ctz(m);
              m &= m - 1;
              const size_t gj = (size_t)((int64_t)(g + j) + (int64_t)nb_dr(n) * nc + nb_dc(n));
              if (VK == VK_F64) nv[j].d += P.it_q64[gj];
              if (CNT) nv[j].n += (CT)P.it_cnt[gj];
            }
          }
        }
        if (!UP && !ITER && __ballot((cut[0] | cut[1] | cut[2] | cut[3]) != 0u)) {
          // Totals of donors across cut edges (sparse: the top row, the
          // outer columns and rare rows).
#pragma unroll
          for (int j = 0; j < W; ++j) {
            uint32_t m = cut[j];
            while (m) {
              const int n = __builtin_ctz(m);
              m &= m - 1;
              const size_t gj = (size_t)((int64_t)(g + j) + (int64_t)nb_dr(n) * nc + nb_dc(n));
              const uint32_t nd = P.node_of[gj];
              if (nd >= P.n_ex) {  // inconsistent bookkeeping: never follow it
                set_status(P.status, FR_ERR_BADCODE);
                continue;
              }
              if (VK == VK_FF) nv[j].f = ff_add(nv[j].f, ff{P.ex_hi[0][nd], P.ex_lo[0][nd]});
              if (VK == VK_F64) nv[j].d += P.ex_q64[0][nd];
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
          if (ex_used + ne > ex_size) {  // uniform
            exit_holes(P, ex_base + ex_used, ex_base + ex_size, lane);
            const uint32_t want = ne > EXIT_CHUNK ? ne : EXIT_CHUNK;
            uint32_t nb = 0;
            if (lane == 0) nb = atomicAdd(P.n_exits, want);
            ex_base = __shfl(nb, 0, 64);
            ex_size = want;
            ex_used = 0;
          }
          const uint64_t lower = lane == 0 ? 0ull : (~0ull >> (64 - lane));
          uint32_t off = ex_base + ex_used;
          ex_used += ne;
#pragma unroll
          for (int j = 0; j < W; ++j) {
            const bool ex = exits[j];
            {
              if (ex) {
                const uint32_t idx = off + (uint32_t)__popcll(em[j] & lower);
                if (idx < P.cap) {
                  P.node_of[g + j] = idx;
                  P.ex_cell[idx] = (uint32_t)(g + j);
                  if (VK == VK_FF) {
                    P.ex_hi[0][idx] = nv[j].f.hi;
                    P.ex_lo[0][idx] = nv[j].f.lo;
                  }
                  if (VK == VK_F64) P.ex_q64[0][idx] = nv[j].d;
                  if (CNT) P.ex_cnt[0][idx] = (uint64_t)nv[j].n;
                }
              }
            }
            off += (uint32_t)__popcll(em[j]);
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
        if (ITER && !P.it_first && P.it_detect) {
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
  if (nf) *nonfinite = true;
  if (ITER && bad) *badcode = true;
  if (ITER && chg) *changed = true;
  if (mass) {
    mass[0] = m_sink;
    mass[1] = m_rain;
  }
}

// Bottom-up sweep (rows r0 .. r0+th-1): the root of every inlet -- the exit
// or sink where its path through the tile ends.
template <bool VEC, bool BORDER>
__device__ __forceinline__ void root_sweep(const D8Params& P, const Tile& T, bool* badcode) {
  const int lane = threadIdx.x;
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
  const int lane = threadIdx.x;
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

// ---------------------------------------------------------------------------
// Phase A, as two independent kernels: the root sweep needs few registers
// and runs at high occupancy; the local sweep carries the values.
template <bool VEC>
__global__ __launch_bounds__(64) void k_d8_root(D8Params P) {
  const Tile T = tile_of(P, blockIdx.x);
  bool badcode = false;
  if (T.border) root_sweep<VEC, true>(P, T, &badcode);
  else root_sweep_interior<VEC>(P, T, &badcode);
  if (badcode) set_status(P.status, FR_ERR_BADCODE);
}

template <int VK, bool CNT, int RAIN, bool VEC>
__global__ __launch_bounds__(64) void k_d8_up(D8Params P) {
  const Tile T = tile_of(P, blockIdx.x);
  bool nonfinite = false;
  if (T.border) sweep<true, VK, CNT, RAIN, VEC, true>(P, T, nullptr, &nonfinite);
  else sweep<true, VK, CNT, RAIN, VEC, false>(P, T, nullptr, &nonfinite);
  if (nonfinite) set_status(P.status, FR_ERR_NONFINITE);
}

// ---------------------------------------------------------------------------
// Phase B: exit forest.
__global__ __launch_bounds__(256) void k_d8_link(D8Params P, uint32_t n) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const uint32_t ec = P.ex_cell[i];
    if (ec == NONE) {  // a hole of a phase-A chunk
      P.anc[0][i] = NONE;
      continue;
    }
    const int64_t e = ec;
    const int cd = P.code[e];
    const int64_t x = e + (int64_t)nb_dr(cd) * P.ncols + nb_dc(cd);
    const int64_t rt = P.root_of[x];
    uint32_t a = NONE;
    if (rt >= 0 && rt < P.nrows * P.ncols) {
      const int64_t rr = rt / P.ncols, rc = rt - rr * P.ncols;
      const int rcd = P.code[rt];
      bool sink = rcd > 7;
      if (!sink) {
        const int64_t tr = rr + nb_dr(rcd), tc = rc + nb_dc(rcd);
        sink = tr < 0 || tr >= P.nrows || tc < 0 || tc >= P.ncols;
      }
      if (!sink) {
        a = P.node_of[rt];
        if (a >= n) {  // inconsistent bookkeeping: never follow it
          a = NONE;
          set_status(P.status, FR_ERR_BADCODE);
        }
      }
    } else {
      set_status(P.status, FR_ERR_BADCODE);
    }
    P.anc[0][i] = a;
  }
}

// Round j sets flag slot j mod 3 when it leaves work for round j + 1, and
// skips itself when round j - 1 left none (so the host can queue rounds
// without waiting for each flag); round j's scatter clears slot j + 1.
__device__ __forceinline__ int32_t* round_flag(const D8Params& P, int j) { return &P.flags[4 + j % 3]; }
__device__ __forceinline__ bool round_idle(const D8Params& P, int j) {
  return j > 0 && __hip_atomic_load(round_flag(P, j + 2), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0;
}

// Round j of pointer doubling (anc[b] = ancestor 2^j exits down, or NONE).
// Part 1: every exit that still has such an ancestor snapshots its sum (the
// sum over its subtree within distance < 2^j) and jumps its pointer.
template <int VK, bool CNT>
__global__ __launch_bounds__(256) void k_d8_copy(D8Params P, uint32_t n, int b, int j) {
  if (round_idle(P, j)) return;  // uniform
  __shared__ int s_active;
  if (threadIdx.x == 0) s_active = 0;
  __syncthreads();
  bool active = false;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const uint32_t a = P.anc[b][i];
    uint32_t a2 = NONE;
    if (a != NONE) {
      if (VK == VK_FF) {
        P.ex_hi[1][i] = P.ex_hi[0][i];
        P.ex_lo[1][i] = P.ex_lo[0][i];
      }
      if (VK == VK_F64) P.ex_q64[1][i] = P.ex_q64[0][i];
      if (CNT) P.ex_cnt[1][i] = P.ex_cnt[0][i];
      a2 = P.anc[b][a];
    }
    P.anc[b ^ 1][i] = a2;
    active |= (a2 != NONE);
  }
  // One store per workgroup, and only while the flag is still clear: an
  // atomic from every wavefront on one word serialises the whole kernel.
  if (__ballot(active) && (threadIdx.x & 63) == 0) s_active = 1;
  __syncthreads();
  if (threadIdx.x == 0 && s_active &&
      __hip_atomic_load(round_flag(P, j), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0)
    __hip_atomic_store(round_flag(P, j), 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Part 2: each such exit adds its snapshot to the ancestor's sum in place.
template <int VK, bool CNT>
__global__ __launch_bounds__(256) void k_d8_scatter(D8Params P, uint32_t n, int b, int j) {
  if (blockIdx.x == 0 && threadIdx.x == 0)
    __hip_atomic_store(round_flag(P, j + 1), 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (round_idle(P, j)) return;  // uniform
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const uint32_t a = P.anc[b][i];
    if (a == NONE) continue;
    if (VK == VK_FF) {
      const float xh = P.ex_hi[1][i], xl = P.ex_lo[1][i];
      const float old = atomicAdd(&P.ex_hi[0][a], xh);
      const ff e = ff_two_sum(old, xh);  // e.hi is what the atomic stored
      atomicAdd(&P.ex_lo[0][a], e.lo + xl);
    }
    if (VK == VK_F64) atomicAdd(&P.ex_q64[0][a], P.ex_q64[1][i]);
    if (CNT) atomicAdd(reinterpret_cast<unsigned long long*>(&P.ex_cnt[0][a]),
                       (unsigned long long)P.ex_cnt[1][i]);
  }
}

// ---------------------------------------------------------------------------
// Phase C.
template <int VK, bool CNT, int RAIN, bool VEC>
__global__ __launch_bounds__(64) void k_d8_down(D8Params P) {
  __shared__ double s_mass[2][64];
  // Row exchange for grids whose rows are not aligned to 4 cells.
  __shared__ float s_q32[VEC || VK != VK_FF ? 1 : TW];
  __shared__ double s_q64[VEC || VK != VK_F64 ? 1 : TW];
  __shared__ uint64_t s_cnt[VEC || !CNT ? 1 : TW];
  const int lane = threadIdx.x;
  const Tile T = tile_of(P, blockIdx.x);
  double m[2] = {0.0, 0.0};
  bool nonfinite = false;
  if (T.border) sweep<false, VK, CNT, RAIN, VEC, true>(P, T, m, &nonfinite, s_q32, s_q64, s_cnt);
  else sweep<false, VK, CNT, RAIN, VEC, false>(P, T, m, &nonfinite, s_q32, s_q64, s_cnt);
  if (P.mass_part) {
    s_mass[0][lane] = m[0];
    s_mass[1][lane] = m[1];
    __syncthreads();
    if (lane == 0) {
      double a = 0.0, b = 0.0;
      for (int l = 0; l < 64; ++l) {
        a += s_mass[0][l];
        b += s_mass[1][l];
      }
      // Indexed by workgroup: the final reduction runs in one fixed order.
      P.mass_part[2 * blockIdx.x] = a;
      P.mass_part[2 * blockIdx.x + 1] = b;
    }
  }
}

// ---------------------------------------------------------------------------
// Block iterations (the paper's I+X scheme, Section 3.3 and Appendix B):
// w <- D^-1 (r + rho w) with blocks = tiles, D = the pairs a tile's top-down
// sweep follows (receiver in the row below, inside the tile), rho = every
// other pair.  One launch is one iteration.
template <int VK, bool CNT, int RAIN, bool VEC>
__global__ __launch_bounds__(64) void k_d8_iter(D8Params P) {
  __shared__ float s_q32[1];
  __shared__ double s_q64[VEC || VK != VK_F64 ? 1 : TW];
  __shared__ uint64_t s_cnt[VEC || !CNT ? 1 : TW];
  const Tile T = tile_of(P, blockIdx.x);
  bool nonfinite = false, badcode = false, changed = false;
  if (T.border)
    sweep<false, VK, CNT, RAIN, VEC, true, true>(P, T, nullptr, &nonfinite, s_q32, s_q64, s_cnt, &badcode,
                                                  &changed);
  else
    sweep<false, VK, CNT, RAIN, VEC, false, true>(P, T, nullptr, &nonfinite, s_q32, s_q64, s_cnt, &badcode,
                                                   &changed);
  if (__ballot(changed) && threadIdx.x == 0 && P.it_changed) *P.it_changed = 1;
  if (badcode) set_status(P.status, FR_ERR_BADCODE);
  if (nonfinite) set_status(P.status, FR_ERR_NONFINITE);
}

__global__ __launch_bounds__(256) void k_bi_combine(int mode, int64_t n, const double* bq, const uint64_t* bc,
                                                    const double* wq, const uint64_t* wc, double* tq,
                                                    uint64_t* tc, double* oq, uint64_t* oc, int32_t* changed) {
  bool chg = false;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    if (mode == 0) {
      if (tq) tq[i] = bq[i] - wq[i] + tq[i];
      if (tc) tc[i] = bc[i] - wc[i] + tc[i];
    } else if (mode == 1) {
      if (oq) oq[i] = wq[i] + tq[i] + oq[i];
      if (oc) {
        const uint64_t v = wc[i] + tc[i] + oc[i];
        oc[i] = v;
        chg |= v != wc[i];
      }
    } else {
      if (oq) oq[i] = 0.0;
      if (oc) oc[i] = 0;
    }
  }
  if (mode == 1 && __ballot(chg) && (threadIdx.x & 63) == 0 && changed && *(volatile int32_t*)changed == 0)
    *changed = 1;
}

int grid_for(uint32_t n) {
  uint32_t b = (n + 255) / 256;
  if (b > 16384) b = 16384;
  return (int)(b < 1 ? 1 : b);
}

}  // namespace

#define D8_DISPATCH(KERNEL, GRID, BLOCK, ...)                                                   \
  do {                                                                                          \
    if (vk == VK_FF) {                                                                          \
      if (cnt) hipLaunchKernelGGL((KERNEL<VK_FF, true>), GRID, BLOCK, 0, s, __VA_ARGS__);       \
      else hipLaunchKernelGGL((KERNEL<VK_FF, false>), GRID, BLOCK, 0, s, __VA_ARGS__);          \
    } else if (vk == VK_F64) {                                                                  \
      if (cnt) hipLaunchKernelGGL((KERNEL<VK_F64, true>), GRID, BLOCK, 0, s, __VA_ARGS__);      \
      else hipLaunchKernelGGL((KERNEL<VK_F64, false>), GRID, BLOCK, 0, s, __VA_ARGS__);         \
    } else {                                                                                    \
      hipLaunchKernelGGL((KERNEL<VK_NONE, true>), GRID, BLOCK, 0, s, __VA_ARGS__);              \
    }                                                                                           \
  } while (0)

// Launches a phase A / phase C kernel for the rain source and the row
// alignment of the grid (float4 / dword row loads when ncols % 4 == 0).
template <int VK, bool CNT, template <int, bool, int, bool> class K>
void d8_sweep_launch(const D8Params& P, hipStream_t s) {
  const dim3 g((unsigned)((int64_t)P.ntr * P.ntc)), b(64);
  const bool vec = (P.ncols % 4) == 0;
  const int rain = P.rain64 ? RAIN_F64 : (P.rain32 ? RAIN_F32 : RAIN_UNIT);
  if (VK == VK_NONE || rain == RAIN_UNIT) {
    if (vec) K<VK, CNT, RAIN_UNIT, true>::launch(g, b, s, P);
    else K<VK, CNT, RAIN_UNIT, false>::launch(g, b, s, P);
  } else if (rain == RAIN_F32) {
    if (vec) K<VK, CNT, RAIN_F32, true>::launch(g, b, s, P);
    else K<VK, CNT, RAIN_F32, false>::launch(g, b, s, P);
  } else {
    if (vec) K<VK, CNT, RAIN_F64, true>::launch(g, b, s, P);
    else K<VK, CNT, RAIN_F64, false>::launch(g, b, s, P);
  }
}

template <int VK, bool CNT, int RAIN, bool VEC>
struct UpK {
  static void launch(dim3 g, dim3 b, hipStream_t s, const D8Params& P) {
    hipLaunchKernelGGL((k_d8_up<VK, CNT, VK == VK_NONE ? RAIN_UNIT : RAIN, VEC>), g, b, 0, s, P);
  }
};
template <int VK, bool CNT, int RAIN, bool VEC>
struct DownK {
  static void launch(dim3 g, dim3 b, hipStream_t s, const D8Params& P) {
    hipLaunchKernelGGL((k_d8_down<VK, CNT, VK == VK_NONE ? RAIN_UNIT : RAIN, VEC>), g, b, 0, s, P);
  }
};

template <int VK, bool CNT, int RAIN, bool VEC>
struct IterK {
  static void launch(dim3 g, dim3 b, hipStream_t s, const D8Params& P) {
    hipLaunchKernelGGL((k_d8_iter<VK, CNT, VK == VK_NONE ? RAIN_UNIT : RAIN, VEC>), g, b, 0, s, P);
  }
};

template <template <int, bool, int, bool> class K>
void d8_sweep_dispatch(ValKind vk, bool cnt, const D8Params& P, hipStream_t s) {
  if (vk == VK_FF) {
    if (cnt) d8_sweep_launch<VK_FF, true, K>(P, s);
    else d8_sweep_launch<VK_FF, false, K>(P, s);
  } else if (vk == VK_F64) {
    if (cnt) d8_sweep_launch<VK_F64, true, K>(P, s);
    else d8_sweep_launch<VK_F64, false, K>(P, s);
  } else {
    d8_sweep_launch<VK_NONE, true, K>(P, s);
  }
}

// A second stream (default priority) per host thread and device, on which
// the root sweep runs beside the local sweep: the first is bound by its
// instruction count, the second by HBM, and neither reads what the other
// writes.
namespace {
struct SideStream {
  hipStream_t s = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
};
hipError_t side_stream(SideStream** out) {
  constexpr int kMaxDevices = 64;
  thread_local SideStream per[kMaxDevices];
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  SideStream& ss = per[dev];
  if (!ss.s) {
    if ((e = hipStreamCreateWithFlags(&ss.s, hipStreamNonBlocking)) != hipSuccess) return e;
    if ((e = hipEventCreateWithFlags(&ss.fork, hipEventDisableTiming)) != hipSuccess) return e;
    if ((e = hipEventCreateWithFlags(&ss.join, hipEventDisableTiming)) != hipSuccess) return e;
  }
  *out = &ss;
  return hipSuccess;
}
}  // namespace

hipError_t launch_d8_up(ValKind vk, bool cnt, const D8Params& P, hipStream_t s) {
  const dim3 g((unsigned)((int64_t)P.ntr * P.ntc)), b(64);
  SideStream* ss = nullptr;
  hipError_t e = side_stream(&ss);
  if (e != hipSuccess) return e;
  if ((e = hipEventRecord(ss->fork, s)) != hipSuccess) return e;
  if ((e = hipStreamWaitEvent(ss->s, ss->fork, 0)) != hipSuccess) return e;
  if ((P.ncols % 4) == 0) hipLaunchKernelGGL(k_d8_root<true>, g, b, 0, ss->s, P);
  else hipLaunchKernelGGL(k_d8_root<false>, g, b, 0, ss->s, P);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  d8_sweep_dispatch<UpK>(vk, cnt, P, s);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = hipEventRecord(ss->join, ss->s)) != hipSuccess) return e;
  return hipStreamWaitEvent(s, ss->join, 0);
}

hipError_t launch_d8_link(const D8Params& P, uint32_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_d8_link, dim3(grid_for(n)), dim3(256), 0, s, P, n);
  return hipGetLastError();
}

hipError_t launch_d8_round(ValKind vk, bool cnt, const D8Params& P, uint32_t n, int j, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int b = j & 1;
  D8_DISPATCH(k_d8_copy, dim3(grid_for(n)), dim3(256), P, n, b, j);
  D8_DISPATCH(k_d8_scatter, dim3(grid_for(n)), dim3(256), P, n, b, j);
  return hipGetLastError();
}

hipError_t launch_bi_combine(int mode, int64_t n, const double* bq, const uint64_t* bc, const double* wq,
                             const uint64_t* wc, double* tq, uint64_t* tc, double* oq, uint64_t* oc,
                             int32_t* changed, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_bi_combine, dim3((unsigned)blocks), dim3(256), 0, s, mode, n, bq, bc, wq, wc, tq, tc, oq,
                     oc, changed);
  return hipGetLastError();
}

hipError_t launch_d8_iter(ValKind vk, bool cnt, const D8Params& P, hipStream_t s) {
  if (vk == VK_FF) return hipErrorInvalidValue;  // float64 values or counts only
  if (vk == VK_F64) {
    if (cnt) d8_sweep_launch<VK_F64, true, IterK>(P, s);
    else d8_sweep_launch<VK_F64, false, IterK>(P, s);
  } else {
    d8_sweep_launch<VK_NONE, true, IterK>(P, s);
  }
  return hipGetLastError();
}

hipError_t launch_d8_down(ValKind vk, bool cnt, const D8Params& P, hipStream_t s) {
  d8_sweep_dispatch<DownK>(vk, cnt, P, s);
  return hipGetLastError();
}
#undef D8_DISPATCH

}  // namespace fr
