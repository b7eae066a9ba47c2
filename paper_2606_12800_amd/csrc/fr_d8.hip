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
//   A. Each 256 x 64 tile is swept by one wavefront, lane = column.  Edges
//      from row r+1 to row r inside the tile are followed in registers
//      (cross-lane shifts); every other edge -- leaving the tile, within a
//      row, or toward a higher row index -- is "cut".  The sweep yields each
//      cut cell's (exit's) local upstream sum, and a reverse sweep yields, for
//      every cell that receives over a cut edge (inlet), the exit or sink
//      where its in-tile path ends (its root).
//   B. The exits form a forest: exit e drains into exit root(receiver(e)),
//      or nowhere when that root is a sink.  Subtree sums over this forest are
//      computed by pointer doubling in ceil(log2(depth)) rounds.  These are
//      the paper's "C + 1 iterations" across block boundaries (Section 3.3,
//      Appendix B.1), collapsed to a logarithmic number of rounds.
//   C. Each tile is swept again with the totals of its cut donors added: the
//      result is final.  The float64 mass balance is reduced in the same pass.
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

// One grid row as seen by a lane: the W codes of its columns packed in a
// dword (byte j = column 4*lane + j of the tile) and the codes just left and
// right of them.  Off-grid cells read as sinks.
struct Row {
  uint32_t w, l, r;
  __device__ __forceinline__ uint32_t code(int j) const { return (w >> (8 * j)) & 0xFFu; }
  __device__ __forceinline__ uint32_t left(int j) const { return j == 0 ? l : code(j - 1); }
  __device__ __forceinline__ uint32_t right(int j) const { return j == W - 1 ? r : code(j + 1); }
};

struct RawRow {
  uint32_t w;     // own codes
  uint32_t side;  // lane 0: column left of the tile; lane 63: right of it
};

template <bool VEC>
__device__ __forceinline__ RawRow fetch_row(const D8Params& P, const Tile& T, int r, int lane) {
  const int nr = (int)P.nrows, nc = (int)P.ncols;
  RawRow x{0xFFFFFFFFu, SINK};
  if (r >= 0 && r < nr) {
    const uint8_t* row = P.code + (size_t)r * (size_t)nc;
    const int c = T.c0 + W * lane;
    if (VEC) {
      if (c < nc) x.w = *reinterpret_cast<const uint32_t*>(row + c);
    } else {
      uint32_t w = 0;
#pragma unroll
      for (int j = 0; j < W; ++j) w |= (c + j < nc ? (uint32_t)row[c + j] : SINK) << (8 * j);
      x.w = w;
    }
    if (lane == 0 && T.c0 > 0) x.side = row[T.c0 - 1];
    if (lane == 63 && T.c0 + TW < nc) x.side = row[T.c0 + TW];
  }
  return x;
}

__device__ __forceinline__ Row expand(const RawRow& x, int lane) {
  Row y;
  y.w = x.w;
  y.l = from_left(x.w, 0xFFFFFFFFu) >> 24;
  y.r = from_right(x.w, 0xFFFFFFFFu) & 0xFFu;
  if (lane == 0) y.l = x.side;
  if (lane == 63) y.r = x.side;
  return y;
}

// Classification of the cell in row r, tile column k = W*lane + j.
struct Cell {
  bool sink;  // no receiver (also malformed codes, columns off the grid)
  bool down;  // receiver in row r-1 inside the tile: followed by the sweep
  bool exit;  // receiver across a cut edge
};

__device__ __forceinline__ Cell classify(const D8Params& P, const Tile& T, int r, int k, uint32_t cd) {
  Cell x;
  bool bad = false;
  if (T.border && cd <= 7) {
    const int rr = r + nb_dr((int)cd), cc = T.c0 + k + nb_dc((int)cd);
    bad = rr < 0 || rr >= (int)P.nrows || cc < 0 || cc >= (int)P.ncols;
  }
  x.sink = cd > 7 || bad || k >= T.tw;
  const int tk = k + (int)cd - 1;  // target column of a down-row code
  x.down = !x.sink && cd <= 2 && r - 1 >= T.r0 && tk >= 0 && tk < T.tw;
  x.exit = !x.sink && !x.down;
  return x;
}

// Donors of the cell (row r, tile column k) that reach it over a cut edge,
// as a bit mask in neighbour order (bit n: neighbour n of the cell gives it
// water).  above = row r+1, here = row r, below = row r-1.  `rare` says
// whether any same-row or towards-higher-row donor can exist in this row.
__device__ __forceinline__ uint32_t cut_donors(const Row& above, const Row& here, const Row& below, int j,
                                               int k, bool top, bool rare, int tw) {
  if (k >= tw) return 0u;
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
  return m;
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

template <int VK, bool CNT>
struct Val {
  ff f;
  double d;
  uint64_t n;
};

// v + (cond ? x : 0), float-float with one renormalisation per call site.
__device__ __forceinline__ void acc_ff(float& s, float& e, bool cond, float xh, float xl) {
  xh = cond ? xh : 0.0f;
  xl = cond ? xl : 0.0f;
  const ff t = ff_two_sum(s, xh);
  s = t.hi;
  e += t.lo + xl;
}

constexpr int CHUNK = 4;  // rows fetched ahead of the sweep

// Top-down sweep over the tile (rows r0+th-1 .. r0), one wavefront, W
// columns per lane.  A cell's value is its rain, plus (phase C) the totals of
// its cut donors, plus the values of its donors in the row above inside the
// tile, which the previous step left in registers.  Codes and rain stream
// through registers CHUNK rows ahead; no LDS.
//   UP   (phase A): record every exit with its local value.
//   DOWN (phase C): write the final water / counts and the mass balance.
template <bool UP, int VK, bool CNT, bool R64, bool VEC>
__device__ void sweep(const D8Params& P, const Tile& T, int fb, double* mass, bool* nonfinite) {
  using RT = typename std::conditional<R64, double, float>::type;
  const int lane = threadIdx.x;
  const int k0 = W * lane;  // first tile column of this lane
  const int c = T.c0 + k0;
  const int nc = (int)P.ncols;
  const bool has_rain = VK != VK_NONE && (R64 ? P.rain64 != nullptr : P.rain32 != nullptr);
  const int rtop = T.r0 + T.th - 1;
  double m_sink = 0.0, m_rain = 0.0;
  Val<VK, CNT> pv[W];
#pragma unroll
  for (int j = 0; j < W; ++j) pv[j] = Val<VK, CNT>{};
  Row above = expand(fetch_row<VEC>(P, T, rtop + 1, lane), lane);
  Row here = expand(fetch_row<VEC>(P, T, rtop, lane), lane);
  RawRow cbuf[CHUNK];
  RT rbuf[CHUNK][W];
#define FR_FETCH(RSTART, CB, RB)                                                        \
  _Pragma("unroll") for (int i_ = 0; i_ < CHUNK; ++i_) {                                \
    const int rr_ = (RSTART) - i_;                                                      \
    CB[i_] = fetch_row<VEC>(P, T, rr_ - 1, lane);                                       \
    _Pragma("unroll") for (int j_ = 0; j_ < W; ++j_) RB[i_][j_] = (RT)1;               \
    if (has_rain && rr_ >= T.r0 && c < nc) {                                            \
      const size_t g_ = (size_t)rr_ * (size_t)nc + (size_t)c;                           \
      if (VEC && !R64) {                                                                \
        const float4 q_ = *reinterpret_cast<const float4*>(P.rain32 + g_);             \
        RB[i_][0] = (RT)q_.x; RB[i_][1] = (RT)q_.y; RB[i_][2] = (RT)q_.z; RB[i_][3] = (RT)q_.w; \
      } else {                                                                          \
        _Pragma("unroll") for (int j_ = 0; j_ < W; ++j_) if (c + j_ < nc)               \
          RB[i_][j_] = R64 ? (RT)P.rain64[g_ + j_] : (RT)P.rain32[g_ + j_];             \
      }                                                                                 \
    }                                                                                   \
  }
  FR_FETCH(rtop, cbuf, rbuf)
  for (int rc = rtop; rc >= T.r0; rc -= CHUNK) {
    RawRow cnext[CHUNK];
    RT rnext[CHUNK][W];
    if (rc - CHUNK >= T.r0) {
      FR_FETCH(rc - CHUNK, cnext, rnext)
    }
#pragma unroll
    for (int i = 0; i < CHUNK; ++i) {
      const int r = rc - i;
      if (r < T.r0) continue;  // uniform: past the bottom row of the tile
      const Row below = expand(cbuf[i], lane);
      const size_t g = (size_t)r * (size_t)nc + (size_t)c;
      const bool top = (r == rtop);
      const bool rare = !UP && rare_donors(here, below);
      // Values of the row above at the columns left and right of this lane.
      Val<VK, CNT> lv, rv;
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
      Val<VK, CNT> nv[W];
      bool exits[W], sinks[W];
#pragma unroll
      for (int j = 0; j < W; ++j) {
        const int k = k0 + j;
        const uint32_t cd = here.code(j);
        const Cell x = classify(P, T, r, k, cd);
        exits[j] = x.exit;
        sinks[j] = x.sink;
        const bool d5 = !top && k > 0 && above.left(j) == 2;
        const bool d6 = !top && above.code(j) == 1;
        const bool d7 = !top && k + 1 < T.tw && above.right(j) == 0;
        const Val<VK, CNT>& a5 = j == 0 ? lv : pv[j == 0 ? 0 : j - 1];
        const Val<VK, CNT>& a7 = j == W - 1 ? rv : pv[j == W - 1 ? 0 : j + 1];
        const double rain = (double)rbuf[i][j];
        if (!isfinite(rain)) *nonfinite = true;
        Val<VK, CNT> v;
        if (VK == VK_FF) {
          float sh = (float)rbuf[i][j], se = R64 ? (float)(rain - (double)(float)rain) : 0.0f;
          acc_ff(sh, se, d5, a5.f.hi, a5.f.lo);
          acc_ff(sh, se, d6, pv[j].f.hi, pv[j].f.lo);
          acc_ff(sh, se, d7, a7.f.hi, a7.f.lo);
          v.f = ff_fast(sh, se);
        }
        if (VK == VK_F64) v.d = rain + (d5 ? a5.d : 0.0) + (d6 ? pv[j].d : 0.0) + (d7 ? a7.d : 0.0);
        if (CNT) v.n = 1 + (d5 ? a5.n : 0) + (d6 ? pv[j].n : 0) + (d7 ? a7.n : 0);
        if (!UP) {
          // Totals of donors across cut edges (sparse).
          const uint32_t cut = cut_donors(above, here, below, j, k, top, rare, T.tw);
          if (cut) {
            for (int n = 0; n < 8; ++n) {
              if (!((cut >> n) & 1u)) continue;
              const size_t gj = (size_t)((int64_t)(g + j) + (int64_t)nb_dr(n) * nc + nb_dc(n));
              const uint32_t nd = P.node_of[gj];
              if (nd >= P.n_ex) {  // inconsistent bookkeeping: never follow it
                set_status(P.status, FR_ERR_BADCODE);
                continue;
              }
              if (VK == VK_FF) v.f = ff_add(v.f, ff{P.ex_hi[0][nd], P.ex_lo[0][nd]});
              if (VK == VK_F64) v.d += P.ex_q64[0][nd];
              if (CNT) v.n += P.ex_cnt[0][nd];
            }
          }
        }
        nv[j] = v;
      }
      bool any_exit = false;
#pragma unroll
      for (int j = 0; j < W; ++j) any_exit |= exits[j];
      if (UP && __ballot(any_exit)) {
        // Record exits (wavefront-compacted append).
#pragma unroll
        for (int j = 0; j < W; ++j) {
          const bool ex = exits[j];
          const uint64_t m = __ballot(ex);
          if (m) {
            uint32_t base = 0;
            if (lane == 0) base = atomicAdd(P.n_exits, (uint32_t)__popcll(m));
            base = __shfl(base, 0, 64);
            if (ex) {
              const uint32_t idx =
                  base + (uint32_t)__popcll(m & ((lane == 0) ? 0ull : (~0ull >> (64 - lane))));
              if (idx < P.cap) {
                P.node_of[g + j] = idx;
                P.ex_cell[idx] = (uint32_t)(g + j);
                if (VK == VK_FF) {
                  P.ex_hi[0][idx] = nv[j].f.hi;
                  P.ex_lo[0][idx] = nv[j].f.lo;
                }
                if (VK == VK_F64) P.ex_q64[0][idx] = nv[j].d;
                if (CNT) P.ex_cnt[0][idx] = nv[j].n;
              }
            }
          }
        }
      }
      if (!UP && c < nc) {
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
            a.x = nv[0].n; a.y = nv[1].n; b.x = nv[2].n; b.y = nv[3].n;
            *reinterpret_cast<ulonglong2*>(P.cnt + g) = a;
            *reinterpret_cast<ulonglong2*>(P.cnt + g + 2) = b;
          }
        } else {
#pragma unroll
          for (int j = 0; j < W; ++j) {
            if (c + j >= nc) continue;
            if (VK == VK_FF) P.q32[g + j] = nv[j].f.hi + nv[j].f.lo;
            if (VK == VK_F64) P.q64[g + j] = nv[j].d;
            if (CNT) P.cnt[g + j] = nv[j].n;
          }
        }
        if (VK != VK_NONE) {
#pragma unroll
          for (int j = 0; j < W; ++j) {
            if (c + j >= nc) continue;
            if (sinks[j]) m_sink += VK == VK_FF ? (double)nv[j].f.hi + (double)nv[j].f.lo : nv[j].d;
            m_rain += (double)rbuf[i][j];
          }
        }
      }
#pragma unroll
      for (int j = 0; j < W; ++j) pv[j] = nv[j];
      above = here;
      here = below;
    }
#pragma unroll
    for (int i = 0; i < CHUNK; ++i) {
      cbuf[i] = cnext[i];
#pragma unroll
      for (int j = 0; j < W; ++j) rbuf[i][j] = rnext[i][j];
    }
  }
#undef FR_FETCH
  if (mass) {
    mass[0] = m_sink;
    mass[1] = m_rain;
  }
}

// Bottom-up sweep (rows r0 .. r0+th-1): the root of every inlet -- the exit
// or sink where its path through the tile ends.
template <bool VEC>
__device__ void root_sweep(const D8Params& P, const Tile& T, bool* badcode) {
  const int lane = threadIdx.x;
  const int k0 = W * lane;
  const int nc = (int)P.ncols;
  const int rtop = T.r0 + T.th - 1;
  Row below = expand(fetch_row<VEC>(P, T, T.r0 - 1, lane), lane);
  Row here = expand(fetch_row<VEC>(P, T, T.r0, lane), lane);
  uint32_t rp[W];  // roots of the row below
#pragma unroll
  for (int j = 0; j < W; ++j) rp[j] = NONE;
  RawRow cbuf[CHUNK];
#pragma unroll
  for (int i = 0; i < CHUNK; ++i) cbuf[i] = fetch_row<VEC>(P, T, T.r0 + i + 1, lane);
  for (int rc = T.r0; rc <= rtop; rc += CHUNK) {
    RawRow cnext[CHUNK];
    if (rc + CHUNK <= rtop) {
#pragma unroll
      for (int i = 0; i < CHUNK; ++i) cnext[i] = fetch_row<VEC>(P, T, rc + CHUNK + i + 1, lane);
    }
#pragma unroll
    for (int i = 0; i < CHUNK; ++i) {
      const int r = rc + i;
      if (r > rtop) continue;  // uniform
      const Row above = expand(cbuf[i], lane);
      const bool top = (r == rtop);
      const bool rare = rare_donors(here, below);
      const uint32_t left = from_left(rp[W - 1], NONE), right = from_right(rp[0], NONE);
      const uint32_t base = (uint32_t)((size_t)r * (size_t)nc + (size_t)(T.c0 + k0));
      uint32_t nr[W];
#pragma unroll
      for (int j = 0; j < W; ++j) {
        const int k = k0 + j;
        const uint32_t cd = here.code(j);
        const Cell x = classify(P, T, r, k, cd);
        if (k < T.tw && cd != SINK && x.sink) *badcode = true;
        const uint32_t rl = j == 0 ? left : rp[j == 0 ? 0 : j - 1];
        const uint32_t rr = j == W - 1 ? right : rp[j == W - 1 ? 0 : j + 1];
        uint32_t root = base + j;
        if (x.down) root = cd == 0 ? rl : (cd == 1 ? rp[j] : rr);
        nr[j] = root;
        // Inlets: the top row, the two outer columns, and rows where a
        // same-row / towards-higher-row donor exists.
        if ((top || rare || k == 0 || k == T.tw - 1) && cut_donors(above, here, below, j, k, top, rare, T.tw))
          P.root_of[base + j] = root;
      }
#pragma unroll
      for (int j = 0; j < W; ++j) rp[j] = nr[j];
      below = here;
      here = above;
    }
#pragma unroll
    for (int i = 0; i < CHUNK; ++i) cbuf[i] = cnext[i];
  }
}

// ---------------------------------------------------------------------------
// Phase A.
template <int VK, bool CNT, bool R64, bool VEC>
__global__ __launch_bounds__(64) void k_d8_up(D8Params P) {
  const Tile T = tile_of(P, blockIdx.x);
  bool badcode = false, nonfinite = false;
  root_sweep<VEC>(P, T, &badcode);
  sweep<true, VK, CNT, R64, VEC>(P, T, 0, nullptr, &nonfinite);
  if (badcode) set_status(P.status, FR_ERR_BADCODE);
  if (nonfinite) set_status(P.status, FR_ERR_NONFINITE);
}

// ---------------------------------------------------------------------------
// Phase B: exit forest.
__global__ __launch_bounds__(256) void k_d8_link(D8Params P, uint32_t n) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int64_t e = P.ex_cell[i];
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

// Round k of pointer doubling (anc[b] = ancestor 2^k exits down, or NONE).
// Part 1: every exit that still has such an ancestor snapshots its sum (the
// sum over its subtree within distance < 2^k) and jumps its pointer.
template <int VK, bool CNT>
__global__ __launch_bounds__(256) void k_d8_copy(D8Params P, uint32_t n, int b) {
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
  if (__ballot(active) && (threadIdx.x & 63) == 0) atomicOr(&P.flags[1], 1);
}

// Part 2: each such exit adds its snapshot to the ancestor's sum in place.
template <int VK, bool CNT>
__global__ __launch_bounds__(256) void k_d8_scatter(D8Params P, uint32_t n, int b) {
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
template <int VK, bool CNT, bool R64, bool VEC>
__global__ __launch_bounds__(64) void k_d8_down(D8Params P, int fb) {
  __shared__ double s_mass[2][64];
  const int lane = threadIdx.x;
  const Tile T = tile_of(P, blockIdx.x);
  double m[2] = {0.0, 0.0};
  bool nonfinite = false;
  sweep<false, VK, CNT, R64, VEC>(P, T, fb, m, &nonfinite);
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

#define D8_LAUNCH(KERNEL, VKV, CNTV, ...)                                                     \
  do {                                                                                         \
    const dim3 g((unsigned)((int64_t)P.ntr * P.ntc)), b(64);                                   \
    const bool r64 = P.rain64 != nullptr;                                                      \
    const bool vec = (P.ncols % 4) == 0;                                                       \
    if (r64) {                                                                                 \
      if (vec) hipLaunchKernelGGL((KERNEL<VKV, CNTV, true, true>), g, b, 0, s, __VA_ARGS__);    \
      else hipLaunchKernelGGL((KERNEL<VKV, CNTV, true, false>), g, b, 0, s, __VA_ARGS__);       \
    } else {                                                                                   \
      if (vec) hipLaunchKernelGGL((KERNEL<VKV, CNTV, false, true>), g, b, 0, s, __VA_ARGS__);   \
      else hipLaunchKernelGGL((KERNEL<VKV, CNTV, false, false>), g, b, 0, s, __VA_ARGS__);      \
    }                                                                                          \
  } while (0)

#define D8_SWEEP_DISPATCH(KERNEL, ...)                                                          \
  do {                                                                                          \
    if (vk == VK_FF) {                                                                          \
      if (cnt) D8_LAUNCH(KERNEL, VK_FF, true, __VA_ARGS__);                                      \
      else D8_LAUNCH(KERNEL, VK_FF, false, __VA_ARGS__);                                         \
    } else if (vk == VK_F64) {                                                                  \
      if (cnt) D8_LAUNCH(KERNEL, VK_F64, true, __VA_ARGS__);                                     \
      else D8_LAUNCH(KERNEL, VK_F64, false, __VA_ARGS__);                                        \
    } else {                                                                                    \
      D8_LAUNCH(KERNEL, VK_NONE, true, __VA_ARGS__);                                             \
    }                                                                                           \
  } while (0)

hipError_t launch_d8_up(ValKind vk, bool cnt, const D8Params& P, hipStream_t s) {
  D8_SWEEP_DISPATCH(k_d8_up, P);
  return hipGetLastError();
}

hipError_t launch_d8_link(const D8Params& P, uint32_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_d8_link, dim3(grid_for(n)), dim3(256), 0, s, P, n);
  return hipGetLastError();
}

hipError_t launch_d8_round(ValKind vk, bool cnt, const D8Params& P, uint32_t n, int b, hipStream_t s) {
  if (n == 0) return hipSuccess;
  D8_DISPATCH(k_d8_copy, dim3(grid_for(n)), dim3(256), P, n, b);
  D8_DISPATCH(k_d8_scatter, dim3(grid_for(n)), dim3(256), P, n, b);
  return hipGetLastError();
}

hipError_t launch_d8_down(ValKind vk, bool cnt, const D8Params& P, int fb, hipStream_t s) {
  D8_SWEEP_DISPATCH(k_d8_down, P, fb);
  return hipGetLastError();
}
#undef D8_SWEEP_DISPATCH
#undef D8_LAUNCH
#undef D8_DISPATCH

}  // namespace fr
