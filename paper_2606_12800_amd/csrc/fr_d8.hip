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
constexpr int TH = D8_TH;
constexpr int HW = D8_TW + 8;  // LDS pitch: left halo at 3, lanes at 4..67, right halo at 68
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

// Column offset of the receiver for down-row codes 0, 1, 2.
__device__ __forceinline__ int down_dc(uint32_t cd) { return (int)cd - 1; }

struct Tile {
  int64_t r0, c0;
  int th, tw;
};

__device__ __forceinline__ Tile tile_of(const D8Params& P, int64_t t) {
  Tile T;
  const int64_t tr = t / P.ntc, tc = t - (t / P.ntc) * P.ntc;
  T.r0 = tr * TH;
  T.c0 = tc * TW;
  T.th = (int)(P.nrows - T.r0 < TH ? P.nrows - T.r0 : TH);
  T.tw = (int)(P.ncols - T.c0 < TW ? P.ncols - T.c0 : TW);
  return T;
}

// Codes of rows r0-1 .. r0+th and columns c0-1 .. c0+64 into LDS (off-grid
// cells read as sinks).  Rows are fetched four at a time with dword loads
// when rows are 4-byte aligned.
__device__ void load_codes(const D8Params& P, const Tile& T, uint8_t* sc) {
  const int lane = threadIdx.x;
  const int nrow = T.th + 2;
  if ((P.ncols % 4) == 0) {
    // lane = 16 * (row % 4) + dword; eight dword loads in flight per lane.
    const int sub = lane >> 4, dw = lane & 15;
    const int64_t c = T.c0 + 4 * dw;
    for (int i0 = 0; i0 < nrow; i0 += 32) {
      uint32_t v[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int i = i0 + 4 * j + sub;
        const int64_t gr = T.r0 - 1 + i;
        v[j] = 0xFFFFFFFFu;
        if (i < nrow && gr >= 0 && gr < P.nrows && c < P.ncols)
          v[j] = *reinterpret_cast<const uint32_t*>(P.code + gr * P.ncols + c);
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int i = i0 + 4 * j + sub;
        if (i < nrow) *reinterpret_cast<uint32_t*>(sc + i * HW + 4 + 4 * dw) = v[j];
      }
    }
  } else {
    const int64_t c = T.c0 + lane;
    for (int i0 = 0; i0 < nrow; i0 += 8) {
      uint8_t v[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int64_t gr = T.r0 - 1 + i0 + j;
        v[j] = (i0 + j < nrow && gr >= 0 && gr < P.nrows && c < P.ncols) ? P.code[gr * P.ncols + c] : SINK;
      }
#pragma unroll
      for (int j = 0; j < 8; ++j)
        if (i0 + j < nrow) sc[(i0 + j) * HW + 4 + lane] = v[j];
    }
  }
  // Halo columns.
  for (int i = lane; i < nrow; i += TW) {
    const int64_t gr = T.r0 - 1 + i;
    const bool row_ok = gr >= 0 && gr < P.nrows;
    const int64_t cl = T.c0 - 1, cr = T.c0 + TW;
    sc[i * HW + 3] = (row_ok && cl >= 0) ? P.code[gr * P.ncols + cl] : SINK;
    sc[i * HW + 4 + TW] = (row_ok && cr < P.ncols) ? P.code[gr * P.ncols + cr] : SINK;
  }
  __syncthreads();
  // Columns beyond a ragged right edge are off the grid.
  if (lane >= T.tw)
    for (int i = 0; i < nrow; ++i) sc[i * HW + 4 + lane] = SINK;
  __syncthreads();
}

// Classification of the cell at LDS row i (grid row r) for this lane.
struct Cell {
  uint32_t cd;
  bool sink;    // no receiver (also malformed codes)
  bool down;    // receiver in the previous row inside the tile: followed
  bool exit;    // receiver across a cut edge
};

__device__ __forceinline__ Cell classify(const D8Params& P, const Tile& T, const uint8_t* sc, int i,
                                         int lane) {
  Cell x;
  x.cd = sc[i * HW + 4 + lane];
  const int64_t r = T.r0 - 1 + i, c = T.c0 + lane;
  bool bad = false;
  if (x.cd <= 7) {
    const int64_t rr = r + nb_dr((int)x.cd), cc = c + nb_dc((int)x.cd);
    bad = rr < 0 || rr >= P.nrows || cc < 0 || cc >= P.ncols;
  }
  x.sink = x.cd > 7 || bad || lane >= T.tw;
  x.down = !x.sink && x.cd <= 2 && i >= 2 && lane + down_dc(x.cd) >= 0 && lane + down_dc(x.cd) < T.tw;
  x.exit = !x.sink && !x.down;
  return x;
}

// Donors of the cell at LDS row i that reach it over a cut edge, as a bit
// mask in neighbour order k (bit k: neighbour k of the cell gives it water).
__device__ __forceinline__ uint32_t cut_donors(const uint8_t* sc, const Tile& T, int i, int lane) {
  const int top = (i == T.th);  // row r0+th-1: the row above is another tile
  const uint8_t* up = sc + (i - 1) * HW + 3 + lane;  // row r-1, columns c-1..c+1
  const uint8_t* mid = sc + i * HW + 3 + lane;
  const uint8_t* dn = sc + (i + 1) * HW + 3 + lane;  // row r+1
  uint32_t m = 0;
  // (r-1, *) giving to (r, c): codes 7, 6, 5 (towards row + 1): always cut.
  m |= (up[0] == 7) << 0;
  m |= (up[1] == 6) << 1;
  m |= (up[2] == 5) << 2;
  // same row: codes 4 (from the left) and 3 (from the right): always cut.
  m |= (mid[0] == 4) << 3;
  m |= (mid[2] == 3) << 4;
  // (r+1, *) giving to (r, c): codes 2, 1, 0: cut across the tile border.
  m |= (dn[0] == 2 && (top || lane == 0)) << 5;
  m |= (dn[1] == 1 && top) << 6;
  m |= (dn[2] == 0 && (top || lane == T.tw - 1)) << 7;
  return m;
}

template <int VK, bool CNT>
struct Val {
  ff f;
  double d;
  uint64_t n;
};

constexpr int CHUNK = 16;  // rows whose rain is fetched ahead of the sweep

// Top-down sweep over the tile (rows r0+th-1 .. r0), one wavefront, lane =
// column.  A cell's value is its rain, plus (phase C) the totals of its cut
// donors, plus the values of its donors in the row above inside the tile,
// which the previous step left in registers.
//   UP   (phase A): record every exit with its local value.
//   DOWN (phase C): write the final water / counts and the mass balance.
template <bool UP, int VK, bool CNT, bool R64>
__device__ void sweep(const D8Params& P, const Tile& T, const uint8_t* sc, int fb, double* mass,
                      bool* nonfinite) {
  using RT = typename std::conditional<R64, double, float>::type;
  const int lane = threadIdx.x;
  const int64_t c = T.c0 + lane;
  const bool live = lane < T.tw;
  const bool has_rain = VK != VK_NONE && (R64 ? P.rain64 != nullptr : P.rain32 != nullptr);
  double m_sink = 0.0, m_rain = 0.0;
  Val<VK, CNT> prev{};
  // Rain of the next CHUNK rows (top-down), fetched before they are needed.
  RT rbuf[CHUNK];
#define FR_FETCH(I_TOP, A)                                                          \
  _Pragma("unroll") for (int j = 0; j < CHUNK; ++j) {                               \
    const int i_ = (I_TOP) - j;                                                     \
    const int64_t g_ = (T.r0 - 1 + i_) * P.ncols + c;                               \
    A[j] = (RT)1;                                                                   \
    if (has_rain && i_ >= 1 && live) A[j] = R64 ? (RT)P.rain64[g_] : (RT)P.rain32[g_]; \
  }
  FR_FETCH(T.th, rbuf)
  for (int i0 = T.th; i0 >= 1; i0 -= CHUNK) {
    RT nbuf[CHUNK];
    if (i0 - CHUNK >= 1) {
      FR_FETCH(i0 - CHUNK, nbuf)
    }
#pragma unroll
    for (int j = 0; j < CHUNK; ++j) {
      const int i = i0 - j;
      if (i < 1) continue;  // uniform: past the bottom row of the tile
      const int64_t g = (T.r0 - 1 + i) * P.ncols + c;
      const Cell x = classify(P, T, sc, i, lane);
      const bool top = (i == T.th);
      const uint8_t* dn = sc + (i + 1) * HW + 3 + lane;
      const bool d5 = !top && lane > 0 && dn[0] == 2;
      const bool d6 = !top && dn[1] == 1;
      const bool d7 = !top && lane + 1 < T.tw && dn[2] == 0;
      Val<VK, CNT> v{};
      const double rain = (double)rbuf[j];
      if (VK == VK_FF) {
        if (R64) v.f = {(float)rain, (float)(rain - (double)(float)rain)};
        else v.f = {(float)rbuf[j], 0.0f};
      }
      if (VK == VK_F64) v.d = rain;
      if (CNT) v.n = 1;
      if (!isfinite(rain)) *nonfinite = true;
      if (!UP) {
        // Totals of donors across cut edges (sparse).
        const uint32_t cut = live ? cut_donors(sc, T, i, lane) : 0u;
        if (cut) {
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            if (!((cut >> k) & 1u)) continue;
            const int64_t gj = g + (int64_t)nb_dr(k) * P.ncols + nb_dc(k);
            const uint32_t nd = P.node_of[gj];
            if (nd >= P.n_ex) {  // inconsistent bookkeeping: never follow it
              set_status(P.status, FR_ERR_BADCODE);
              continue;
            }
            if (VK == VK_FF) v.f = ff_add(v.f, ff{P.ex_hi[fb][nd], P.ex_lo[fb][nd]});
            if (VK == VK_F64) v.d += P.ex_q64[fb][nd];
            if (CNT) v.n += P.ex_cnt[fb][nd];
          }
        }
      }
      if (VK == VK_FF) {
        const float lh = from_left(prev.f.hi), ll = from_left(prev.f.lo);
        const float rh = from_right(prev.f.hi), rl = from_right(prev.f.lo);
        if (d5) v.f = ff_add(v.f, ff{lh, ll});
        if (d6) v.f = ff_add(v.f, prev.f);
        if (d7) v.f = ff_add(v.f, ff{rh, rl});
      }
      if (VK == VK_F64) {
        const double l = from_left(prev.d), rr = from_right(prev.d);
        if (d5) v.d += l;
        if (d6) v.d += prev.d;
        if (d7) v.d += rr;
      }
      if (CNT) {
        const uint64_t l = from_left(prev.n), rr = from_right(prev.n);
        if (d5) v.n += l;
        if (d6) v.n += prev.n;
        if (d7) v.n += rr;
      }
      if (UP) {
        // Record exits (wavefront-compacted append).
        const bool ex = live && x.exit;
        const uint64_t m = __ballot(ex);
        if (m) {
          uint32_t base = 0;
          if (lane == 0) base = atomicAdd(P.n_exits, (uint32_t)__popcll(m));
          base = __shfl(base, 0, 64);
          if (ex) {
            const uint32_t idx =
                base + (uint32_t)__popcll(m & ((lane == 0) ? 0ull : (~0ull >> (64 - lane))));
            if (idx < P.cap) {
              P.node_of[g] = idx;
              P.ex_cell[idx] = (uint32_t)g;
              if (VK == VK_FF) {
                P.ex_hi[0][idx] = v.f.hi;
                P.ex_lo[0][idx] = v.f.lo;
              }
              if (VK == VK_F64) P.ex_q64[0][idx] = v.d;
              if (CNT) P.ex_cnt[0][idx] = v.n;
            }
          }
        }
      } else if (live) {
        if (VK == VK_FF) P.q32[g] = v.f.hi + v.f.lo;
        if (VK == VK_F64) P.q64[g] = v.d;
        if (CNT) P.cnt[g] = v.n;
        if (VK != VK_NONE) {
          if (x.sink) m_sink += VK == VK_FF ? (double)v.f.hi + (double)v.f.lo : v.d;
          m_rain += rain;
        }
      }
      prev = v;
    }
#pragma unroll
    for (int j = 0; j < CHUNK; ++j) rbuf[j] = nbuf[j];
  }
#undef FR_FETCH
  if (mass) {
    mass[0] = m_sink;
    mass[1] = m_rain;
  }
}

// ---------------------------------------------------------------------------
// Phase A.
template <int VK, bool CNT, bool R64>
__global__ __launch_bounds__(64) void k_d8_up(D8Params P) {
  __shared__ uint8_t sc[(TH + 2) * HW];
  const int lane = threadIdx.x;
  const Tile T = tile_of(P, blockIdx.x);
  load_codes(P, T, sc);
  const int64_t c = T.c0 + lane;
  bool badcode = false, nonfinite = false;

  // Bottom-up sweep (rows r0 .. r0+th-1): roots of inlets.
  uint32_t root_prev = NONE;
  for (int i = 1; i <= T.th; ++i) {
    const int64_t r = T.r0 - 1 + i;
    const Cell x = classify(P, T, sc, i, lane);
    if (lane < T.tw && x.cd != SINK && x.sink) badcode = true;
    const uint32_t rl = from_left(root_prev, NONE), rr = from_right(root_prev, NONE);
    const uint32_t self = (uint32_t)(r * P.ncols + c);
    uint32_t root = self;
    if (x.down) root = x.cd == 0 ? rl : (x.cd == 1 ? root_prev : rr);
    if (lane < T.tw && cut_donors(sc, T, i, lane)) P.root_of[self] = root;
    root_prev = root;
  }
  sweep<true, VK, CNT, R64>(P, T, sc, 0, nullptr, &nonfinite);
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

// Round k of pointer doubling, part 1: copy the sums and jump the pointers.
template <int VK, bool CNT>
__global__ __launch_bounds__(256) void k_d8_copy(D8Params P, uint32_t n, int b) {
  bool active = false;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    if (VK == VK_FF) {
      P.ex_hi[b ^ 1][i] = P.ex_hi[b][i];
      P.ex_lo[b ^ 1][i] = P.ex_lo[b][i];
    }
    if (VK == VK_F64) P.ex_q64[b ^ 1][i] = P.ex_q64[b][i];
    if (CNT) P.ex_cnt[b ^ 1][i] = P.ex_cnt[b][i];
    const uint32_t a = P.anc[b][i];
    const uint32_t a2 = a == NONE ? NONE : P.anc[b][a];
    P.anc[b ^ 1][i] = a2;
    active |= (a2 != NONE);
  }
  if (__ballot(active) && (threadIdx.x & 63) == 0) atomicOr(&P.flags[1], 1);
}

// Part 2: every exit with an ancestor 2^k steps down adds its sum there.
template <int VK, bool CNT>
__global__ __launch_bounds__(256) void k_d8_scatter(D8Params P, uint32_t n, int b) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const uint32_t a = P.anc[b][i];
    if (a == NONE) continue;
    if (VK == VK_FF) {
      const float xh = P.ex_hi[b][i], xl = P.ex_lo[b][i];
      const float old = atomicAdd(&P.ex_hi[b ^ 1][a], xh);
      const ff e = ff_two_sum(old, xh);  // e.hi is what the atomic stored
      atomicAdd(&P.ex_lo[b ^ 1][a], e.lo + xl);
    }
    if (VK == VK_F64) atomicAdd(&P.ex_q64[b ^ 1][a], P.ex_q64[b][i]);
    if (CNT) atomicAdd(reinterpret_cast<unsigned long long*>(&P.ex_cnt[b ^ 1][a]),
                       (unsigned long long)P.ex_cnt[b][i]);
  }
}

// ---------------------------------------------------------------------------
// Phase C.
template <int VK, bool CNT, bool R64>
__global__ __launch_bounds__(64) void k_d8_down(D8Params P, int fb) {
  __shared__ uint8_t sc[(TH + 2) * HW];
  __shared__ double s_mass[2][64];
  const int lane = threadIdx.x;
  const Tile T = tile_of(P, blockIdx.x);
  load_codes(P, T, sc);
  double m[2] = {0.0, 0.0};
  bool nonfinite = false;
  sweep<false, VK, CNT, R64>(P, T, sc, fb, m, &nonfinite);
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

#define D8_SWEEP_DISPATCH(KERNEL, ...)                                                          \
  do {                                                                                          \
    const dim3 g((unsigned)((int64_t)P.ntr * P.ntc)), b(64);                                    \
    const bool r64 = P.rain64 != nullptr;                                                       \
    if (vk == VK_FF) {                                                                          \
      if (cnt) {                                                                                \
        if (r64) hipLaunchKernelGGL((KERNEL<VK_FF, true, true>), g, b, 0, s, __VA_ARGS__);      \
        else hipLaunchKernelGGL((KERNEL<VK_FF, true, false>), g, b, 0, s, __VA_ARGS__);         \
      } else {                                                                                  \
        if (r64) hipLaunchKernelGGL((KERNEL<VK_FF, false, true>), g, b, 0, s, __VA_ARGS__);     \
        else hipLaunchKernelGGL((KERNEL<VK_FF, false, false>), g, b, 0, s, __VA_ARGS__);        \
      }                                                                                         \
    } else if (vk == VK_F64) {                                                                  \
      if (cnt) {                                                                                \
        if (r64) hipLaunchKernelGGL((KERNEL<VK_F64, true, true>), g, b, 0, s, __VA_ARGS__);     \
        else hipLaunchKernelGGL((KERNEL<VK_F64, true, false>), g, b, 0, s, __VA_ARGS__);        \
      } else {                                                                                  \
        if (r64) hipLaunchKernelGGL((KERNEL<VK_F64, false, true>), g, b, 0, s, __VA_ARGS__);    \
        else hipLaunchKernelGGL((KERNEL<VK_F64, false, false>), g, b, 0, s, __VA_ARGS__);       \
      }                                                                                         \
    } else {                                                                                    \
      hipLaunchKernelGGL((KERNEL<VK_NONE, true, false>), g, b, 0, s, __VA_ARGS__);              \
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
#undef D8_DISPATCH

}  // namespace fr
