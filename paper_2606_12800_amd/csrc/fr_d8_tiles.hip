// Tile-forest path for single-receiver codes (D8 / D4) whose flow runs in
// every direction, as on depression-filled terrain (the paper's workflow,
// Section 4: fill, then route).
//
// The row sweeps (fr_d8_a.hip) follow only the edges toward the previous
// row; every other cell becomes an exit of the forest, and on filled terrain
// so many do that the exit list overflows.  Here each tile of 32 x 64 cells
// solves its own part of (I - W^T) q = r (Section 2.2) for any flow
// direction, in LDS, so that only the cells whose receiver lies in another
// tile are exits -- at most the tile's perimeter, 188 of its 2048 cells.
// Like the paper's per-process solves (Section 2.4, Section 3.3), the tiles
// are independent blocks; the exits then feed a fixed-point exit forest
// (fr_d8_forest.hip: the row sweeps' link and totals, with a work queue in
// place of their pointer-doubling rounds), which joins them, and a second
// pass over every tile adds its donors' totals.
//
// Inside a tile (one workgroup of 256 threads, 8 cells each):
//   1. the codes with a one-cell halo into LDS; each cell's receiver inside
//      the tile, or none (a sink, or an exit); each cell marks itself in its
//      receiver's donor mask;
//   2. pointer jumping over those receivers: each cell's root -- the sink or
//      exit where its in-tile path ends -- and its depth, the number of
//      in-tile edges to the root, in about log2(depth) rounds;
//   3. phase A (up) needs only each exit's upstream sum: every cell whose
//      root is an exit adds its rain to the exit's accumulator, a 128-bit
//      fixed point in LDS (unit from the tile's largest |rain|; integer
//      atomics, so the order of the additions changes no bit);
//   4. phase C (down) needs every cell's value: a counting sort of the cells
//      with donors inside the tile by depth, then the levels of depth,
//      deepest first, on one wavefront.  A cell's donors inside the tile lie
//      exactly one level deeper, so each cell of the level reads its
//      finished donors at once (the LDS serves one wavefront's accesses in
//      order: no barrier between levels) and adds them in neighbour order:
//      a fixed order, so results repeat bit for bit.
// Steps 1 and 2 run once: phase A leaves every cell a 32-bit word (its
// depth, its in-tile and out-of-tile donor masks, a sink flag) in the
// output buffer (q, or the low half of each 64-bit value or count), and
// phase C reads the word back instead of the codes, then overwrites it with
// the cell's result; phase C fetches only the forest totals of the halo
// cells that drain into the tile.
// Phase C's counts live in LDS as 32 bits (at most the grid's cell count,
// below 2^31), so that four workgroups fit on a compute unit; phase A holds
// no per-cell values at all.
// Global loads that depend on nothing else (codes or words, rain, the exit
// indices of the halo) are issued together at the start of a tile.
// Phase A stores the local sums of the exits in the exit list and, for every
// cell receiving water over the tile's edge (inlet), its root.  Phase C
// (down) starts the inlets from their out-of-tile donors' forest totals;
// its values are final and go out with the tile's mass-balance partial.
//
// The path runs only after the row sweeps' exit list overflowed, or when the
// caller chose it: every launch first reads the control block's gate and
// returns at once when it is closed, and each workgroup walks a stride of tiles, so that a closed gate
// costs a few thousand short workgroups.
#include "fr_d8.hpp"

namespace fr {
namespace {

constexpr int HR = D8T_ROWS;   // tile rows
constexpr int HC = D8T_COLS;   // tile columns
constexpr int HN = HR * HC;    // cells per tile
constexpr int HT = 256;        // threads per workgroup
constexpr int HK = HN / HT;    // cells per thread
constexpr int HW = HC + 2;     // halo row width
constexpr uint32_t PT_TERM = 0x8000u;  // pointer flag: the target is a root
constexpr int NO_LEVEL = 0x7FFF;       // not on a path to a root (cycle) or off the grid
static_assert(HC == 64, "a tile row is one wavefront");
static_assert(HN % HT == 0 && HN <= 0x8000, "pointers fit 15 bits");

struct TT {
  int64_t r0, c0;
  int h, w, id;
};

// Virtual tile t runs on XCD t % 8 (the grid is a multiple of 8 workgroups,
// dispatched round-robin): give each XCD a contiguous run of tiles, whose
// shared halo rows and columns then meet in one L2.
__device__ __forceinline__ TT tile_at(const D8Params& P, int t, int ntiles) {
  const int q = ntiles / 8;
  const int id = t < 8 * q ? (t % 8) * q + t / 8 : t;
  const int ntc = (int)((P.ncols + HC - 1) / HC);
  const int tr = id / ntc, tc = id - tr * ntc;
  TT T;
  T.id = id;
  T.r0 = (int64_t)tr * HR;
  T.c0 = (int64_t)tc * HC;
  T.h = (int)min((int64_t)HR, P.nrows - T.r0);
  T.w = (int)min((int64_t)HC, P.ncols - T.c0);
  return T;
}

template <int VK>
struct TV;
template <>
struct TV<VK_FF> {
  using T = ff;
  __device__ static T zero() { return {0.0f, 0.0f}; }
  __device__ static T add(T a, T b) { return ff_add(a, b); }
  __device__ static double mass(T a) { return (double)a.hi + (double)a.lo; }
};
template <>
struct TV<VK_F64> {
  using T = double;
  __device__ static T zero() { return 0.0; }
  __device__ static T add(T a, T b) { return a + b; }
  __device__ static double mass(T a) { return a; }
};
template <>
struct TV<VK_NONE> {
  using T = int;  // unused
  __device__ static T zero() { return 0; }
  __device__ static T add(T a, T) { return a; }
  __device__ static double mass(T) { return 0.0; }
};

template <int RAIN>
__device__ __forceinline__ double rain_at(const D8Params& P, int64_t g) {
  if (RAIN == RAIN_F32) return (double)P.rain32[g];
  if (RAIN == RAIN_F64) return P.rain64[g];
  return 1.0;
}

template <int VK, int RAIN>
__device__ __forceinline__ typename TV<VK>::T src_of(const D8Params& P, int64_t g) {
  if constexpr (VK == VK_FF) {
    if (RAIN == RAIN_F32) return ff{P.rain32[g], 0.0f};
    if (RAIN == RAIN_F64) {
      const double r = P.rain64[g];
      const float hi = (float)r;
      return ff{hi, (float)(r - (double)hi)};
    }
    return ff{1.0f, 0.0f};
  } else if constexpr (VK == VK_F64) {
    return rain_at<RAIN>(P, g);
  } else {
    return 0;
  }
}

__device__ __forceinline__ int wave_max(int x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x = max(x, __shfl_xor(x, off, 64));
  return x;
}
__device__ __forceinline__ double wave_max_d(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x = fmax(x, __shfl_xor(x, off, 64));
  return x;
}

// A tile's exits lie on its perimeter.
constexpr int D8T_MAX_EXITS = 2 * HC + 2 * (HR - 2);

// Between the two phases each cell's structure travels in the output buffer
// (32-bit words: q as float32, or the low half of a float64 / count slot),
// which phase C then overwrites with the cell's result: its depth in bits
// 0-11 (CW_NOLEVEL when its path ends on a cycle), its donor mask (in-tile
// donors | out-of-tile donors << 8) in bits 12-27, bit 28 when it is a sink.
constexpr uint32_t CW_NOLEVEL = 0xFFFu;
template <int VK>
__device__ __forceinline__ uint32_t* cw_at(const D8Params& P, int64_t g) {
  if (VK == VK_FF) return reinterpret_cast<uint32_t*>(P.q32) + g;
  if (VK == VK_F64) return reinterpret_cast<uint32_t*>(P.q64) + 2 * g;
  return reinterpret_cast<uint32_t*>(P.cnt) + 2 * g;
}

// Halo positions (the ring of cells around the tile): top row, bottom row,
// then the left and right columns.
constexpr int NHALO = 2 * HW + 2 * HR;
__device__ __forceinline__ int halo_id(int hr, int hc) {  // frame coordinates, on the ring
  if (hr == 0) return hc;
  if (hr == HR + 1) return HW + hc;
  return 2 * HW + (hc == 0 ? 0 : HR) + (hr - 1);
}
__device__ __forceinline__ void halo_pos(int h, int& hr, int& hc) {
  if (h < HW) {
    hr = 0;
    hc = h;
  } else if (h < 2 * HW) {
    hr = HR + 1;
    hc = h - HW;
  } else {
    const int k = h - 2 * HW;
    hr = 1 + (k % HR);
    hc = k < HR ? 0 : HW - 1;
  }
}

// Tile-local offset of the neighbour in direction n (row-major, 64 columns):
// byte n of the constant holds the offset + 65.
__device__ __forceinline__ int nb_off(int n) {
  return (int)((0x8281804240020100ull >> (8 * n)) & 0xFFull) - 65;
}

// Level entries (one 32-bit word per cell with in-tile donors): the cell in
// bits 0-10, its in-tile donor mask (bit n: neighbour n gives it water) in
// bits 11-18, and the directions of its first four donors, 3 bits each, from
// bit 19.  Value and count arrays hold one more slot, LV_ZERO, that stays
// zero: a missing donor reads it.
constexpr int LV_ZERO = HN;

__device__ __forceinline__ uint32_t level_entry(int i, uint32_t mask) {
  uint32_t d = 0, m = mask;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    d |= ((uint32_t)__builtin_ctz(m | 0x100u) & 7u) << (3 * q);
    m &= m - 1;
  }
  return (uint32_t)i | (mask << 11) | (d << 19);
}

// One cell of a level: its value (rain and out-of-tile inflow so far) plus
// the finished values of its in-tile donors, in neighbour order.  The first
// four donors are read at once and added without branches (a missing donor
// reads the zero slot and adds an exact zero, which changes no bit of the
// sum); float-float sums are normalised once.  Cells with more donors finish
// in a loop (rare).
template <int VK, bool CNT, class CT>
__device__ __forceinline__ void level_cell(typename TV<VK>::T* s_v, CT* s_c, uint32_t ent) {
  using V = typename TV<VK>::T;
  const int i = (int)(ent & 0x7FFu);
  const uint32_t mask = (ent >> 11) & 0xFFu;
  const int kq = __popc(mask);
  int a[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) a[q] = q < kq ? i + nb_off((int)((ent >> (19 + 3 * q)) & 7u)) : LV_ZERO;
  V own{}, x[4];
  uint32_t cown = 0, y[4];
  if (VK != VK_NONE) {
    own = s_v[i];
#pragma unroll
    for (int q = 0; q < 4; ++q) x[q] = s_v[a[q]];
  }
  if (CNT) {
    cown = s_c[i];
#pragma unroll
    for (int q = 0; q < 4; ++q) y[q] = s_c[a[q]];
  }
  uint32_t rest = 0;  // donors after the fourth (rare)
  if (kq > 4) {
    rest = mask;
#pragma unroll
    for (int q = 0; q < 4; ++q) rest &= rest - 1;
  }
  if constexpr (VK == VK_FF) {
    float h = own.hi, e = own.lo;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const ff t = ff_two_sum(h, x[q].hi);
      h = t.hi;
      e += t.lo + x[q].lo;
    }
    for (uint32_t r = rest; r; r &= r - 1) {
      const ff xv = s_v[i + nb_off(__builtin_ctz(r))];
      const ff t = ff_two_sum(h, xv.hi);
      h = t.hi;
      e += t.lo + xv.lo;
    }
    s_v[i] = ff_fast(h, e);
  }
  if constexpr (VK == VK_F64) {
    double v = own;
#pragma unroll
    for (int q = 0; q < 4; ++q) v += x[q];
    for (uint32_t r = rest; r; r &= r - 1) v += s_v[i + nb_off(__builtin_ctz(r))];
    s_v[i] = v;
  }
  if (CNT) {
    uint32_t c = cown;
#pragma unroll
    for (int q = 0; q < 4; ++q) c += y[q];
    for (uint32_t r = rest; r; r &= r - 1) c += s_c[i + nb_off(__builtin_ctz(r))];
    s_c[i] = (CT)c;
  }
}

template <int RAIN>
struct RainReg {
  using T = typename std::conditional<RAIN == RAIN_F64, double, float>::type;
};

// Waves per SIMD the register budget is cut for: phase A holds no per-cell
// values, so six of its waves fit (five with float64 rain, whose registers
// would spill), and its 22.6 KB of LDS allows that many workgroups; phase C
// is held to four by its LDS.
template <bool UP, int VK, bool CNT, int RAIN>
__global__ __launch_bounds__(HT, UP ? (RAIN == RAIN_F64 ? 5 : 6) : 4) void k_d8t(D8Params P, int ntiles) {
  if (__hip_atomic_load(&P.ctl->d8_tiles, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) return;  // uniform
  const uint32_t n_ex = *P.n_exits;
  if (!UP && n_ex > P.cap) return;  // uniform: the engine takes over
  using V = typename TV<VK>::T;
  using RT = typename RainReg<RAIN>::T;
  constexpr int NCODE = (HR + 2) * HW;
  constexpr int NCU = (NCODE + HT - 1) / HT;  // code loads per thread
  constexpr int VB = VK == VK_NONE ? 0 : (HN + 2) * 8;  // one more slot (zero), 16-byte multiple
  // Phase C's counts in LDS: at most the grid's cell count, below 2^31 (32
  // bits); with the level histogram over the donor masks its LDS stays
  // within a quarter of a compute unit's.  (Phase A keeps no per-cell
  // values.)
  using CT = uint32_t;
  constexpr int CB = CNT ? (HN + 8) * (int)sizeof(CT) : 0;  // one more slot (zero), 16-byte multiple
  constexpr int HB = (UP ? 0 : NHALO * ((VK == VK_NONE ? 0 : 8) + (CNT ? 4 : 0)));
  constexpr int MB = HN * 2 > HB ? HN * 2 : HB;
  // Phase C: values and counts; phase A: the exits' fixed-point sums and
  // counts (two 64-bit words and one 32-bit word per exit).
  constexpr int AB = D8T_MAX_EXITS * (8 + 8 + 4);
  __shared__ __align__(16) unsigned char s_buf[UP ? (AB + 15) / 16 * 16 : VB + CB];
  // Donor masks (16 bits per cell: in-tile donors, out-of-tile donors);
  // once read, the forest totals of the halo cells, and once those are
  // added, the level histogram (phase C).
  __shared__ __align__(16) unsigned char s_mb[MB];
  // Pointer jumping (receiver | root flag, depth << 16 per cell), then the
  // cells with in-tile donors in level order (cell | donor mask << 16).
  __shared__ uint32_t s_x[HN];
  __shared__ __align__(16) uint32_t s_lev_a[UP ? HN / 2 : 4];  // phase A's level histogram
  __shared__ uint8_t s_code[NCODE];
  __shared__ int s_int[16];
  __shared__ int s_open[16];
  constexpr int NEED_WORDS = (NHALO + 31) / 32;
  __shared__ uint32_t s_need[NEED_WORDS];  // phase C: halo cells that drain into the tile
  __shared__ double s_dbl[8];
  __shared__ float s_flt[4];
  V* s_v = reinterpret_cast<V*>(s_buf);
  CT* s_c = reinterpret_cast<CT*>(s_buf + VB);
  uint32_t* s_msk = reinterpret_cast<uint32_t*>(s_mb);
  V* s_hv = reinterpret_cast<V*>(s_mb);
  CT* s_hc = reinterpret_cast<CT*>(s_mb + (VK == VK_NONE ? 0 : NHALO * 8));
  // Level histogram, then level offsets: 16 bits per level.
  uint32_t* s_lev = UP ? s_lev_a : reinterpret_cast<uint32_t*>(s_mb);
  uint16_t* s_off = reinterpret_cast<uint16_t*>(s_lev);
  const int64_t nr = P.nrows, nc = P.ncols;
  // The wavefront that sweeps the levels (any one wavefront of the group
  // gives the same result): the one on SIMD (workgroup slot mod 4), read
  // from the hardware's wave identity register (SIMD in bits 5:4, the
  // workgroup's slot on its compute unit in bits 19:16), so that the level
  // sweeps of the workgroups sharing a compute unit issue on different
  // SIMDs.  Published in LDS so that the choice is uniform in the group.
  __shared__ int s_simd[5];
  {
    const uint32_t hw = __builtin_amdgcn_s_getreg((31 << 11) | 4);
    if ((threadIdx.x & 63) == 0) s_simd[threadIdx.x >> 6] = (int)((hw >> 4) & 3u);
    if (threadIdx.x == 0) s_simd[4] = (int)((hw >> 16) & 3u);
  }
  __syncthreads();
  int lw = 0;
  for (int w = 3; w >= 0; --w)
    if (s_simd[w] == s_simd[4]) lw = w;
  // The zero slot that missing donors read (no tile writes it; the tile
  // loop's barriers order this before any level).
  if (!UP && threadIdx.x == 0) {
    if (VK != VK_NONE) s_v[LV_ZERO] = TV<VK>::zero();
    if (CNT) s_c[LV_ZERO] = (CT)0;
  }
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const TT T = tile_at(P, t, ntiles);
    // The thread index, opaque to the compiler once per tile: offsets derived
    // from it are recomputed per tile instead of held in registers (and
    // spilled) across the loop.
    int tid = (int)threadIdx.x;
    asm volatile("" : "+v"(tid));
    const int lane = tid & 63, wave = tid >> 6;
    // 1. Every global load of the tile that depends on nothing else, issued
    // together: the codes with a one-cell halo (off the grid: sinks), the
    // rain of the own cells, and in phase C the exit index of each halo
    // cell (used only where the halo cell drains into the tile).
    // Phase C reads, instead of the codes, the words phase A left for its
    // own cells (depth, donor masks, sink).
    uint32_t cv[NCU];
    if (UP) {
#pragma unroll
      for (int u = 0; u < NCU; ++u) {
        const int e = tid + u * HT;
        const int hr = e / HW, hc = e - (e / HW) * HW;
        const int64_t r = T.r0 + hr - 1, c = T.c0 + hc - 1;
        const bool in = e < NCODE && r >= 0 && r < nr && c >= 0 && c < nc;
        cv[u] = in ? (uint32_t)P.code[r * nc + c] : (uint32_t)SINK;
      }
    }
    uint32_t vmask = 0;  // bit k: own cell k lies on the grid
    RT rq[HK];
    uint32_t cw[HK];
#pragma unroll
    for (int k = 0; k < HK; ++k) {
      const int lr = wave + 4 * k;
      const bool ok = lr < T.h && lane < T.w;
      vmask |= ok ? 1u << k : 0u;
      const int64_t g = ok ? (T.r0 + lr) * nc + T.c0 + lane : 0;
      if (RAIN == RAIN_F32) rq[k] = P.rain32[g];
      else if (RAIN == RAIN_F64) rq[k] = P.rain64[g];
      else rq[k] = (RT)1;
      cw[k] = (!UP && ok) ? *cw_at<VK>(P, g) : 0u;
    }
    int hh_r = 0, hh_c = 0;
    uint32_t hnd = NONE;
    if (tid < NHALO) halo_pos(tid, hh_r, hh_c);
    if (!UP && tid < NHALO) {
      const int64_t r = T.r0 + hh_r - 1, c = T.c0 + hh_c - 1;
      if (r >= 0 && r < nr && c >= 0 && c < nc) hnd = P.node_of[r * nc + c];
    }
    if (UP) {
      for (int w = tid; w < HN / 2; w += HT) s_msk[w] = 0u;
      if (tid < 16) s_open[tid] = 0;
#pragma unroll
      for (int u = 0; u < NCU; ++u)
        if (tid + u * HT < NCODE) s_code[tid + u * HT] = (uint8_t)cv[u];
    } else if (tid < NEED_WORDS) {
      s_need[tid] = 0u;
    }
    // Sources: rain (unit rain: 1) and one cell each.
    double m_rain = 0.0, rmax = 0.0;
    bool nonfinite = false;
#pragma unroll
    for (int k = 0; k < HK; ++k) {
      const int i = (wave + 4 * k) * HC + lane;
      const bool ok = (vmask >> k) & 1u;
      const double r = (double)rq[k];
      if (UP) {
        nonfinite |= ok && !isfinite(r);
        if (ok && isfinite(r)) rmax = fmax(rmax, fabs(r));
        continue;  // phase A sums per exit (below), not per cell
      }
      m_rain += ok ? r : 0.0;
      if constexpr (VK == VK_FF) {
        const float hi = (float)rq[k];
        s_v[i] = ok ? ff{hi, RAIN == RAIN_F64 ? (float)((double)rq[k] - (double)hi) : 0.0f} : ff{0.0f, 0.0f};
      }
      if constexpr (VK == VK_F64) s_v[i] = ok ? (double)rq[k] : 0.0;
      if (CNT) s_c[i] = ok ? (CT)1 : (CT)0;
    }
    if (UP && nonfinite) set_status(P.status, FR_ERR_NONFINITE);
    __syncthreads();
    // 2. Own cells: receiver inside the tile or not; each cell marks itself
    // in its receiver's donor mask (bit n: the donor lies in direction n).
    // Halo cells that drain into the tile mark the out-of-tile bits.
    // (Phase C takes all of this, and step 3's depths, from the words.)
    uint32_t pd[HK];  // receiver or root (| PT_TERM once it is a root), depth << 16
    uint32_t smask = 0, xmask = 0;  // bit k: own cell k is a sink / an exit
    bool bad = false;
    uint32_t mk[HK];  // in-tile donors | out-of-tile donors << 8
    V hv = TV<VK>::zero();
    uint64_t hcnt = 0;
    if constexpr (!UP) {
#pragma unroll
      for (int k = 0; k < HK; ++k) {
        const int lr = wave + 4 * k;
        const bool ok = (vmask >> k) & 1u;
        const uint32_t L = cw[k] & 0xFFFu;
        mk[k] = ok ? (cw[k] >> 12) & 0xFFFFu : 0u;
        smask |= (ok && ((cw[k] >> 28) & 1u)) ? 1u << k : 0u;
        pd[k] = !ok ? PT_TERM : (L == CW_NOLEVEL ? 0u : (PT_TERM | (L << 16)));
        // The halo cells this cell takes water from.
        for (uint32_t m = mk[k] >> 8; m; m &= m - 1) {
          const int n = __builtin_ctz(m);
          const int h = halo_id(lr + 1 + nb_dr(n), lane + 1 + nb_dc(n));
          atomicOr(&s_need[h >> 5], 1u << (h & 31));
        }
      }
      __syncthreads();
      // Their forest totals, for the inlets.
      if (tid < NHALO && ((s_need[tid >> 5] >> (tid & 31)) & 1u)) {
        if (hnd < n_ex) {
          if constexpr (VK != VK_NONE) {
            // The exit's total and count, one 16-byte record.
            const ulonglong2 rec = *reinterpret_cast<const ulonglong2*>(tile_total_rec(P, hnd));
            if constexpr (VK == VK_FF)
              hv = ff{__uint_as_float((uint32_t)rec.x), __uint_as_float((uint32_t)(rec.x >> 32))};
            if constexpr (VK == VK_F64) hv = __longlong_as_double((long long)rec.x);
            if (CNT) hcnt = rec.y;
          } else {
            hcnt = P.ex_cnt[0][hnd];
          }
        } else {
          set_status(P.status, FR_ERR_BADCODE);  // inconsistent bookkeeping: never follow it
        }
      }
    }
    if constexpr (UP) {
#pragma unroll
    for (int k = 0; k < HK; ++k) {
      const int lr = wave + 4 * k;
      const int i = lr * HC + lane;
      const uint32_t cd = s_code[(lr + 1) * HW + lane + 1];
      bool sk = true, inside = false;
      int rcv = i;
      if ((vmask >> k) & 1u) {
        if (cd <= 7u) {
          const int tr = lr + nb_dr((int)cd), tc = lane + nb_dc((int)cd);
          const int64_t gr = T.r0 + tr, gc = T.c0 + tc;
          if (gr < 0 || gr >= nr || gc < 0 || gc >= nc) {
            bad = true;  // receiver off the grid: malformed, treated as a sink
          } else {
            sk = false;
            inside = tr >= 0 && tr < HR && tc >= 0 && tc < HC;
            if (inside) rcv = tr * HC + tc;
          }
        } else if (cd != SINK) {
          bad = true;
        }
        smask |= sk ? 1u << k : 0u;
        xmask |= (!sk && !inside) ? 1u << k : 0u;  // receiver in another tile
      }
      if (inside) atomicOr(&s_msk[rcv >> 1], (1u << (7 - cd)) << (16 * (rcv & 1)));
      pd[k] = inside ? ((uint32_t)rcv | (1u << 16)) : ((uint32_t)i | PT_TERM);
      s_x[i] = pd[k];
    }
    if (tid < NHALO) {
      const uint32_t cd = s_code[hh_r * HW + hh_c];
      if (cd <= 7u) {
        const int tr = hh_r - 1 + nb_dr((int)cd), tc = hh_c - 1 + nb_dc((int)cd);
        if (tr >= 0 && tr < T.h && tc >= 0 && tc < T.w) {
          const int rcv = tr * HC + tc;
          atomicOr(&s_msk[rcv >> 1], (1u << (8 + 7 - cd)) << (16 * (rcv & 1)));
        }
      }
    }
    if (bad) set_status(P.status, FR_ERR_BADCODE);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < HK; ++k) {
      const int i = (wave + 4 * k) * HC + lane;
      mk[k] = (vmask >> k) & 1u ? (s_msk[i >> 1] >> (16 * (i & 1))) & 0xFFFFu : 0u;
    }
    }  // phase A's step 2
    if (!UP) {
      // Phase C: the halo's forest totals into LDS over the masks (every
      // thread has read its own), then the inlets add their out-of-tile
      // donors' totals in neighbour order; the level histogram then takes
      // the masks' place.
      __syncthreads();
      if (tid < NHALO) {
        if (VK != VK_NONE) s_hv[tid] = hv;
        if (CNT) s_hc[tid] = (CT)hcnt;
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < HK; ++k) {
        if (!(mk[k] >> 8)) continue;
        const int lr = wave + 4 * k;
        const int i = lr * HC + lane;
        V v = TV<VK>::zero();
        uint32_t c = 0;
        if (VK != VK_NONE) v = s_v[i];
        if (CNT) c = s_c[i];
        uint32_t m = mk[k] >> 8;
        while (m) {
          const int n = __builtin_ctz(m);
          m &= m - 1;
          const int h = halo_id(lr + 1 + nb_dr(n), lane + 1 + nb_dc(n));
          if (VK != VK_NONE) v = TV<VK>::add(v, s_hv[h]);
          if (CNT) c += s_hc[h];
        }
        if (VK != VK_NONE) s_v[i] = v;
        if (CNT) s_c[i] = (CT)c;
      }
      __syncthreads();
      for (int w = tid; w < HN / 2; w += HT) s_lev[w] = 0u;
      __syncthreads();  // cleared before any wave counts into it (step 4)
    }
    // 3. Pointer jumping: after round j every pointer spans 2^(j+1) edges or
    // ends at a root; a path inside the tile has fewer than HN edges.
    if constexpr (UP)
    for (int j = 0; j <= 12; ++j) {
      uint32_t np[HK];
      bool open = false;
#pragma unroll
      for (int k = 0; k < HK; ++k) {
        np[k] = pd[k];
        if (!(pd[k] & PT_TERM)) {
          // Jump to the target's target, adding its depth.
          const uint32_t w = s_x[pd[k] & 0xFFFFu];
          np[k] = (w & 0xFFFFu) | ((pd[k] & 0xFFFF0000u) + (w & 0xFFFF0000u));
          open = true;
        }
      }
      if (__ballot(open) && lane == 0) s_open[j] = 1;
      __syncthreads();  // every read above is done (the masks' too)
      if (!s_open[j] || j == 12) break;  // uniform
#pragma unroll
      for (int k = 0; k < HK; ++k) {
        pd[k] = np[k];
        s_x[(wave + 4 * k) * HC + lane] = np[k];
      }
      __syncthreads();
    }
    // 4. Depths (a cell whose path never reaches a root lies on or above a
    // cycle: malformed codes); the level histogram of the cells with
    // in-tile donors; phase A: the roots of the inlets.
    uint32_t ls[HK];  // level | slot << 16 (level NO_LEVEL: nothing to do)
    int dmax = 0;
    bool cyc = false;
#pragma unroll
    for (int k = 0; k < HK; ++k) {
      const bool on = (vmask >> k) & 1u;
      const bool ok = on && (pd[k] & PT_TERM);
      const int L = (int)(pd[k] >> 16);
      cyc |= on && !(pd[k] & PT_TERM);
      if (ok) dmax = max(dmax, L);
      ls[k] = NO_LEVEL;
      if (!UP && ok && (mk[k] & 0xFFu)) {
        const uint32_t old = atomicAdd(&s_lev[L >> 1], 1u << (16 * (L & 1)));
        ls[k] = (uint32_t)L | (((old >> (16 * (L & 1))) & 0xFFFFu) << 16);
      }
      if (UP && on) {
        // The cell's word for phase C.
        const uint32_t lw = (pd[k] & PT_TERM) ? (uint32_t)L : CW_NOLEVEL;
        *cw_at<VK>(P, (T.r0 + wave + 4 * k) * nc + T.c0 + lane) =
            lw | (mk[k] << 12) | (((smask >> k) & 1u) << 28);
      }
      if (UP && on && (mk[k] >> 8)) {
        uint32_t rt = NONE;
        if (pd[k] & PT_TERM) {
          const int p = (int)(pd[k] & 0x7FFFu);
          rt = (uint32_t)((T.r0 + p / HC) * nc + T.c0 + (p % HC));
        }
        P.root_of[(T.r0 + wave + 4 * k) * nc + T.c0 + lane] = rt;
      }
    }
    if (UP && cyc) set_status(P.status, FR_ERR_NOTDAG);
    dmax = wave_max(dmax);
    if (lane == 0) s_int[wave] = dmax;
    __syncthreads();
    if constexpr (!UP) {
    const int D = max(max(s_int[0], s_int[1]), max(s_int[2], s_int[3]));
    // 5. Level offsets (exclusive prefix sums, 8 levels per thread).
    uint32_t hl[8], run = 0;
    {
      const uint4 w4 = reinterpret_cast<const uint4*>(s_lev)[tid];
      const uint32_t ws[4] = {w4.x, w4.y, w4.z, w4.w};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        hl[2 * q] = run;
        run += ws[q] & 0xFFFFu;
        hl[2 * q + 1] = run;
        run += ws[q] >> 16;
      }
    }
    uint32_t incl = run;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = (uint32_t)__shfl_up((int)incl, o, 64);
      if (lane >= o) incl += y;
    }
    if (lane == 63) s_int[8 + wave] = (int)incl;
    __syncthreads();
    {
      uint32_t base = incl - run;
      for (int w = 0; w < wave; ++w) base += (uint32_t)s_int[8 + w];
      uint4 o4;
      o4.x = (base + hl[0]) | ((base + hl[1]) << 16);
      o4.y = (base + hl[2]) | ((base + hl[3]) << 16);
      o4.z = (base + hl[4]) | ((base + hl[5]) << 16);
      o4.w = (base + hl[6]) | ((base + hl[7]) << 16);
      reinterpret_cast<uint4*>(s_lev)[tid] = o4;  // every histogram read is done
    }
    __syncthreads();
    // 6. The cells with in-tile donors, in level order.
#pragma unroll
    for (int k = 0; k < HK; ++k) {
      if ((ls[k] & 0xFFFFu) != NO_LEVEL) {
        const int i = (wave + 4 * k) * HC + lane;
        s_x[s_off[ls[k] & 0xFFFFu] + (ls[k] >> 16)] = level_entry(i, mk[k] & 0xFFu);
      }
    }
    __syncthreads();
    // 7. Levels, deepest first, on one wavefront alone: a cell's in-tile
    // donors are one level deeper and final.  The LDS processes one
    // wavefront's instructions in order, so a level's reads see the previous
    // level's writes with no barrier or wait between them (the compiler is
    // only kept from moving LDS accesses across levels); the next level's
    // entries are read a level ahead.
    if (wave == lw && D > 0) {
      // Level L spans entries [off[L], off[L + 1]); offsets are read two
      // levels ahead, entries one, unconditionally (clamped indexes; off[0]
      // is 0), so that no branch keeps the compiler from leaving them in
      // flight.
      int o1 = s_off[D], o0 = s_off[D - 1], n0 = s_off[max(D - 2, 0)];
      uint32_t e = s_x[min(o0 + lane, HN - 1)];
      for (int L = D - 1; L >= 0; --L) {
        const int nn0 = s_off[max(L - 2, 0)];
        const uint32_t ne = s_x[min(n0 + lane, HN - 1)];
        if (lane < o1 - o0) level_cell<VK, CNT, CT>(s_v, s_c, e);
        for (int j = o0 + 64 + lane; j < o1; j += 64) level_cell<VK, CNT, CT>(s_v, s_c, s_x[j]);  // wide levels
        __builtin_amdgcn_wave_barrier();
        e = ne;
        o1 = o0;
        o0 = n0;
        n0 = nn0;
      }
    }
    __syncthreads();
    }  // phase C's levels
    if (UP) {
      // 8a. Phase A needs only each exit's upstream sum, not every cell's
      // value: the cells whose root is an exit add their rain to it, in a
      // 128-bit fixed point whose unit 2^Et follows from the tile's largest
      // |rain| (at most 2048 terms each below 2^113 units), with integer
      // atomics, so that the order of the additions changes no bit.  The
      // exits take consecutive slots of the list (one atomic per tile; slot
      // order inside the wavefront: cell k of every lane before cell k + 1
      // of any lane), and the sums are rounded back to float-float /
      // float64 once.
      const uint64_t lower = lane == 0 ? 0ull : (~0ull >> (64 - lane));
      uint32_t off[HK], wtot = 0;
#pragma unroll
      for (int k = 0; k < HK; ++k) {
        const uint64_t m = __ballot((xmask >> k) & 1u);
        off[k] = wtot + (uint32_t)__popcll(m & lower);
        wtot += (uint32_t)__popcll(m);
      }
      rmax = wave_max_d(rmax);
      if (lane == 0) {
        s_int[4 + wave] = (int)wtot;
        s_dbl[4 + wave] = rmax;
      }
      // Accumulators of the tile's exits (in the value and count area, which
      // phase A does not use otherwise) and the map cell -> exit slot (in the
      // histogram area).
      unsigned long long* acc_lo = reinterpret_cast<unsigned long long*>(s_buf);
      unsigned long long* acc_hi = acc_lo + D8T_MAX_EXITS;
      uint32_t* acc_c = reinterpret_cast<uint32_t*>(acc_hi + D8T_MAX_EXITS);
      uint16_t* s_map = reinterpret_cast<uint16_t*>(s_lev);
      if (tid < D8T_MAX_EXITS) {
        acc_lo[tid] = 0ull;
        acc_hi[tid] = 0ull;
        acc_c[tid] = 0u;
      }
      __syncthreads();
      uint32_t lbase = 0;
      for (int w = 0; w < wave; ++w) lbase += (uint32_t)s_int[4 + w];
#pragma unroll
      for (int k = 0; k < HK; ++k) {
        const int i = (wave + 4 * k) * HC + lane;
        s_map[i] = ((xmask >> k) & 1u) ? (uint16_t)(lbase + off[k]) : (uint16_t)0xFFFFu;
      }
      const double tmax = fmax(fmax(s_dbl[4], s_dbl[5]), fmax(s_dbl[6], s_dbl[7]));
      int et = 0;
      if (tmax > 0.0) (void)frexp(tmax, &et);  // tmax < 2^et
      const int Et = et + 11 + 2 - 126;
      __syncthreads();
#pragma unroll
      for (int k = 0; k < HK; ++k) {
        if (!((vmask >> k) & 1u) || !(pd[k] & PT_TERM)) continue;
        const uint32_t slot = s_map[pd[k] & 0x7FFFu];
        if (slot == 0xFFFFu) continue;  // drains to a sink inside the tile
        if (VK != VK_NONE) {
          const u128 x = (u128)fx_from(rq[k], Et);
          if (x != 0) {
            const unsigned long long xl = (unsigned long long)x, xh = (unsigned long long)(x >> 64);
            const unsigned long long old = atomicAdd(&acc_lo[slot], xl);
            const unsigned long long h = xh + ((old + xl < old) ? 1ull : 0ull);
            if (h) atomicAdd(&acc_hi[slot], h);
          }
        }
        if (CNT) atomicAdd(&acc_c[slot], 1u);
      }
      __syncthreads();
      float lmf = 0.0f;
      double lmd = 0.0;
      ff vf[HK];
      double vd[HK];
#pragma unroll
      for (int k = 0; k < HK; ++k) {
        vf[k] = ff{0.0f, 0.0f};
        vd[k] = 0.0;
        if (!((xmask >> k) & 1u)) continue;
        const uint32_t slot = lbase + off[k];
        const i128 v = (i128)(((u128)acc_hi[slot] << 64) | (u128)acc_lo[slot]);
        if constexpr (VK == VK_FF) {
          vf[k] = fx_to_ff(v, Et);
          lmf = fmaxf(lmf, fabsf(vf[k].hi));
        }
        if constexpr (VK == VK_F64) {
          vd[k] = fx_to_double(v, Et);
          lmd = fmax(lmd, fabs(vd[k]));
        }
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        lmf = fmaxf(lmf, __shfl_xor(lmf, o, 64));
        lmd = fmax(lmd, __shfl_xor(lmd, o, 64));
      }
      if (lane == 0) {
        s_flt[wave] = lmf;
        s_dbl[wave] = lmd;
      }
      __syncthreads();
      if (tid == 0) {
        const uint32_t tot = (uint32_t)(s_int[4] + s_int[5] + s_int[6] + s_int[7]);
        s_int[12] = tot ? (int)atomicAdd(P.n_exits, tot) : 0;
        if constexpr (VK == VK_FF) {
          const float m = fmaxf(fmaxf(s_flt[0], s_flt[1]), fmaxf(s_flt[2], s_flt[3]));
          if (m > 0.0f) atomicMax(&P.ctl->loc_max_f, __float_as_uint(m));
        }
        if constexpr (VK == VK_F64) {
          const double m = fmax(fmax(s_dbl[0], s_dbl[1]), fmax(s_dbl[2], s_dbl[3]));
          if (m > 0.0)
            atomicMax(reinterpret_cast<unsigned long long*>(&P.ctl->loc_max_d),
                      (unsigned long long)__double_as_longlong(m));
        }
      }
      __syncthreads();
      const uint32_t base = (uint32_t)s_int[12] + lbase;
#pragma unroll
      for (int k = 0; k < HK; ++k) {
        if (!((xmask >> k) & 1u)) continue;
        const int64_t g = (T.r0 + wave + 4 * k) * nc + T.c0 + lane;
        const uint32_t idx = base + off[k];
        if (idx < P.cap) {
          P.node_of[g] = idx;
          P.ex_cell[idx] = (uint32_t)g;
          if (!CNT) P.anc[1][idx] = 0u;  // the exit forest's child count (the link step adds)
          if constexpr (VK == VK_FF) {
            P.ex_hi[idx] = vf[k].hi;
            P.ex_lo[idx] = vf[k].lo;
          }
          if constexpr (VK == VK_F64) P.ex_d[idx] = vd[k];
          // With counts, the count sits above the exit forest's child count.
          if (CNT) P.ex_cnt[0][idx] = (uint64_t)acc_c[lbase + off[k]] << 32;
        }
      }
    } else {
      // 8b. Final values and the tile's {sum over sinks, sum of rain}.
      double m_sink = 0.0;
#pragma unroll
      for (int k = 0; k < HK; ++k) {
        if (!((vmask >> k) & 1u)) continue;
        const int i = (wave + 4 * k) * HC + lane;
        const int64_t g = (T.r0 + wave + 4 * k) * nc + T.c0 + lane;
        if constexpr (VK == VK_FF) {
          const ff v = s_v[i];
          if (P.q32) P.q32[g] = v.hi + v.lo;
          if ((smask >> k) & 1u) m_sink += TV<VK>::mass(v);
        }
        if constexpr (VK == VK_F64) {
          const double v = s_v[i];
          if (P.q64) P.q64[g] = v;
          if ((smask >> k) & 1u) m_sink += v;
        }
        if (CNT) P.cnt[g] = (uint64_t)s_c[i];
      }
      if (P.mass_part) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
          m_sink += __shfl_xor(m_sink, o, 64);
          m_rain += __shfl_xor(m_rain, o, 64);
        }
        if (lane == 0) {
          s_dbl[2 * wave] = m_sink;
          s_dbl[2 * wave + 1] = m_rain;
        }
        __syncthreads();
        if (tid == 0) {
          P.mass_part[2 * (int64_t)T.id] = (s_dbl[0] + s_dbl[2]) + (s_dbl[4] + s_dbl[6]);
          P.mass_part[2 * (int64_t)T.id + 1] = (s_dbl[1] + s_dbl[3]) + (s_dbl[5] + s_dbl[7]);
        }
      }
    }
    __syncthreads();  // the next tile reuses every LDS array
  }
}

// The gate: the tile-forest path serves the call when the row sweeps' exit
// list overflowed (or the caller chose it: `force`).  It starts from a clean
// forest state (its own exit count and round flags are separate words; the
// fixed-point unit is re-derived) and closes the engine's gate again.
__global__ void k_d8t_gate(CallCtl* C, int force) {
  if (threadIdx.x == 0 && (force || C->fallback)) {
    C->d8_tiles = 1;
    C->fallback = 0;
    C->loc_max_f = 0u;
    C->loc_max_d = 0ull;
  }
}

// The probe: rows 32, 96, 160, ... (row 0 on grids of fewer rows); every
// workgroup adds its count once.
constexpr int PROBE_STRIDE = 64;
__global__ __launch_bounds__(256) void k_d8_probe(D8Params P) {
  const int64_t nc = P.ncols;
  const int64_t nsr = P.nrows > PROBE_STRIDE / 2 ? (P.nrows - PROBE_STRIDE / 2 + PROBE_STRIDE - 1) / PROBE_STRIDE : 1;
  const int64_t total = nsr * nc;
  uint32_t cnt = 0;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total; k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t sr = k / nc;
    const int64_t r = P.nrows > PROBE_STRIDE / 2 ? PROBE_STRIDE / 2 + sr * PROBE_STRIDE : 0;
    const uint32_t cd = P.code[r * nc + (k - sr * nc)];
    cnt += (cd >= 3u && cd <= 7u) ? 1u : 0u;
  }
  __shared__ uint32_t s_cnt;
  if (threadIdx.x == 0) s_cnt = 0u;
  __syncthreads();
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) cnt += (uint32_t)__shfl_xor((int)cnt, o, 64);
  if ((threadIdx.x & 63) == 0 && cnt) atomicAdd(&s_cnt, cnt);
  __syncthreads();
  if (threadIdx.x == 0 && s_cnt) atomicAdd(&P.ctl->probe_cnt, s_cnt);
}

// Predicted exits above the limit: mark the list overflowed, so that the
// row sweeps return at once and the tile forest serves the call.
__global__ void k_d8_probe_decide(D8Params P, uint64_t sampled, double limit) {
  if (threadIdx.x != 0) return;
  const double est = (double)P.ctl->probe_cnt * ((double)(P.nrows * P.ncols) / (double)sampled);
  if (est > limit) *P.n_exits = P.cap + 1u;
}

// Mass-balance partials of the tiles, first stage: each workgroup sums a
// fixed run of D8T_MASS_RUN tiles in a fixed order.
__global__ __launch_bounds__(256) void k_d8t_mass(const double* part, int ntiles, double* out, const CallCtl* C) {
  if (__hip_atomic_load(&C->d8_tiles, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) return;
  __shared__ double rs[256], rt[256];
  const int b0 = blockIdx.x * D8T_MASS_RUN;
  const int b1 = min(ntiles, b0 + D8T_MASS_RUN);
  double s = 0.0, t = 0.0;
  for (int b = b0 + threadIdx.x; b < b1; b += 256) {
    s += part[2 * (int64_t)b];
    t += part[2 * (int64_t)b + 1];
  }
  rs[threadIdx.x] = s;
  rt[threadIdx.x] = t;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      rs[threadIdx.x] += rs[threadIdx.x + w];
      rt[threadIdx.x] += rt[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[2 * blockIdx.x] = rs[0];
    out[2 * blockIdx.x + 1] = rt[0];
  }
}

// Workgroups of a tile launch: as many as fit on the device at once (a
// multiple of 8, for the XCD mapping), at most one per tile.
template <bool UP, int VK, bool CNT, int RAIN>
int d8t_grid(int ntiles) {
  static int resident = 0;
  if (resident == 0) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_d8t<UP, VK, CNT, RAIN>, HT, 0) != hipSuccess ||
        cus <= 0 || per <= 0) {
      cus = 256;
      per = 2;
    }
    resident = cus * per;
  }
  int g = resident < ntiles ? resident : ntiles;
  if (g >= 8) g -= g % 8;
  return g < 1 ? 1 : g;
}

template <bool UP, int VK, bool CNT, int RAIN>
void d8t_launch(const D8Params& P, int ntiles, hipStream_t s) {
  hipLaunchKernelGGL((k_d8t<UP, VK, CNT, RAIN>), dim3((unsigned)d8t_grid<UP, VK, CNT, RAIN>(ntiles)), dim3(HT), 0,
                     s, P, ntiles);
}

template <bool UP, int VK, bool CNT>
void d8t_rain(const D8Params& P, int ntiles, hipStream_t s) {
  if (VK == VK_NONE || (!P.rain32 && !P.rain64)) d8t_launch<UP, VK, CNT, RAIN_UNIT>(P, ntiles, s);
  else if (P.rain32) d8t_launch<UP, VK, CNT, RAIN_F32>(P, ntiles, s);
  else d8t_launch<UP, VK, CNT, RAIN_F64>(P, ntiles, s);
}

template <bool UP>
void d8t_dispatch(ValKind vk, bool cnt, const D8Params& P, int ntiles, hipStream_t s) {
  if (vk == VK_FF) {
    if (cnt) d8t_rain<UP, VK_FF, true>(P, ntiles, s);
    else d8t_rain<UP, VK_FF, false>(P, ntiles, s);
  } else if (vk == VK_F64) {
    if (cnt) d8t_rain<UP, VK_F64, true>(P, ntiles, s);
    else d8t_rain<UP, VK_F64, false>(P, ntiles, s);
  } else {
    d8t_rain<UP, VK_NONE, true>(P, ntiles, s);
  }
}

}  // namespace

int64_t d8t_tiles(int64_t nrows, int64_t ncols) {
  return ((nrows + D8T_ROWS - 1) / D8T_ROWS) * ((ncols + D8T_COLS - 1) / D8T_COLS);
}

// Cells that can be exits: those on a tile's perimeter (every cell of a tile
// one cell high or wide).
uint64_t d8t_exit_bound(int64_t nrows, int64_t ncols) {
  auto per = [](int64_t h, int64_t w) -> uint64_t {
    return (uint64_t)(h <= 2 || w <= 2 ? h * w : 2 * (h + w) - 4);
  };
  const int64_t fr = nrows / D8T_ROWS, fc = ncols / D8T_COLS;
  const int64_t hr = nrows % D8T_ROWS, hc = ncols % D8T_COLS;
  uint64_t b = (uint64_t)(fr * fc) * per(D8T_ROWS, D8T_COLS);
  if (hr) b += (uint64_t)fc * per(hr, D8T_COLS);
  if (hc) b += (uint64_t)fr * per(D8T_ROWS, hc);
  if (hr && hc) b += per(hr, hc);
  return b;
}

size_t d8t_mass_words(int64_t nrows, int64_t ncols) {
  const int64_t nt = d8t_tiles(nrows, ncols);
  return (size_t)(2 * (nt + (nt + D8T_MASS_RUN - 1) / D8T_MASS_RUN));
}

hipError_t launch_d8_probe(const D8Params& P, double limit, hipStream_t s) {
  const int64_t nsr = P.nrows > PROBE_STRIDE / 2 ? (P.nrows - PROBE_STRIDE / 2 + PROBE_STRIDE - 1) / PROBE_STRIDE : 1;
  const int64_t total = nsr * P.ncols;
  int64_t b = (total + 255) / 256;
  if (b > 1024) b = 1024;
  hipLaunchKernelGGL(k_d8_probe, dim3((unsigned)(b < 1 ? 1 : b)), dim3(256), 0, s, P);
  hipLaunchKernelGGL(k_d8_probe_decide, dim3(1), dim3(64), 0, s, P, (uint64_t)(total > 0 ? total : 1), limit);
  return hipGetLastError();
}

hipError_t launch_d8t_gate(CallCtl* C, bool force, hipStream_t s) {
  hipLaunchKernelGGL(k_d8t_gate, dim3(1), dim3(64), 0, s, C, force ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_d8t(bool up, ValKind vk, bool cnt, const D8Params& P, hipStream_t s) {
  const int64_t nt = d8t_tiles(P.nrows, P.ncols);
  if (nt <= 0 || nt > 0x7FFFFFFF) return hipErrorInvalidValue;
  if (up) d8t_dispatch<true>(vk, cnt, P, (int)nt, s);
  else d8t_dispatch<false>(vk, cnt, P, (int)nt, s);
  return hipGetLastError();
}

hipError_t launch_d8t_mass(const double* part, int64_t ntiles, double* out, CallCtl* C, hipStream_t s) {
  const int64_t nb = (ntiles + D8T_MASS_RUN - 1) / D8T_MASS_RUN;
  double* stage = const_cast<double*>(part) + 2 * ntiles;
  hipLaunchKernelGGL(k_d8t_mass, dim3((unsigned)nb), dim3(256), 0, s, part, (int)ntiles, stage, C);
  if (hipGetLastError() != hipSuccess) return hipErrorLaunchFailure;
  return launch_mass_final_if(stage, (int)nb, out, &C->d8_tiles, s);
}

}  // namespace fr
