// Windowed wavefront sweep: general accumulation for any routing rule,
// forward (I - W^T) q = r or adjoint (I - W) rbar = qbar (Section 2.1,
// Section 2.2, Appendix A).
//
// The paper's sequential algorithm visits cells high-to-low so that every
// cell comes after all cells that feed it (Section 2.1); any order with that
// property gives the same solution (Section 3.2).  On terrain that drains
// mostly along one grid axis, visiting rows in flow order is almost such an
// order: a cell's inputs lie in the row visited before it, in its own row
// (chains resolved inside the row), or -- rarely, where the terrain locally
// rises against the row order -- in a row visited later.
//
// GPU mapping.  One wavefront owns a strip of 64 columns (lane = column) and
// visits the strip's rows in one direction.  Rows enter a ring of RING rows
// in LDS (state, value, MFD fractions).  A cell is computed once all of its
// inputs are final, by pulling them in fixed neighbour order, so results do
// not depend on timing.  Cells whose inputs are not yet final stay pending
// for up to WIN rows after their row entered; every newly final cell marks
// the neighbouring rows whose pending cells wait for it, which are then
// retried.  Columns next to a strip boundary read the neighbouring strip's
// edge cells from per-row records in HBM (written with device-coherent
// 64-bit stores of words that start out all ones, polled without blocking).
// No wavefront ever waits for another, so no schedule can hang.
//
// Cells still pending when their row leaves the window are left for a later
// pass; passes alternate the row direction and each one finishes at least
// the highest unfinished cell, so a valid DAG always completes and a pass
// that finishes nothing proves a cycle (FR_ERR_NOTDAG).  A pass marks the
// cells it leaves unfinished with a sentinel in a value array (NaN in the
// float-float low part or the float64 value, all ones in counts), so no
// separate done flags are stored.
//
// Precision: float-float (VK_FF, float32 output = hi), float64 (VK_F64),
// exact uint64 counts (CNT).  MFD fractions are computed as in the engine:
// float32 (s / s_max)^p via exp2/log2, or float64 pow.
#include <math.h>

#include "fr_internal.hpp"

namespace fr {
namespace {

constexpr int RING = 16;       // rows held in LDS
constexpr int WIN = RING - 2;  // rows that may still finish (plus one ahead, one behind)
constexpr int LW = 66;         // LDS row: side cell, 64 lanes, side cell
// Strips overlap: a wavefront computes 64 columns, owns the middle WS_OWN
// and recomputes GHOST columns of each neighbour (as GHOST columns of its
// own are recomputed by the neighbours).  A value handed across a strip
// boundary then reaches the other strip's owned columns only after passing
// 2 * GHOST columns, which along lateral flow takes as many rows: the
// exchange has that many rows of slack.
constexpr int GHOST = 8;
constexpr int WS_OWN = 64 - 2 * GHOST;
// Lanes whose cells the neighbours read as their side cells.
constexpr int REC_LANE_L = 2 * GHOST;    // read by the left neighbour's lane 63
constexpr int REC_LANE_R = WS_OWN - 1;   // read by the right neighbour's lane 0
// A strip does not start a row more than LEAD rows ahead of a neighbour
// (bounded wait), so neighbours stay within the exchange's slack.
constexpr int LEAD = 4;
constexpr int LEAD_SPIN = 1 << 14;  // polls before a neighbour counts as absent

constexpr uint32_t S_DONE = 1u << 8;
constexpr uint32_t S_PRIOR = 1u << 9;  // finished in an earlier pass

// ---------------------------------------------------------------------------
// Float-float arithmetic (Dekker 1971; Knuth TAOCP vol. 2, 4.2.2).
struct ff {
  float hi, lo;
};
__device__ __forceinline__ ff ff_two_sum(float a, float b) {
  const float s = a + b;
  const float bb = s - a;
  return {s, (a - (s - bb)) + (b - bb)};
}
__device__ __forceinline__ ff ff_fast_two_sum(float a, float b) {
  const float s = a + b;
  return {s, b - (s - a)};
}
__device__ __forceinline__ ff ff_add(ff x, ff y) {
  const ff s = ff_two_sum(x.hi, y.hi);
  return ff_fast_two_sum(s.hi, s.lo + (x.lo + y.lo));
}
__device__ __forceinline__ ff ff_mul_f(ff x, float f) {
  const float p = x.hi * f;
  return ff_fast_two_sum(p, fmaf(x.hi, f, -p) + x.lo * f);
}

__device__ constexpr float kInvSqrt2f = 0x1.6a09e6p-1f;
__device__ constexpr double kSqrt2 = 1.4142135623730950488;

template <int VK>
struct ValOf {
  using T = float;  // VK_NONE: unused placeholder
};
template <>
struct ValOf<VK_FF> {
  using T = ff;
};
template <>
struct ValOf<VK_F64> {
  using T = double;
};
template <int RK, int VK>
struct FracOf {
  using T = float;
};
template <>
struct FracOf<RK_MULTI, VK_F64> {
  using T = double;
};

__device__ __forceinline__ void vzero(float& v) { v = 0.0f; }
__device__ __forceinline__ void vzero(ff& v) { v = {0.0f, 0.0f}; }
__device__ __forceinline__ void vzero(double& v) { v = 0.0; }
__device__ __forceinline__ void vadd(float&, float) {}
__device__ __forceinline__ void vadd(ff& a, ff b) { a = ff_add(a, b); }
__device__ __forceinline__ void vadd(double& a, double b) { a += b; }
__device__ __forceinline__ float vmul(float v, float) { return v; }
__device__ __forceinline__ ff vmul(ff v, float f) { return ff_mul_f(v, f); }
__device__ __forceinline__ double vmul(double v, double f) { return v * f; }

// Lane shifts across the whole wavefront (DPP wave_shr:1 / wave_shl:1); the
// lane shifted in receives 0.
__device__ __forceinline__ uint32_t from_left(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x138, 0xF, 0xF, false);
}
__device__ __forceinline__ uint32_t from_right(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x130, 0xF, 0xF, false);
}
__device__ __forceinline__ float from_left(float x) { return __uint_as_float(from_left(__float_as_uint(x))); }
__device__ __forceinline__ float from_right(float x) { return __uint_as_float(from_right(__float_as_uint(x))); }
__device__ __forceinline__ uint64_t from_left(uint64_t x) {
  return ((uint64_t)from_left((uint32_t)(x >> 32)) << 32) | from_left((uint32_t)x);
}
__device__ __forceinline__ uint64_t from_right(uint64_t x) {
  return ((uint64_t)from_right((uint32_t)(x >> 32)) << 32) | from_right((uint32_t)x);
}
__device__ __forceinline__ double from_left(double x) {
  return __longlong_as_double((long long)from_left((uint64_t)__double_as_longlong(x)));
}
__device__ __forceinline__ double from_right(double x) {
  return __longlong_as_double((long long)from_right((uint64_t)__double_as_longlong(x)));
}
__device__ __forceinline__ ff from_left(ff x) { return {from_left(x.hi), from_left(x.lo)}; }
__device__ __forceinline__ ff from_right(ff x) { return {from_right(x.hi), from_right(x.lo)}; }

template <int RK>
__device__ __forceinline__ bool sends(uint32_t code, int k) {
  return RK == RK_SINGLE ? (code == (uint32_t)k) : (((code >> k) & 1u) != 0);
}

// Edge records: 64-bit payload words, initialised to all ones -- a pattern
// no payload takes (finite values and fractions, counts below 2^63).  Each
// word is written and read with one 64-bit atomic access, so a word that is
// no longer all ones holds its final payload.
constexpr uint64_t REC_EMPTY = ~0ull;
__device__ __forceinline__ void rec_put(uint64_t* p, uint64_t v) {
  __hip_atomic_store(reinterpret_cast<unsigned long long*>(p), (unsigned long long)v, __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t rec_get(const uint64_t* p) {
  return (uint64_t)__hip_atomic_load(reinterpret_cast<unsigned long long*>(const_cast<uint64_t*>(p)),
                                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void prog_put(int32_t* p, int32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int32_t prog_get(const int32_t* p) {
  return __hip_atomic_load(const_cast<int32_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t pack2(float a, float b) {
  return (uint64_t)__float_as_uint(a) | ((uint64_t)__float_as_uint(b) << 32);
}
__device__ __forceinline__ float lo_f(uint64_t w) { return __uint_as_float((uint32_t)w); }
__device__ __forceinline__ float hi_f(uint64_t w) { return __uint_as_float((uint32_t)(w >> 32)); }
__device__ __forceinline__ uint64_t dbits(double d) { return (uint64_t)__double_as_longlong(d); }
__device__ __forceinline__ double bitsd(uint64_t w) { return __longlong_as_double((long long)w); }

// Record words of a configuration: the value (one word, float-float packed)
// then, MFD forward, the three fractions toward the neighbouring column
// (float32: two words; float64: three); D8 forward with counts: the count.
template <int RK, int DK, int VK, bool CNT>
constexpr int rec_words() {
  return DK == DIR_ADJ ? 1
                       : (RK == RK_MULTI ? 1 + (VK == VK_F64 ? 3 : 2) : (VK != VK_NONE ? 1 : 0) + (CNT ? 1 : 0));
}
static_assert(rec_words<RK_MULTI, DIR_FWD, VK_F64, false>() <= WS_EW, "edge record too small");

template <int RK, int VK, bool CNT>
struct WsShared {
  using V = typename ValOf<VK>::T;
  using F = typename FracOf<RK, VK>::T;
  uint32_t st[RING][LW];   // bits 0-7 routing code, S_DONE, S_PRIOR
  uint8_t miss[RING][LW];  // pending cells: directions of inputs not yet final
  V val[RING][LW];         // final value, or the source term while pending
  uint64_t cnt[CNT ? RING : 1][LW];
  F frac[RK == RK_MULTI ? RING : 1][8][LW];  // MFD: fraction sent in direction k
};

// One row of geometry for this lane: own cell and (lanes 0, 63) the cell
// across the strip boundary.
struct Geo {
  uint32_t code, scode;
  float z, sz;
};

template <int VK>
struct Src {
  typename ValOf<VK>::T v;
  uint64_t n;
  bool prior;
};

// Orders this wavefront's LDS accesses across lanes.  One wavefront per
// workgroup executes its LDS instructions in order, so only the compiler
// must not move accesses across this point; no wait for global memory.
__device__ __forceinline__ void lds_sync() { asm volatile("" ::: "memory"); }

template <int RK, int DK, int VK, bool CNT>
__global__ __launch_bounds__(64) void k_ws_pass(WsParams P, int dir, int first) {
  using V = typename ValOf<VK>::T;
  using F = typename FracOf<RK, VK>::T;
  constexpr int EWN = rec_words<RK, DK, VK, CNT>();
  constexpr uint32_t NOC = RK == RK_SINGLE ? (uint32_t)SINK : 0u;
  __shared__ WsShared<RK, VK, CNT> S;

  const int lane = threadIdx.x;
  const int li = lane + 1;
  const int64_t strip = blockIdx.x;
  const int64_t nr = P.nrows, nc = P.ncols;
  const int64_t c = strip * WS_OWN - GHOST + lane;
  const bool live = c >= 0 && c < nc;
  const bool owned = live && lane >= GHOST && lane < GHOST + WS_OWN;
  const bool sideL = lane == 0 && c - 1 >= 0 && c - 1 < nc;
  const bool sideR = lane == 63 && c + 1 >= 0 && c + 1 < nc;
  const bool has_side = sideL || sideR;
  const bool edge_lane = lane == 0 || lane == 63;
  // This lane publishes its cells for a neighbour's edge lane.
  const int64_t nstrips = (nc + WS_OWN - 1) / WS_OWN;
  const bool has_record = live && ((lane == REC_LANE_L && strip > 0) || (lane == REC_LANE_R && strip + 1 < nstrips));
  const int64_t cs = lane == 0 ? c - 1 : c + 1;
  const int sidx = lane == 0 ? 0 : LW - 1;
  // Records this lane writes (its strip's edge) and reads (the neighbour's).
  const int my_side = lane == REC_LANE_L ? 0 : 1;
  const int64_t rd_strip = lane == 0 ? strip - 1 : strip + 1;
  const int rd_side = lane == 0 ? 1 : 0;
  const float pf = (float)P.p;

  auto row_of = [&](int64_t t) -> int64_t { return dir < 0 ? nr - 1 - t : t; };

  auto load_geo = [&](int64_t t) -> Geo {
    Geo g{NOC, NOC, INFINITY, INFINITY};
    if (t < 0 || t >= nr) return g;
    const int64_t rb = row_of(t) * nc;
    if (live) {
      g.code = P.code[rb + c];
      if (RK == RK_MULTI) g.z = P.z[rb + c];
    }
    if (has_side) {
      g.scode = P.code[rb + cs];
      if (RK == RK_MULTI) g.sz = P.z[rb + cs];
    }
    return g;
  };

  auto load_src = [&](int64_t t) -> Src<VK> {
    Src<VK> s;
    vzero(s.v);
    s.n = 1;
    s.prior = false;
    if (t < 0 || t >= nr || !live) return s;
    const int64_t i = row_of(t) * nc + c;
    if constexpr (VK == VK_FF) {
      if (P.src64) {
        const double d = P.src64[i];
        s.v.hi = (float)d;
        s.v.lo = (float)(d - (double)s.v.hi);
      } else {
        s.v = {P.src32 ? P.src32[i] : 1.0f, 0.0f};
      }
      if (!first) {
        const float lo = P.vlo[i];
        if (!isnan(lo)) {
          s.v = {P.vhi[i], lo};
          s.prior = true;
        }
      }
    } else if constexpr (VK == VK_F64) {
      s.v = P.src64 ? P.src64[i] : (P.src32 ? (double)P.src32[i] : 1.0);
      if (!first) {
        const double y = P.v64[i];
        if (!isnan(y)) {
          s.v = y;
          s.prior = true;
        }
      }
    } else {
      if (CNT && !first && P.cnt[i] != ~0ull) s.prior = true;
    }
    if (CNT && s.prior) s.n = P.cnt[i];
    return s;
  };

  bool bad = false, nonfinite = false;
  uint32_t n_wait = 0, n_pace = 0, n_resolve = 0;  // diagnostics

  // A row enters its slot: state, source term, MFD fractions (from the rows
  // at steps y-1, y, y+1) and the side cells' codes.
  auto enter_row = [&](int64_t y, const Geo& ga, const Geo& gb, const Geo& gc, const Src<VK>& sr) {
    const int sb = (int)(y & (RING - 1));
    const uint32_t code = gb.code;
    if constexpr (RK == RK_MULTI) {
      const Geo& gu = dir < 0 ? gc : ga;  // grid row r - 1
      const Geo& gd = dir < 0 ? ga : gc;  // grid row r + 1
      float zn[8];
      zn[0] = from_left(gu.z);
      zn[1] = gu.z;
      zn[2] = from_right(gu.z);
      zn[3] = from_left(gb.z);
      zn[4] = from_right(gb.z);
      zn[5] = from_left(gd.z);
      zn[6] = gd.z;
      zn[7] = from_right(gd.z);
      if (lane == 0) {
        zn[0] = sideL ? gu.sz : INFINITY;
        zn[3] = sideL ? gb.sz : INFINITY;
        zn[5] = sideL ? gd.sz : INFINITY;
      }
      if (lane == 63) {
        zn[2] = sideR ? gu.sz : INFINITY;
        zn[4] = sideR ? gb.sz : INFINITY;
        zn[7] = sideR ? gd.sz : INFINITY;
      }
      const float zi = gb.z;
      if (live && !isfinite(zi)) nonfinite = true;
      F fr[8];
      if constexpr (VK == VK_F64) {
        double w[8], sum = 0.0;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          w[k] = 0.0;
          if (!live || !sends<RK>(code, k)) continue;
          if (!(zn[k] < zi)) {
            bad = true;
            continue;
          }
          const double sl = ((double)zi - (double)zn[k]) / (nb_diag(k) ? kSqrt2 : 1.0);
          w[k] = pow(sl, P.p);
          sum += w[k];
        }
        const double iw = sum > 0.0 ? 1.0 / sum : 0.0;
#pragma unroll
        for (int k = 0; k < 8; ++k) fr[k] = w[k] * iw;
      } else {
        float sl[8], smax = 0.0f;
        bool rcv[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          sl[k] = 0.0f;
          rcv[k] = false;
          if (!live || !sends<RK>(code, k)) continue;
          if (!(zn[k] < zi)) {
            bad = true;
            continue;
          }
          rcv[k] = true;
          const float drop = zi - zn[k];
          sl[k] = nb_diag(k) ? drop * kInvSqrt2f : drop;
          smax = sl[k] > smax ? sl[k] : smax;
        }
        const float rs = smax > 0.0f ? 1.0f / smax : 0.0f;
        float tk[8], sum = 0.0f;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          tk[k] = rcv[k] ? exp2f(pf * log2f(sl[k] * rs)) : 0.0f;
          sum += tk[k];
        }
        const float iw = sum > 0.0f ? 1.0f / sum : 0.0f;
#pragma unroll
        for (int k = 0; k < 8; ++k) fr[k] = tk[k] * iw;
      }
#pragma unroll
      for (int k = 0; k < 8; ++k) S.frac[sb][k][li] = fr[k];
    } else {
      if (live && code != SINK) {
        if (code > 7) {
          bad = true;
        } else {
          const int k = (int)code;
          const int64_t rr = row_of(y) + nb_dr(k), cc = c + nb_dc(k);
          if (rr < 0 || rr >= nr || cc < 0 || cc >= nc) bad = true;
        }
      }
    }
    if constexpr (VK == VK_FF) {
      if (live && !isfinite(sr.v.hi)) nonfinite = true;
    } else if constexpr (VK == VK_F64) {
      if (live && !isfinite(sr.v)) nonfinite = true;
    }
    uint32_t st = live ? (code & 0xFFu) : (NOC | S_DONE);
    if (live && sr.prior) st |= S_DONE | S_PRIOR;
    S.st[sb][li] = st;
    S.miss[sb][li] = 0;
    V v = sr.v;
    if (!live) vzero(v);
    S.val[sb][li] = v;
    if constexpr (CNT) S.cnt[sb][li] = live ? sr.n : 0;
    if (edge_lane) {
      S.st[sb][sidx] = has_side ? (gb.scode & 0xFFu) : (NOC | S_DONE);
      V v0;
      vzero(v0);
      S.val[sb][sidx] = v0;
      if constexpr (CNT) S.cnt[sb][sidx] = 0;
      if constexpr (RK == RK_MULTI) {
#pragma unroll
        for (int k = 0; k < 8; ++k) S.frac[sb][k][sidx] = (F)0;
      }
    }
  };

  // Forward: whether a row's side cell gives water to this strip's edge
  // column (directions from the side cell toward it).
  auto side_gives = [&](uint32_t scode) -> bool {
    if (!has_side) return false;
    if (lane == 0) return sends<RK>(scode, 2) || sends<RK>(scode, 4) || sends<RK>(scode, 7);
    return sends<RK>(scode, 0) || sends<RK>(scode, 3) || sends<RK>(scode, 5);
  };
  // Adjoint: the side cells (as steps relative to the edge cell's step) that
  // the edge cell gives water to, as bits 0 (step - 1), 1 (same), 2 (step + 1).
  auto own_gives_side = [&](uint32_t code) -> uint32_t {
    if (!has_side) return 0u;
    const int ka = lane == 0 ? 0 : 2, kb = lane == 0 ? 3 : 4, kc = lane == 0 ? 5 : 7;
    // Grid row offsets -1, 0, +1 map to step offsets -dir, 0, +dir.
    const uint32_t up = sends<RK>(code, ka) ? 1u : 0u, mid = sends<RK>(code, kb) ? 1u : 0u,
                   dn = sends<RK>(code, kc) ? 1u : 0u;
    return dir < 0 ? (dn | (mid << 1) | (up << 2)) : (up | (mid << 1) | (dn << 2));
  };

  // Publishes a newly final edge cell for the neighbouring strip.
  auto put_record = [&](int64_t x, int sb, const V& v, uint64_t n) {
    uint64_t* rec = P.edge + ((strip * nr + row_of(x)) * 2 + my_side) * WS_EW;
    int w = 0;
    if constexpr (VK == VK_FF) rec_put(rec + w++, pack2(v.hi, v.lo));
    else if constexpr (VK == VK_F64) rec_put(rec + w++, dbits(v));
    if constexpr (DK == DIR_FWD && RK == RK_MULTI) {
      // Fractions toward the neighbouring column, grid rows r-1, r, r+1.
      const F f0 = S.frac[sb][my_side == 0 ? 0 : 2][li];
      const F f1 = S.frac[sb][my_side == 0 ? 3 : 4][li];
      const F f2 = S.frac[sb][my_side == 0 ? 5 : 7][li];
      if constexpr (VK == VK_F64) {
        rec_put(rec + w++, dbits(f0));
        rec_put(rec + w++, dbits(f1));
        rec_put(rec + w++, dbits(f2));
      } else {
        rec_put(rec + w++, pack2(f0, f1));
        rec_put(rec + w++, pack2(f2, 0.0f));
      }
    }
    if constexpr (DK == DIR_FWD && RK == RK_SINGLE && CNT) rec_put(rec + w++, n);
    (void)n;
  };

  // Tries to finish the pending cells of the row at step x (slot sb).
  // Returns the lanes finished.
  auto resolve = [&](int64_t x, int sb) -> uint64_t {
    const uint32_t me = S.st[sb][li];
    const bool pend = !(me & S_DONE);
    const uint32_t code = me & 0xFFu;
    V acc = S.val[sb][li];
    uint64_t accn = CNT ? S.cnt[sb][li] : 0;
    bool ok = pend;
    uint32_t miss = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if (k == 3 || k == 4) continue;
      const int64_t xn = x + nb_dr(k) * dir;
      if (xn < 0 || xn >= nr) continue;
      const int sn = (int)(xn & (RING - 1));
      const int ln = li + nb_dc(k);
      const uint32_t sj = S.st[sn][ln];
      const bool input = pend && (DK == DIR_FWD ? sends<RK>(sj & 0xFFu, 7 - k) : sends<RK>(code, k));
      if (!input) continue;
      if (!(sj & S_DONE)) {
        ok = false;
        miss |= 1u << k;
        continue;
      }
      if constexpr (VK != VK_NONE) {
        V vj = S.val[sn][ln];
        if constexpr (RK == RK_MULTI) vj = vmul(vj, DK == DIR_FWD ? S.frac[sn][7 - k][ln] : S.frac[sb][k][li]);
        vadd(acc, vj);
      }
      if constexpr (CNT) accn += S.cnt[sn][ln];
    }
    // Same-row inputs, iterated along the row with lane shifts.
    const uint32_t sl = S.st[sb][li - 1], sr = S.st[sb][li + 1];
    const bool in_l = pend && (DK == DIR_FWD ? sends<RK>(sl & 0xFFu, 4) : sends<RK>(code, 3));
    const bool in_r = pend && (DK == DIR_FWD ? sends<RK>(sr & 0xFFu, 3) : sends<RK>(code, 4));
    F fl = (F)1, fr_ = (F)1;
    if constexpr (RK == RK_MULTI) {
      fl = DK == DIR_FWD ? S.frac[sb][4][li - 1] : S.frac[sb][3][li];
      fr_ = DK == DIR_FWD ? S.frac[sb][3][li + 1] : S.frac[sb][4][li];
    }
    // Side cells of lanes 0 and 63 (another strip) come from LDS.
    bool dside = false;
    V vside;
    vzero(vside);
    uint64_t nside = 0;
    if (edge_lane) {
      dside = ((lane == 0 ? sl : sr) & S_DONE) != 0;
      vside = S.val[sb][sidx];
      if constexpr (CNT) nside = S.cnt[sb][sidx];
    }
    uint32_t cd = pend ? 0u : 1u;
    V cv = S.val[sb][li];
    uint64_t cn = CNT ? S.cnt[sb][li] : 0;
    bool newly = false, dl = false, dr = false;
    for (int it = 0; it < 66; ++it) {
      dl = from_left(cd) != 0;
      dr = from_right(cd) != 0;
      V vl = from_left(cv), vr = from_right(cv);
      uint64_t nl = 0, nrr = 0;
      if constexpr (CNT) {
        nl = from_left(cn);
        nrr = from_right(cn);
      }
      if (lane == 0) {
        dl = dside;
        vl = vside;
        nl = nside;
      }
      if (lane == 63) {
        dr = dside;
        vr = vside;
        nrr = nside;
      }
      const bool can = ok && !cd && (!in_l || dl) && (!in_r || dr);
      if (can) {
        V w = acc;
        uint64_t wn = accn;
        if (in_l) {
          if constexpr (RK == RK_MULTI) vadd(w, vmul(vl, fl));
          else vadd(w, vl);
          wn += nl;
        }
        if (in_r) {
          if constexpr (RK == RK_MULTI) vadd(w, vmul(vr, fr_));
          else vadd(w, vr);
          wn += nrr;
        }
        cv = w;
        cn = wn;
        cd = 1u;
        newly = true;
      }
      if (__ballot(can) == 0) break;
    }
    if (newly) {
      S.st[sb][li] = me | S_DONE;
      S.val[sb][li] = cv;
      if constexpr (CNT) S.cnt[sb][li] = cn;
      if (has_record) put_record(x, sb, cv, cn);
    } else if (pend) {
      if (in_l && !dl) miss |= 1u << 3;
      if (in_r && !dr) miss |= 1u << 4;
      S.miss[sb][li] = (uint8_t)miss;
    }
    return __ballot(newly);
  };

  // Whether pending cells of row y wait for cells of row x finished in D.
  auto affected = [&](int64_t y, int64_t x, uint64_t D) -> bool {
    const int sy = (int)(y & (RING - 1));
    const uint32_t m = S.miss[sy][li];
    const bool pend = !(S.st[sy][li] & S_DONE);
    const int kb = ((x - y) * dir) < 0 ? 0 : 5;
    bool a = false;
    if (pend) {
      a = a || (((m >> kb) & 1u) && lane >= 1 && ((D >> (lane - 1)) & 1ull));
      a = a || (((m >> (kb + 1)) & 1u) && ((D >> lane) & 1ull));
      a = a || (((m >> (kb + 2)) & 1u) && lane <= 62 && ((D >> (lane + 1)) & 1ull));
    }
    return __ballot(a) != 0;
  };

  // pend_rows: a bit per slot whose row (in the window) has pending cells.
  // want (edge lanes): slots whose side cell is wanted and not yet final.
  uint32_t pend_rows = 0, want = 0, nfin = 0;

  // Polls in flight (edge lanes): step of the row polled, record words.
  // Wanted rows are polled round-robin, so rows whose side cell finishes
  // only in a later pass cannot starve the others.
  constexpr int NPOLL = 3;
  int64_t prow[NPOLL];
  uint64_t pw[NPOLL][EWN];
  int64_t pcur = 0;
#pragma unroll
  for (int p = 0; p < NPOLL; ++p) prow[p] = -1;

  auto issue_polls = [&](int64_t lo, int64_t hi) {
    int64_t x = (pcur < lo || pcur > hi) ? lo : pcur;
    int rem = want ? (int)(hi - lo + 1) : 0;
#pragma unroll
    for (int p = 0; p < NPOLL; ++p) {
      prow[p] = -1;
      while (rem > 0) {
        const int64_t y = x;
        x = (x == hi) ? lo : x + 1;
        --rem;
        if ((want >> (y & (RING - 1))) & 1u) {
          prow[p] = y;
          break;
        }
      }
      if (prow[p] < 0) continue;
      pcur = x;
      const uint64_t* rec = P.edge + ((rd_strip * nr + row_of(prow[p])) * 2 + rd_side) * WS_EW;
#pragma unroll
      for (int w = 0; w < EWN; ++w) pw[p][w] = rec_get(rec + w);
    }
  };

  // Moves arrived records into LDS; returns the slots to retry (rows
  // lo..hi whose edge cell waits for an arrived side cell).
  auto consume_polls = [&](int64_t lo, int64_t hi) -> uint32_t {
    uint32_t dirty = 0;
#pragma unroll
    for (int p = 0; p < NPOLL; ++p) {
      const int64_t x = prow[p];
      bool okp = x >= 0;
#pragma unroll
      for (int w = 0; w < EWN; ++w) okp = okp && pw[p][w] != REC_EMPTY;
      if (okp) {
        const int sx = (int)(x & (RING - 1));
        int w = 0;
        V v;
        vzero(v);
        if constexpr (VK == VK_FF) {
          v.hi = lo_f(pw[p][w]);
          v.lo = hi_f(pw[p][w]);
          ++w;
        } else if constexpr (VK == VK_F64) {
          v = bitsd(pw[p][w]);
          ++w;
        }
        S.val[sx][sidx] = v;
        if constexpr (DK == DIR_FWD && RK == RK_MULTI) {
          // The side cell's fractions toward this strip's edge column.
          F f0, f1, f2;
          if constexpr (VK == VK_F64) {
            f0 = bitsd(pw[p][w]);
            f1 = bitsd(pw[p][w + 1]);
            f2 = bitsd(pw[p][w + 2]);
            w += 3;
          } else {
            f0 = lo_f(pw[p][w]);
            f1 = hi_f(pw[p][w]);
            f2 = lo_f(pw[p][w + 1]);
            w += 2;
          }
          S.frac[sx][lane == 0 ? 2 : 0][sidx] = f0;
          S.frac[sx][lane == 0 ? 4 : 3][sidx] = f1;
          S.frac[sx][lane == 0 ? 7 : 5][sidx] = f2;
        }
        if constexpr (DK == DIR_FWD && RK == RK_SINGLE && CNT) S.cnt[sx][sidx] = pw[p][w++];
        S.st[sx][sidx] |= S_DONE;
        want &= ~(1u << sx);
#pragma unroll
        for (int d = -1; d <= 1; ++d) {
          const int64_t y = x + d;
          if (y < lo || y > hi) continue;
          const int sy = (int)(y & (RING - 1));
          // Direction from the edge cell at step y to the side cell at step x.
          const int dr = (int)((x - y) * dir);
          const int k = lane == 0 ? (dr < 0 ? 0 : (dr == 0 ? 3 : 5)) : (dr < 0 ? 2 : (dr == 0 ? 4 : 7));
          if (!(S.st[sy][li] & S_DONE) && ((S.miss[sy][li] >> k) & 1u)) dirty |= 1u << sy;
        }
      }
      prow[p] = -1;
    }
    return (uint32_t)__builtin_amdgcn_readlane((int)dirty, 0) | (uint32_t)__builtin_amdgcn_readlane((int)dirty, 63);
  };

  // Retries rows until nothing changes; window = steps lo..t.
  auto settle = [&](uint32_t dirty, int64_t lo, int64_t t) {
    while (dirty) {
      const int sb = __builtin_ctz(dirty);
      dirty &= dirty - 1;
      const int64_t x = t - (int64_t)((((int)(t & (RING - 1))) - sb) & (RING - 1));
      if (x < lo || !((pend_rows >> sb) & 1u)) continue;
      lds_sync();
      ++n_resolve;
      const uint64_t D = resolve(x, sb);
      lds_sync();
      const bool still = __ballot(!(S.st[sb][li] & S_DONE)) != 0;
      pend_rows = still ? (pend_rows | (1u << sb)) : (pend_rows & ~(1u << sb));
      if (D) {
#pragma unroll
        for (int d = -1; d <= 1; d += 2) {
          const int64_t y = x + d;
          if (y < lo || y > t) continue;
          const int sy = (int)(y & (RING - 1));
          if (((pend_rows >> sy) & 1u) && affected(y, x, D)) dirty |= 1u << sy;
        }
      }
    }
  };

  // Writes a row leaving the window to HBM; in the first pass unfinished
  // cells get the sentinel so a later pass can tell them apart.
  auto freeze = [&](int64_t f) {
    const int sf = (int)(f & (RING - 1));
    const uint32_t me = S.st[sf][li];
    pend_rows &= ~(1u << sf);
    if (!owned) return;
    const int64_t i = row_of(f) * nc + c;
    if ((me & S_DONE) && !(me & S_PRIOR)) {
      ++nfin;
      if constexpr (VK == VK_FF) {
        const ff v = S.val[sf][li];
        P.vhi[i] = v.hi;
        P.vlo[i] = v.lo;
      } else if constexpr (VK == VK_F64) {
        P.v64[i] = S.val[sf][li];
      }
      if constexpr (CNT) P.cnt[i] = S.cnt[sf][li];
    } else if ((first || P.debug) && !(me & S_DONE)) {
      if constexpr (VK == VK_FF) {
        P.vlo[i] = __uint_as_float(0x7FC00000u);
      } else if constexpr (VK == VK_F64) {
        const uint64_t tag = P.debug ? (((uint64_t)S.miss[sf][li] << 24) | (me & 0xFFFFFFu)) : 0ull;
        P.v64[i] = __longlong_as_double((long long)(0x7FF8000000000000ull | tag));
      } else if constexpr (CNT) {
        P.cnt[i] = ~0ull;
      }
    }
  };

  // Side rows wanted by the adjoint: set when the row that needs them has
  // entered; the bit for the step after the newest entered row waits here.
  uint32_t want_next = 0;
  auto mark_wanted = [&](int64_t y, uint32_t code, uint32_t scode) {
    const int sy = (int)(y & (RING - 1));
    if (DK == DIR_FWD) {
      if (side_gives(scode)) want |= 1u << sy;
    } else {
      const uint32_t g = own_gives_side(code);
      uint32_t w = (want_next || (g & 2u)) ? (1u << sy) : 0u;
      if ((g & 1u) && y >= 1) {
        const int sp = (int)((y - 1) & (RING - 1));
        if (!(S.st[sp][sidx] & S_DONE)) w |= 1u << sp;
      }
      want |= w;
      want_next = (g & 4u) ? 1u : 0u;
    }
  };

  // Bounded wait, before row f leaves the window, for side cells that its
  // edge cells still need; other strips are never waited for otherwise.
  auto wait_edges = [&](int64_t f, int64_t lo, int64_t t) {
    const int sf = (int)(f & (RING - 1));
    int idle = 0;
    for (int it = 0; it < 128 && idle < 16; ++it) {
      bool need = false;
      if (has_side && !(S.st[sf][li] & S_DONE)) need = (S.miss[sf][li] & (lane == 0 ? 0x29u : 0x94u)) != 0;
      if (__ballot(need) == 0) break;
      ++n_wait;
      issue_polls(lo, t);
      const uint32_t dirty = consume_polls(lo, t);
      if (dirty) {
        idle = 0;
        settle(dirty, lo, t);
      } else {
        ++idle;
        __builtin_amdgcn_s_sleep(4);
      }
    }
  };

  // ---- prologue: row 0 enters ---------------------------------------------
  Geo g0 = load_geo(0), g1 = load_geo(1), g2 = load_geo(2);
  Src<VK> s1 = load_src(1);
  {
    const Geo gm = load_geo(-1);
    const Src<VK> s0 = load_src(0);
    enter_row(0, gm, g0, g1, s0);
    if (__ballot(live && !s0.prior)) pend_rows |= 1u;
    mark_wanted(0, g0.code, g0.scode);
  }

  // Pacing: the neighbours' progress as last read (edge lanes), and whether
  // a neighbour stopped answering (then it is no longer waited for).
  const bool has_nb = (lane == 0 && strip > 0) || (lane == 63 && strip + 1 < nstrips);
  const int32_t* nb_prog = P.progress + (lane == 0 ? strip - 1 : strip + 1);
  int32_t nb_seen = -1;
  bool nb_absent = !has_nb;

  for (int64_t t = 0; t < nr; ++t) {
    // Wait while a neighbour is more than LEAD rows behind (nb_seen was
    // read at the start of the previous step).
    if (t > LEAD) {
      int spins = 0;
      for (;;) {
        const bool behind = !nb_absent && (int64_t)nb_seen < t - 1 - LEAD;
        if (__ballot(behind) == 0) break;
        ++n_pace;
        if (behind) {
          nb_seen = prog_get(nb_prog);
          if (++spins > LEAD_SPIN) nb_absent = true;
        }
        if ((int64_t)nb_seen < t - 1 - LEAD) __builtin_amdgcn_s_sleep(1);
      }
    }
    // Loads for later steps go out first, ahead of this step's stores, so
    // that waiting for them never waits for the stores as well.
    const Geo g3 = load_geo(t + 3);
    const Src<VK> s2 = load_src(t + 2);
    const int32_t nb_next = (has_nb && !nb_absent) ? prog_get(nb_prog) : nb_seen;
    const int64_t lo = t - (WIN - 1) > 0 ? t - (WIN - 1) : 0;
    // Polls issued in the previous step (their rows are still in LDS); the
    // next ones go out at once so that they complete during this step.
    uint32_t dirty = consume_polls(lo, t);
    issue_polls(lo, t);
    if (t + 1 < nr) {
      // Row t + 1 enters; its slot's old row left the window two steps ago.
      const int sn = (int)((t + 1) & (RING - 1));
      want &= ~(1u << sn);
      pend_rows &= ~(1u << sn);
      lds_sync();
      enter_row(t + 1, g0, g1, g2, s1);
      if (__ballot(live && !s1.prior)) pend_rows |= 1u << sn;
      mark_wanted(t + 1, g1.code, g1.scode);
    }
    dirty |= 1u << (t & (RING - 1));
    settle(dirty, lo, t);
    if (t - (WIN - 1) >= 0) {
      const int64_t f = t - (WIN - 1);
      if ((pend_rows >> (f & (RING - 1))) & 1u) {
        // Finish the polls in flight first: they are consumed here.
        dirty = consume_polls(lo, t);
        if (dirty) settle(dirty, lo, t);
        wait_edges(f, lo, t);
        issue_polls(lo, t);
      }
      lds_sync();
      freeze(f);
    }
    if (lane == 0) prog_put(P.progress + strip, (int32_t)t);
    nb_seen = nb_next;
    g0 = g1;
    g1 = g2;
    g2 = g3;
    s1 = s2;
  }

  // ---- drain: bounded wait for the last edge records ----------------------
  {
    const int64_t t = nr - 1;
    const int64_t lo = t - (WIN - 2) > 0 ? t - (WIN - 2) : 0;
    uint32_t dirty = consume_polls(lo, t);
    if (dirty) settle(dirty, lo, t);
    int idle = 0;
    for (int it = 0; it < 4096 && idle < 64; ++it) {
      const uint32_t pr = (uint32_t)__builtin_amdgcn_readfirstlane((int)pend_rows);
      const uint32_t wa = (uint32_t)__builtin_amdgcn_readlane((int)want, 0) |
                          (uint32_t)__builtin_amdgcn_readlane((int)want, 63);
      if (pr == 0 || wa == 0) break;
      issue_polls(lo, t);
      dirty = consume_polls(lo, t);
      if (dirty) {
        idle = 0;
        settle(dirty, lo, t);
      } else {
        ++idle;
        __builtin_amdgcn_s_sleep(8);
      }
    }
    lds_sync();
    for (int64_t f = lo; f <= t; ++f) freeze(f);
  }

  if (lane == 0) prog_put(P.progress + strip, (int32_t)nr + LEAD + 1);
  if (first && P.status) {
    if (bad) atomicCAS(P.status, 0, FR_ERR_BADCODE);
    if (nonfinite) atomicCAS(P.status, 0, FR_ERR_NONFINITE);
  }
  uint32_t tot = nfin;
  for (int off = 32; off > 0; off >>= 1) tot += (uint32_t)__shfl_xor((int)tot, off, 64);
  if (lane == 0 && tot) atomicAdd(P.ctr, tot);
  if (lane == 0 && P.debug) {
    atomicAdd(P.ctr + 3, n_wait);
    atomicAdd(P.ctr + 4, n_pace);
    atomicAdd(P.ctr + 5, n_resolve);
  }
}

// Samples rows for the prevailing vertical flow direction: ctr[1] counts
// receivers in the row above (r - 1), ctr[2] in the row below.
template <int RK>
__global__ __launch_bounds__(256) void k_ws_probe(WsParams P, int nsample) {
  const int64_t r = (int64_t)blockIdx.x * P.nrows / nsample;
  uint32_t up = 0, dn = 0;
  for (int64_t c = threadIdx.x; c < P.ncols; c += blockDim.x) {
    const uint32_t code = P.code[r * P.ncols + c];
    if (RK == RK_SINGLE) {
      up += code <= 2u ? 1u : 0u;
      dn += (code >= 5u && code <= 7u) ? 1u : 0u;
    } else {
      up += (uint32_t)__popc(code & 0x07u);
      dn += (uint32_t)__popc(code & 0xE0u);
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    up += (uint32_t)__shfl_xor((int)up, off, 64);
    dn += (uint32_t)__shfl_xor((int)dn, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    if (up) atomicAdd(P.ctr + 1, up);
    if (dn) atomicAdd(P.ctr + 2, dn);
  }
}

__global__ __launch_bounds__(256) void k_fill_u64(uint64_t* p, int64_t n, uint64_t v) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

template <int RK, int DK, int VK, bool CNT>
hipError_t pass_t(const WsParams& P, int dir, int first, hipStream_t s) {
  const unsigned strips = (unsigned)((P.ncols + WS_OWN - 1) / WS_OWN);
  hipLaunchKernelGGL((k_ws_pass<RK, DK, VK, CNT>), dim3(strips), dim3(64), 0, s, P, dir, first);
  return hipGetLastError();
}

}  // namespace

int64_t ws_strips(int64_t ncols) { return (ncols + WS_OWN - 1) / WS_OWN; }

__global__ __launch_bounds__(256) void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

hipError_t launch_ws_progress_reset(const WsParams& P, hipStream_t s) {
  const int64_t n = ws_strips(P.ncols);
  int64_t b = (n + 255) / 256;
  if (b > 1024) b = 1024;
  hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)(b < 1 ? 1 : b)), dim3(256), 0, s, P.progress, n, -1);
  return hipGetLastError();
}

size_t ws_edge_words(int64_t nrows, int64_t ncols) {
  return (size_t)((ncols + WS_OWN - 1) / WS_OWN) * (size_t)nrows * 2 * WS_EW;
}

hipError_t launch_ws_setup(const EngineConfig& cfg, const WsParams& P, hipStream_t s) {
  const int64_t n = (int64_t)ws_edge_words(P.nrows, P.ncols);
  int64_t b = (n + 255) / 256;
  if (b > 8192) b = 8192;
  hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)(b < 1 ? 1 : b)), dim3(256), 0, s, P.edge, n, REC_EMPTY);
  hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, s, reinterpret_cast<uint64_t*>(P.ctr), (int64_t)2, 0ull);
  const int ns = P.nrows < 64 ? (int)P.nrows : 64;
  if (cfg.rk == RK_SINGLE)
    hipLaunchKernelGGL(k_ws_probe<RK_SINGLE>, dim3(ns), dim3(256), 0, s, P, ns);
  else
    hipLaunchKernelGGL(k_ws_probe<RK_MULTI>, dim3(ns), dim3(256), 0, s, P, ns);
  return hipGetLastError();
}

hipError_t launch_ws_pass(const EngineConfig& cfg, const WsParams& P, int dir, int first, hipStream_t s) {
  if (cfg.dir == DIR_FWD) {
    if (cfg.rk == RK_MULTI) {
      if (cfg.vk == VK_F64) return pass_t<RK_MULTI, DIR_FWD, VK_F64, false>(P, dir, first, s);
      return pass_t<RK_MULTI, DIR_FWD, VK_FF, false>(P, dir, first, s);
    }
    if (cfg.counts) {
      if (cfg.vk == VK_FF) return pass_t<RK_SINGLE, DIR_FWD, VK_FF, true>(P, dir, first, s);
      if (cfg.vk == VK_F64) return pass_t<RK_SINGLE, DIR_FWD, VK_F64, true>(P, dir, first, s);
      return pass_t<RK_SINGLE, DIR_FWD, VK_NONE, true>(P, dir, first, s);
    }
    if (cfg.vk == VK_F64) return pass_t<RK_SINGLE, DIR_FWD, VK_F64, false>(P, dir, first, s);
    return pass_t<RK_SINGLE, DIR_FWD, VK_FF, false>(P, dir, first, s);
  }
  if (cfg.rk == RK_MULTI) {
    if (cfg.vk == VK_F64) return pass_t<RK_MULTI, DIR_ADJ, VK_F64, false>(P, dir, first, s);
    return pass_t<RK_MULTI, DIR_ADJ, VK_FF, false>(P, dir, first, s);
  }
  if (cfg.vk == VK_F64) return pass_t<RK_SINGLE, DIR_ADJ, VK_F64, false>(P, dir, first, s);
  return pass_t<RK_SINGLE, DIR_ADJ, VK_FF, false>(P, dir, first, s);
}

}  // namespace fr
